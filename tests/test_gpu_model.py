"""Parity of the GNN forward, the hand-written backward, one full training step
and whole runs against the FP64 oracle, through the C ABI."""

import numpy as np
import pytest
import torch

from helpers import (N_GEMM_CFGS, assert_close_array, assert_close_scalar, assert_update_close,
                     check_relu_decisions, need_gpu, say, to_dev)
from oracle import evaluate as oev
from oracle import exact as oexact
from oracle import gnn as ognn
from oracle import objective as oobj
from oracle import train as otrain
from workloads import disjoint_union, erdos_renyi_graph, get_preset, init_params, random_regular_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def mods():
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    return api, CPRAConfig, CPRASolver


def small_batch():
    return disjoint_union([erdos_renyi_graph(60, 0.08, 1), random_regular_graph(40, 3, 2),
                           erdos_renyi_graph(5, 0.0, 3), erdos_renyi_graph(120, 0.05, 4)])


MODEL_CASES = [
    # name, graph fn, kind, layers, in_dim, hidden, S
    ("gcn2_h32_s10", lambda: random_regular_graph(100, 3, 1), "gcn", 2, 32, 32, 10),
    ("sage2_h64_s100_af_last", lambda: erdos_renyi_graph(300, 1.5 / 299, 2), "sage", 2, 64, 64, 100),
    ("sage2_h256_s100", lambda: random_regular_graph(2000, 5, 3), "sage", 2, 256, 256, 100),
    ("gcn3_lf_first_batch", small_batch, "gcn", 3, 24, 16, 8),
    ("gcn1_single_layer", lambda: random_regular_graph(50, 4, 5), "gcn", 1, 12, 12, 7),
    ("sage3_h128_s64", lambda: random_regular_graph(1000, 20, 6), "sage", 3, 128, 128, 64),
    # five square layers in a row: transpose-first backwards with alternating T buffers, side-stream
    # weight gradients still reading the previous T and dY while the next layer runs
    ("gcn6_h32_deep_square", lambda: random_regular_graph(400, 4, 8), "gcn", 6, 32, 32, 8),
    # a widening first layer (gradient-first backward) below square layers (transpose-first)
    ("sage5_widening_then_square", lambda: erdos_renyi_graph(500, 6 / 499, 9), "sage", 5, 16, 32, 8),
]


@pytest.mark.parametrize("case", MODEL_CASES, ids=[c[0] for c in MODEL_CASES])
def test_model_forward_backward(case):
    api, CPRAConfig, CPRASolver = mods()
    name, gfn, kind, L, in_dim, H, S = case
    g = gfn()
    say(f"model {name} n={g.n} nnz={g.nnz}")
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem="maxcut", layer_kind=kind, n_layers=L, hidden=H, S=S, in_dim=in_dim)
    sol = CPRASolver(dg, cfg)
    p = init_params(kind, g.n, L, H, S, seed=7, in_dim=in_dim)
    if kind == "sage":
        for Ly in p["layers"]:
            Ly["b"] = np.random.default_rng(1).standard_normal(Ly["b"].shape).astype(np.float32) * 0.1
    sol.load_params(p)
    sol.forward()
    torch.cuda.synchronize()
    p64 = ognn.to_f64(p)
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    Zo, cache = ognn.forward(p64, M)
    assert_close_array(sol.Z.cpu().numpy()[: g.n], Zo, what="Z")
    dZ = np.random.default_rng(2).standard_normal((g.n, S)).astype(np.float32)
    grads = torch.empty_like(sol.params)
    api.model_backward(dg, sol.model_cfg, sol.params, to_dev(dZ), grads, sol.ws)
    torch.cuda.synchronize()
    go = ognn.backward(p64, M, cache, dZ.astype(np.float64))
    gg = sol.unpack(grads)
    assert_close_array(gg["emb"], go["emb"], what="d emb")
    for k in range(L):
        for key in go["layers"][k]:
            assert_close_array(gg["layers"][k][key], go["layers"][k][key], what=f"d {key}{k}")
    # recomputation gives bit-identical gradients
    cfg_r = CPRAConfig(problem="maxcut", layer_kind=kind, n_layers=L, hidden=H, S=S, in_dim=in_dim,
                       recompute=True)
    sol_r = CPRASolver(dg, cfg_r)
    sol_r.load_params(p)
    sol_r.forward()
    grads_r = torch.empty_like(sol.params)
    api.model_backward(dg, sol_r.model_cfg, sol_r.params, to_dev(dZ), grads_r, sol_r.ws)
    torch.cuda.synchronize()
    assert torch.equal(sol_r.Z, sol.Z)
    assert torch.equal(grads_r, grads)


def _oracle_step(p64, g, preset_like, gamma):
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    return otrain.loss_and_grads(p64, M, g, preset_like, gamma)


@pytest.mark.parametrize("pname", ["C1", "C3s_small", "sage_mis"])
def test_train_step_teacher_forced(pname):
    api, CPRAConfig, CPRASolver = mods()
    if pname == "C1":
        pr = get_preset("C1")
        g = pr.graph()
        cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=32, S=10, T=2000)
        lam = pr.lam
    elif pname == "C3s_small":
        g = small_batch()
        cfg = CPRAConfig(problem="maxcut", layer_kind="gcn", n_layers=2, hidden=64, S=32, nu=0.1,
                         T=2000)
        lam = None
    else:
        g = random_regular_graph(2000, 5, 9)
        cfg = CPRAConfig(problem="mis", layer_kind="sage", n_layers=2, hidden=256, S=100, T=5000)
        lam = np.logspace(-1, 1, 100).astype(np.float32)
    say(f"train_step {pname} n={g.n}")
    dg = api.DeviceGraph.from_csr(g)
    sol = CPRASolver(dg, cfg, lam)
    p = init_params(cfg.layer_kind, g.n, cfg.n_layers, cfg.hidden, cfg.S, seed=3)
    sol.load_params(p)
    ocfg = otrain.StepConfig(problem=cfg.problem, lam=None if lam is None else lam.astype(np.float64),
                             alpha=2, nu=cfg.nu, lr=cfg.lr)
    from paper_2402_02190_amd.solver import gamma_schedule
    for round_ in range(3):
        t = sol.t
        p_before = sol.unpack(sol.params)
        m_before = sol.unpack(sol.m)
        v_before = sol.unpack(sol.v)
        sol.step()
        torch.cuda.synchronize()
        gamma = gamma_schedule(t, cfg.T, cfg.gamma_start, cfg.gamma_end)
        p64 = ognn.to_f64(p_before)
        Zo, terms_o, dZo, go = _oracle_step(p64, g, ocfg, gamma)
        assert_close_array(sol.Z.cpu().numpy()[: g.n], Zo, what=f"[{t}] Z")
        assert_close_array(sol.dZ.cpu().numpy()[: g.n], dZo, what=f"[{t}] dZ")
        T_gpu = sol.terms.cpu().numpy()
        for gi, to in enumerate(terms_o):
            for s in range(cfg.S):
                assert_close_scalar(T_gpu[gi, s], to["head"][s], abs(to["head"][s]) + 1.0 + 1e-9,
                                    what="l_s")
            assert_close_scalar(T_gpu[gi, cfg.S], to["entropy"], to["entropy"], what="S(P)")
            assert_close_scalar(T_gpu[gi, cfg.S + 1], to["psi"], abs(to["psi"]), what="Psi")
        gg = sol.unpack(sol.grads)
        assert_close_array(gg["emb"], go["emb"], what=f"[{t}] d emb")
        for k in range(cfg.n_layers):
            for key in go["layers"][k]:
                assert_close_array(gg["layers"][k][key], go["layers"][k][key], what=f"[{t}] d{key}{k}")
        # Adam from the GPU's own gradient, in FP64, over every parameter array
        pn = ognn.to_f64(p_before)
        mo, vo = ognn.to_f64(m_before), ognn.to_f64(v_before)
        g64 = ognn.to_f64(gg)
        after = sol.unpack(sol.params)
        otrain.adam_update(pn["emb"], g64["emb"], mo["emb"], vo["emb"], t + 1, cfg.lr)
        assert_update_close(after["emb"], p_before["emb"], pn["emb"], what=f"[{t}] emb update")
        for k in range(cfg.n_layers):
            for key in pn["layers"][k]:
                otrain.adam_update(pn["layers"][k][key], g64["layers"][k][key], mo["layers"][k][key],
                                   vo["layers"][k][key], t + 1, cfg.lr)
                assert_update_close(after["layers"][k][key], p_before["layers"][k][key],
                                    pn["layers"][k][key], what=f"[{t}] {key}{k} update")
        sol.run(5, use_graph=False)


def test_graph_replay_is_bit_identical_to_eager():
    api, CPRAConfig, CPRASolver = mods()
    pr = get_preset("C1")
    g = pr.graph()
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=32, S=10, T=2000)
    p = init_params("gcn", g.n, 2, 32, 10, seed=4)
    a = CPRASolver(dg, cfg, pr.lam)
    b = CPRASolver(dg, cfg, pr.lam)
    a.load_params(p)
    b.load_params(p)
    a.run(25, use_graph=False)
    b.run(10, use_graph=True)
    b.run(15, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(a.params, b.params)
    assert torch.equal(a.terms, b.terms)
    assert int(b.step_counter.item()) == 25


def test_autograd_function_matches_backward():
    api, CPRAConfig, CPRASolver = mods()
    from paper_2402_02190_amd.autograd import CPRALoss
    g = random_regular_graph(200, 3, 11)
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem="mis", layer_kind="sage", n_layers=2, hidden=16, S=6)
    lam = np.linspace(0.5, 3, 6).astype(np.float32)
    sol = CPRASolver(dg, cfg, lam)
    p = init_params("sage", g.n, 2, 16, 6, seed=2)
    sol.load_params(p)
    params = sol.params.clone().requires_grad_(True)
    R = CPRALoss.apply(params, sol, -0.5)
    R.backward()
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ocfg = otrain.StepConfig(problem="mis", lam=lam.astype(np.float64))
    Zo, terms, dZo, go = otrain.loss_and_grads(ognn.to_f64(p), M, g, ocfg, -0.5)
    assert abs(float(R.detach()) - terms[0]["total"]) <= 1e-5 * (np.abs(terms[0]["head"]).sum() + 0.5 * terms[0]["entropy"])
    gg = sol.unpack(params.grad)
    assert_close_array(gg["emb"], go["emb"], what="autograd d emb")
    assert_close_array(gg["layers"][1]["Wn"], go["layers"][1]["Wn"], what="autograd dWn1")


@pytest.mark.parametrize("kind", ["node_weights", "per_head_node_weights", "instances"])
def test_autograd_function_uses_the_solvers_objective(kind):
    """CPRALoss on a weighted-MIS solver (node weights per node or per head) and on a
    solver with one instance per head (per-head edge weights, MaxCut): R, dZ and the
    parameter gradients follow that solver's objective, as the training step does."""
    api, CPRAConfig, CPRASolver = mods()
    from paper_2402_02190_amd.autograd import CPRALoss
    from workloads import instance_edge_weights
    g = random_regular_graph(240, 4, 12)
    dg = api.DeviceGraph.from_csr(g)
    S = 8
    rng = np.random.default_rng(3)
    nw = ew = None
    if kind == "instances":
        problem, lam = "maxcut", None
        ew = instance_edge_weights(g, S, 5, "uniform", 0.2)
    else:
        problem, lam = "mis", np.linspace(0.5, 3, S).astype(np.float32)
        nw = rng.uniform(0, 1, (g.n, S) if kind == "per_head_node_weights" else g.n).astype(np.float32)
    cfg = CPRAConfig(problem=problem, layer_kind="sage", n_layers=2, hidden=16, S=S, nu=0.1)
    sol = CPRASolver(dg, cfg, lam, node_weight=nw, edge_weight=ew)
    p = init_params("sage", g.n, 2, 16, S, seed=4)
    sol.load_params(p)
    gamma = -0.7
    params = sol.params.clone().requires_grad_(True)
    R = CPRALoss.apply(params, sol, gamma)
    assert R.is_cuda and R.dtype == torch.float64
    R.backward()
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ocfg = otrain.StepConfig(problem=problem, lam=None if lam is None else lam.astype(np.float64),
                             nu=0.1, node_weight=nw, edge_weight=ew)
    Zo, terms, dZo, go = otrain.loss_and_grads(ognn.to_f64(p), M, g, ocfg, gamma)
    t = terms[0]
    scale = np.abs(t["head"]).sum() + abs(gamma) * t["entropy"] + 0.1 * abs(t["psi"]) + g.n * S
    assert_close_scalar(float(R.detach()), t["total"], scale, what=f"{kind} R")
    assert_close_array(sol.dZ.cpu().numpy()[: g.n], dZo, what=f"{kind} dZ")
    gg = sol.unpack(params.grad)
    assert_close_array(gg["emb"], go["emb"], what=f"{kind} d emb")
    for k in range(2):
        for key in go["layers"][k]:
            assert_close_array(gg["layers"][k][key], go["layers"][k][key], what=f"{kind} d{key}{k}")
    # the plain objective differs: the weights really entered the loss
    plain = otrain.loss_and_grads(ognn.to_f64(p), M, g, otrain.StepConfig(
        problem=problem, lam=ocfg.lam, nu=0.1), gamma)[1][0]["total"]
    assert abs(plain - t["total"]) > 1e-3 * scale
    sol.close()


ES_CASES = [("absolute", 1e-5, 20, False), ("relative", 1e-3, 10, True)]


@pytest.mark.parametrize("name,tol,patience,relative", ES_CASES, ids=[c[0] for c in ES_CASES])
def test_early_stopping_on_device_matches_the_rule(name, tol, patience, relative):
    """The device's stopping rule against the oracle's rule recomputed on the GPU's own
    loss history (the head losses and annealing terms the steps wrote): same stopping
    step; once stopped, further steps change neither the parameters, the Adam moments
    nor the step counter; a replayed run that polls the flag every 25 steps stops at
    the same step with the same parameters, bit for bit."""
    api, CPRAConfig, CPRASolver = mods()
    from paper_2402_02190_amd.solver import gamma_schedule
    g = random_regular_graph(200, 3, 21)
    dg = api.DeviceGraph.from_csr(g)
    S = 8
    lam = np.linspace(0.5, 3, S).astype(np.float32)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=16, S=S, T=150,
                     gamma_start=-2.0, gamma_end=0.5, lr=1e-2)
    p = init_params("gcn", g.n, 2, 16, S, seed=9)
    a = CPRASolver(dg, cfg, lam)
    a.load_params(p)
    a.enable_early_stopping(tol, patience, relative)
    head, phi = [], []
    max_steps = 4000
    for t in range(max_steps):
        a.step()
        T = a.terms_host()
        head.append(float(T[:, :S].sum()))
        phi.append(float(np.float64(gamma_schedule(t, cfg.T, cfg.gamma_start, cfg.gamma_end))
                         * T[:, S].sum()))
        if a.early_stop_state()["stopped"]:
            break
    expected = otrain.early_stop_step(head, phi, tol, patience, relative)
    st = a.early_stop_state()
    say(f"  {name}: rule fires at step {expected}; device {st}")
    assert expected is not None and st["stopped"] == 1
    assert st["stop_step"] == expected == len(head) - 1
    assert int(a.step_counter.item()) == expected
    frozen = [x.clone() for x in (a.params, a.m, a.v)]
    for _ in range(3):
        a.step()
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(frozen, (a.params, a.m, a.v)))
    assert int(a.step_counter.item()) == expected
    b = CPRASolver(dg, cfg, lam)
    b.load_params(p)
    b.enable_early_stopping(tol, patience, relative)
    n, stop = b.run_with_early_stopping(max_steps, check_every=25)
    assert stop == expected and n >= expected + 1 and n - (expected + 1) < 25
    assert torch.equal(b.params, a.params)
    a.close()
    b.close()


def test_early_stopping_rejects_a_step_without_terms_or_counter():
    api, CPRAConfig, CPRASolver = mods()
    g = random_regular_graph(50, 3, 2)
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=8, S=4)
    sol = CPRASolver(dg, cfg, np.ones(4, np.float32))
    sol.enable_early_stopping(1e-5, 10)
    with pytest.raises(api.CpraError):
        api.train_step(sol.graph, sol.step_cfg, sol.params, sol.grads, sol.m, sol.v, sol.Z, sol.dZ,
                       None, sol.ws, 1, sol.step_counter)
    with pytest.raises(api.CpraError):
        api.train_step(sol.graph, sol.step_cfg, sol.params, sol.grads, sol.m, sol.v, sol.Z, sol.dZ,
                       sol.terms, sol.ws, 1, None)
    sol.step_cfg.early_stop.patience = 0
    with pytest.raises(api.CpraError):
        sol.step()
    sol.close()


def test_run_until_binary_stops_at_the_first_check_below_eps():
    """run_until_binary replays in chunks and stops at the first chunk boundary where
    the annealing term per entry S(P) / (N S) is below eps: the same boundary as a
    run that reads the terms at every boundary itself."""
    api, CPRAConfig, CPRASolver = mods()
    g = random_regular_graph(300, 3, 5)
    dg = api.DeviceGraph.from_csr(g)
    S = 6
    lam = np.linspace(0.5, 3, S).astype(np.float32)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=16, S=S, T=200,
                     gamma_start=-2.0, gamma_end=1.0, lr=1e-2)
    p = init_params("gcn", g.n, 2, 16, S, seed=13)
    eps, K, steps = 1e-3, 50, 3000
    a = CPRASolver(dg, cfg, lam)
    a.load_params(p)
    n = a.run_until_binary(steps, eps=eps, check_every=K)
    b = CPRASolver(dg, cfg, lam)
    b.load_params(p)
    done, expect = 0, steps
    while done < steps:
        b.replay(K)
        done += K
        if float(b.terms_host()[:, S].sum()) / (g.n * S) < eps:
            expect = done
            break
    say(f"  run_until_binary stopped after {n} steps (reference {expect})")
    assert n == expect < steps
    assert torch.equal(a.params, b.params)
    a.close()
    b.close()


@pytest.mark.parametrize("preset", ["C3s", "C2"])
def test_persistent_launches_are_bit_identical(preset, monkeypatch):
    """The persistent aggregation and loss launches (CPRA_PERSISTENT=1: at most the
    resident blocks, taking row blocks / graph-segmented items from XCD-local work
    queues) give the same bits as one block per unit: three replayed training steps
    on the 32-graph ER batch (ragged graphs, per-graph items) and on the 10,000-node
    graph, and the standalone loss call."""
    api, CPRAConfig, CPRASolver = mods()
    pr = get_preset(preset)
    g = pr.graph()
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem=pr.problem, layer_kind=pr.layer_kind, n_layers=pr.n_layers,
                     hidden=pr.hidden, S=pr.S, alpha=pr.alpha, nu=pr.nu, T=pr.T)
    p = init_params(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S, seed=3)
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("CPRA_PERSISTENT", mode)
        sol = CPRASolver(dg, cfg, pr.lam)
        sol.load_params(p)
        sol.run(3, use_graph=True)
        dZ2 = torch.empty_like(sol.Z)
        t2 = torch.empty_like(sol.terms)
        api.loss_fwd_bwd(sol.graph, sol.loss_cfg, sol.Z, dZ2, t2, sol.loss_workspace())
        torch.cuda.synchronize()
        out[mode] = [x.clone() for x in (sol.params, sol.Z, sol.dZ, sol.terms, dZ2, t2)]
        sol.close()
    for name, x, y in zip(("params", "Z", "dZ", "terms", "loss dZ", "loss terms"), out["0"], out["1"]):
        assert torch.equal(x, y), name


@pytest.mark.parametrize("preset", ["C2", "C3s", "C4"])
def test_fork_orders_and_one_stream_are_bit_identical(preset, monkeypatch):
    """The backward's two capture orders at each fork (the input gradient captured
    ahead of the side-stream weight gradients, the default; the side work first,
    CPRA_SIDE_FIRST=1) and the single-stream schedule (CPRA_OVERLAP=0) run the
    same kernels on the same data, so three replayed training steps give the same
    bits: GraphSAGE with bias gradients (C2), a ragged ER batch (C3s), and three
    GCN layers whose transform buffers are reused across the backward (C4)."""
    api, CPRAConfig, CPRASolver = mods()
    pr = get_preset(preset)
    g = pr.graph()
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem=pr.problem, layer_kind=pr.layer_kind, n_layers=pr.n_layers,
                     hidden=pr.hidden, S=pr.S, alpha=pr.alpha, nu=pr.nu, T=pr.T)
    p = init_params(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S, seed=5)
    out = {}
    for name, env in (("main first", {}), ("side first", {"CPRA_SIDE_FIRST": "1"}),
                      ("one stream", {"CPRA_OVERLAP": "0"})):
        for k in ("CPRA_SIDE_FIRST", "CPRA_OVERLAP"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        say(f"  {preset}: {name}")
        sol = CPRASolver(dg, cfg, pr.lam)
        sol.load_params(p)
        sol.run(3, use_graph=True)
        torch.cuda.synchronize()
        out[name] = [x.clone() for x in (sol.params, sol.Z, sol.dZ, sol.terms)]
        sol.close()
    for other in ("side first", "one stream"):
        for what, x, y in zip(("params", "Z", "dZ", "terms"), out["main first"], out[other]):
            assert torch.equal(x, y), f"{other}: {what}"


def test_multi_step_graph_replays_equal_one_step_replays():
    """Ten steps replayed through a graph of four recorded steps (two launches, then
    two launches of the one-step graph) give the same bits as ten one-step
    replays: the steps of a graph take Adam's index and the annealing weight from
    the device step counter like separate launches do."""
    api, CPRAConfig, CPRASolver = mods()
    pr = get_preset("C3s")
    g = pr.graph()
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem=pr.problem, layer_kind=pr.layer_kind, n_layers=pr.n_layers,
                     hidden=pr.hidden, S=pr.S, alpha=pr.alpha, nu=pr.nu, T=pr.T)
    p = init_params(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S, seed=9)
    out = []
    for k in (1, 4):
        sol = CPRASolver(dg, cfg, pr.lam)
        sol.load_params(p)
        sol.capture(steps_per_graph=k)
        assert [n for _, n in sol.launch_plan(10)] == ([1] * 10 if k == 1 else [4, 4, 1, 1])
        sol.replay(10)
        torch.cuda.synchronize()
        out.append([x.clone() for x in (sol.params, sol.m, sol.v, sol.Z, sol.terms, sol.step_counter)])
        sol.close()
    for what, x, y in zip(("params", "m", "v", "Z", "terms", "step counter"), *out):
        assert torch.equal(x, y), what
    assert int(out[1][5].item()) == 10


def test_c1_end_to_end_against_oracle_and_exact_optimum():
    api, CPRAConfig, CPRASolver = mods()
    pr = get_preset("C1")
    g = pr.graph()
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=32, S=10, T=pr.T,
                     gamma_start=pr.gamma_start, gamma_end=pr.gamma_end, lr=pr.lr)
    p = init_params("gcn", g.n, 2, 32, 10, seed=11)
    sol = CPRASolver(dg, cfg, pr.lam)
    sol.load_params(p)
    sol.run(pr.T, use_graph=True)
    sol.forward()
    ev = sol.evaluate()
    Zg = sol.Z.cpu().numpy()[: g.n].astype(np.float64)
    # integer evaluation of the GPU's own output is bit-exact against the oracle
    Xo = oev.round_solutions(Zg)
    evo = oev.evaluate(Xo, g, "mis")[0]
    assert np.array_equal(ev["X"], Xo)
    assert np.array_equal(ev["value"][0], evo["size"])
    assert np.array_equal(ev["violations"][0], evo["violations"])
    # free-running FP64 oracle from the same initial bytes
    ocfg = otrain.StepConfig(problem="mis", lam=pr.lam.astype(np.float64), lr=pr.lr)
    ores = otrain.solve(p, g, ocfg, pr.T, pr.gamma_start, pr.gamma_end)
    Zo = ores["Z"]
    margin = np.abs(Zo) > 1e-4 * np.maximum(1.0, np.abs(Zo))
    agree = np.mean((Zg > 0) == (Zo > 0))
    per_head = [(np.array_equal((Zg[:, s] > 0), (Zo[:, s] > 0))) for s in range(10)]
    alpha_g = oexact.mis_size_milp(g)
    best_gpu = oev.best_feasible_mis(evo)
    best_orc = oev.best_feasible_mis(ores["eval"][0])
    say(f"C1: agreement {agree:.4f}, identical heads {sum(per_head)}/10, inside margin "
        f"{int((~margin).sum())}, best GPU {best_gpu} oracle {best_orc} alpha {alpha_g}, "
        f"min|Z| {np.abs(Zg).min():.3e}")
    assert best_gpu <= alpha_g and best_gpu >= 0.9 * alpha_g
    assert np.all(ev["violations"][0][pr.lam > 1.0] == 0)
    assert agree >= 0.9


@pytest.mark.parametrize("cfg", range(N_GEMM_CFGS))
def test_sage_bias_gradient_under_every_weight_gradient_plan(cfg):
    """The bias gradient is summed inside the weight-gradient GEMM by the first
    column tile: check db (and dWs) of a 2-layer SAGE model with every tile
    configuration forced on those GEMMs, with and without split-K (150 splits
    leave some splits without a K tile, whose partial sums must be zeros).  The
    interleaved configurations run their two-deep twins for it, the LDS-ring
    ones sum the bias from their stages.  The same configuration is forced on
    the step's other products too (the two-piece [X | MX] forward and the input
    gradients), and every gradient is checked."""
    api, CPRAConfig, CPRASolver = mods()
    g = random_regular_graph(700, 5, 9)
    dg = api.DeviceGraph.from_csr(g)
    cfgc = CPRAConfig(problem="mis", layer_kind="sage", n_layers=2, hidden=64, S=32)
    lam = np.logspace(-1, 1, 32).astype(np.float32)
    p = init_params("sage", g.n, 2, 64, 32, seed=4)
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ocfg = otrain.StepConfig(problem="mis", lam=lam.astype(np.float64))
    _, _, _, go = otrain.loss_and_grads(ognn.to_f64(p), M, g, ocfg, cfgc.gamma_start)
    # find the weight-gradient problem keys from one tuned step
    sol = CPRASolver(dg, cfgc, lam)
    sol.load_params(p)
    table = sol.autotune()
    keys = [e[0] for e in table]
    assert any(k.startswith("TN") for k in keys) and any(not k.startswith("TN") for k in keys)
    try:
        for splits in (1, 4, 150):
            api.autotune_reset()
            for k in keys:
                api.autotune_set(k, cfg, splits if k.startswith("TN") else 1)
            sol.load_params(p)
            sol.step()
            torch.cuda.synchronize()
            gg = sol.unpack(sol.grads)
            for k in range(2):
                for name in ("b", "Ws", "Wn"):
                    assert_close_array(gg["layers"][k][name], go["layers"][k][name],
                                       what=f"cfg {cfg} splits {splits} d{name}{k}")
            assert_close_array(gg["emb"], go["emb"], what=f"cfg {cfg} splits {splits} dE")
    finally:
        api.autotune_reset()
        sol.close()


FROZEN_CASES = [
    # name, kind, layers, hidden, S, train_from  (AF or LF output layer)
    ("sage2_af_last_from1", "sage", 2, 32, 64, 1),
    ("gcn3_lf_last_from2", "gcn", 3, 32, 10, 2),
    ("gcn3_from1", "gcn", 3, 32, 16, 1),
]


@pytest.mark.parametrize("case", FROZEN_CASES, ids=[c[0] for c in FROZEN_CASES])
def test_frozen_encoder_step(case):
    """Frozen encoder: trained layers get the full gradient (oracle), frozen
    gradients and parameters are left exactly as they were, and Adam moves only
    the trained tail; reusing the saved prefix activations gives identical bits."""
    api, CPRAConfig, CPRASolver = mods()
    name, kind, L, H, S, tf = case
    g = random_regular_graph(400, 4, 11)
    dg = api.DeviceGraph.from_csr(g)
    lam = np.linspace(0.5, 4, S).astype(np.float32)
    cfg = CPRAConfig(problem="mis", layer_kind=kind, n_layers=L, hidden=H, S=S, train_from_layer=tf)
    p = init_params(kind, g.n, L, H, S, seed=21)
    sols = []
    for reuse in (False, True):
        sol = CPRASolver(dg, cfg, lam)
        sol.load_params(p)
        sentinel = 12345.0
        sol.grads.fill_(sentinel)
        sol.step()
        torch.cuda.synchronize()
        sols.append(sol)
        if not reuse:
            M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
            ocfg = otrain.StepConfig(problem="mis", lam=lam.astype(np.float64))
            _, _, _, go = otrain.loss_and_grads(ognn.to_f64(p), M, g, ocfg, cfg.gamma_start)
            gg = sol.unpack(sol.grads)
            after = sol.unpack(sol.params)
            assert np.all(gg["emb"] == sentinel) and np.array_equal(after["emb"], p["emb"])
            for k in range(L):
                for key in p["layers"][k]:
                    if k < tf:
                        assert np.all(gg["layers"][k][key] == sentinel)
                        assert np.array_equal(after["layers"][k][key], p["layers"][k][key])
                    else:
                        assert_close_array(gg["layers"][k][key], go["layers"][k][key],
                                           what=f"{name} d{key}{k}")
                        assert not np.array_equal(after["layers"][k][key], p["layers"][k][key])
        else:
            sol.set_reuse_frozen_prefix(True)
    # three more steps each: the reused-prefix run replays them from a captured graph
    sols[0].run(3, use_graph=False)
    sols[1].run(3, use_graph=True)
    torch.cuda.synchronize()
    for attr in ("Z", "grads", "params", "m", "v"):
        assert torch.equal(getattr(sols[0], attr), getattr(sols[1], attr)), attr
    for s in sols:
        s.close()


@pytest.mark.parametrize("t_at", [10, 1000, 1999])
def test_train_step_teacher_forced_late_steps(t_at):
    """Step parity later in the schedule (t = 10, T/2, T-1 of T = 2000): the GPU runs
    t steps from the captured graph, then one more eager step whose loss terms and
    gradients the oracle recomputes in FP64 from the GPU's parameters at t (ReLU
    decisions taken from the GPU's forward).  Late steps have gamma > 0 and
    saturated P, where 1 - P must not be formed by cancellation."""
    api, CPRAConfig, CPRASolver = mods()
    from paper_2402_02190_amd.solver import gamma_schedule
    pr = get_preset("C1")
    g = pr.graph()
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=32, S=10, T=pr.T,
                     gamma_start=pr.gamma_start, gamma_end=pr.gamma_end, lr=pr.lr)
    sol = CPRASolver(dg, cfg, pr.lam)
    sol.load_params(init_params("gcn", g.n, 2, 32, 10, seed=13))
    sol.run(t_at, use_graph=True)
    torch.cuda.synchronize()
    t = int(sol.step_counter.item())
    assert t == t_at
    p_before = sol.unpack(sol.params)
    sol.step()
    torch.cuda.synchronize()
    gamma = gamma_schedule(t, cfg.T, cfg.gamma_start, cfg.gamma_end)
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ocfg = otrain.StepConfig(problem="mis", lam=pr.lam.astype(np.float64), lr=pr.lr)
    active = sol.relu_active()
    Zo, terms_o, dZo, go, cache = otrain.loss_and_grads(ognn.to_f64(p_before), M, g, ocfg, gamma,
                                                        relu_active=active, return_cache=True)
    check_relu_decisions(active, [c["Y"] for c in cache[: len(active)]], f"t={t}")
    say(f"t={t}: gamma={gamma:.4f}, max |Z|={np.abs(Zo).max():.1f}")
    assert_close_array(sol.Z.cpu().numpy()[: g.n], Zo, what=f"[{t}] Z")
    assert_close_array(sol.dZ.cpu().numpy()[: g.n], dZo, what=f"[{t}] dZ")
    gg = sol.unpack(sol.grads)
    assert_close_array(gg["emb"], go["emb"], what=f"[{t}] d emb")
    for k in range(2):
        for key in go["layers"][k]:
            assert_close_array(gg["layers"][k][key], go["layers"][k][key], what=f"[{t}] d{key}{k}")
    T_gpu = sol.terms.cpu().numpy()
    to = terms_o[0]
    for s in range(cfg.S):
        assert_close_scalar(T_gpu[0, s], to["head"][s], abs(to["head"][s]) + 1.0, what="l_s")
    assert_close_scalar(T_gpu[0, cfg.S], to["entropy"], to["entropy"] + 1e-9, what="S(P)")
    assert int(sol.step_counter.item()) == t + 1
    sol.close()


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
def test_solve_trains_rounds_and_scores_every_head(problem):
    """solve(): T replayed steps from seeded parameters, then the trained logits rounded
    and scored -- the same bits as driving CPRASolver by hand, scores equal to the
    oracle's exact evaluation of the returned X, and the best feasible head chosen."""
    api, CPRAConfig, CPRASolver = mods()
    from paper_2402_02190_amd.solver import solve
    g = random_regular_graph(400, 3, 21)
    dg = api.DeviceGraph.from_csr(g)
    S = 8
    cfg = CPRAConfig(problem=problem, layer_kind="gcn", n_layers=2, hidden=16, S=S, T=300, lr=1e-2)
    lam = np.linspace(0.5, 3, S).astype(np.float32) if problem == "mis" else None
    say(f"solve {problem} N={g.n} S={S} T={cfg.T}")
    r = solve(dg, cfg, lam=lam, seed=4)
    ref = CPRASolver(dg, cfg, lam)
    ref.load_params(init_params("gcn", g.n, 2, 16, S, seed=4))
    ref.run(cfg.T)
    ref.forward()
    ev = ref.evaluate()
    ref.close()
    assert r.steps == cfg.T and r.stop_step is None
    assert np.array_equal(r.X, ev["X"]) and np.array_equal(r.value, ev["value"])
    e = oev.evaluate_one(r.X, g, problem)
    if problem == "mis":
        assert np.array_equal(r.value[0], e["size"])
        assert np.array_equal(r.violations[0], e["violations"])
    else:
        assert np.array_equal(r.value[0], e["cut_edges"])
        assert not r.violations.any()
    feas = r.violations[0] == 0
    assert feas.any()
    assert r.best_head[0] >= 0 and feas[r.best_head[0]]
    assert r.best_value[0] == r.value[0][feas].max()
    say(f"  best head {r.best_head[0]}: {r.best_value[0]:.0f} in {r.seconds:.3f} s")


def test_solve_with_early_stopping_reports_the_firing_step():
    """solve(early_stopping=...): a tolerance that every step meets fires the rule
    after `patience` stalled steps; the result names that step."""
    api, CPRAConfig, CPRASolver = mods()
    from paper_2402_02190_amd.solver import solve
    g = random_regular_graph(200, 3, 22)
    S = 4
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=8, S=S, T=400)
    r = solve(g, cfg, seed=1, early_stopping={"tol": 1e30, "patience": 7})
    say(f"  stopped at step {r.stop_step} after {r.steps} replayed steps")
    assert r.stop_step == 7
    assert r.steps <= cfg.T
