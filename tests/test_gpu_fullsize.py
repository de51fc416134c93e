"""Parity at the full workload sizes, in the launch configuration bench.py times
(the committed MI355X GEMM plans bench.py loads, side-stream overlap, a
captured and replayed step, the same presets; also with one instance per
head, as ``bench.py --instances`` runs them), and the hand-written backward
against finite differences on a 1,000-node subgraph of the 100,000-node
workload.

The oracle is fast enough at these sizes (sparse aggregation + BLAS in FP64)
to be compared on every element, so no sampling is needed.
"""

import numpy as np
import pytest
import torch

from helpers import assert_close_array, assert_close_scalar, check_relu_decisions, need_gpu, say
from oracle import gnn as ognn
from oracle import objective as oobj
from oracle import train as otrain
from workloads import bfs_ball, get_preset, induced_subgraph, init_params

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _solver_for(pr, g, seed, edge_weight=None):
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem=pr.problem, layer_kind=pr.layer_kind, n_layers=pr.n_layers,
                     hidden=pr.hidden, S=pr.S, alpha=pr.alpha, nu=pr.nu, gamma_start=pr.gamma_start,
                     gamma_end=pr.gamma_end, T=pr.T, lr=pr.lr, recompute=pr.recompute)
    sol = CPRASolver(dg, cfg, pr.lam, edge_weight=edge_weight)
    params = init_params(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S, seed=seed)
    sol.load_params(params)
    return sol


def committed_plans(name):
    """Load the committed MI355X GEMM tuning table of a workload, as bench.py does;
    returns the plans loaded (key -> (configuration, split count))."""
    import json
    import os
    from paper_2402_02190_amd import api
    path = os.path.join(os.path.dirname(api.__file__), "tuning", f"{name.lower()}_mi355x.json")
    with open(path) as f:
        table = json.load(f)
    api.autotune_reset()
    for e in table:
        api.autotune_set(e["key"], e["cfg"], e["splits"])
    return {e["key"]: (e["cfg"], e["splits"]) for e in table}


FULL_CASES = [("C2", None, 0.0), ("C4", None, 0.0), ("C3s", None, 0.0), ("C3", None, 0.0),
              ("C2", "integer", 0.0), ("C4", "signed", 0.2)]  # the last two: one instance per head


@pytest.mark.parametrize("preset,instances,drop", FULL_CASES,
                         ids=[f"{p}{'_' + i if i else ''}" for p, i, _ in FULL_CASES])
def test_full_size_step_teacher_forced(preset, instances, drop):
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import gamma_schedule
    from workloads import instance_edge_weights
    pr = get_preset(preset)
    g = pr.graph()
    say(f"full-size {preset}: n={g.n} edges={g.n_edges} graphs={g.n_graphs} instances={instances}")
    plans = committed_plans(preset)
    say("  plans: " + ", ".join(f"{k} -> cfg {c} x{sp}" for k, (c, sp) in plans.items()))
    try:
        _teacher_forced(pr, g, preset, instances, drop, instance_edge_weights, gamma_schedule)
    finally:
        api.autotune_reset()


def _teacher_forced(pr, g, preset, instances, drop, instance_edge_weights, gamma_schedule):
    W = instance_edge_weights(g, pr.S, 2025, instances, drop) if instances else None
    sol = _solver_for(pr, g, seed=7, edge_weight=W)
    sol.step()  # step 0, eager, with the committed plans
    torch.cuda.synchronize()
    t = sol.t
    p_before = sol.unpack(sol.params)
    sol.capture()
    sol.replay(1)  # step 1 from the captured graph, as bench.py times it
    torch.cuda.synchronize()
    gamma = gamma_schedule(t, pr.T, pr.gamma_start, pr.gamma_end)
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ocfg = otrain.StepConfig(problem=pr.problem, lam=None if pr.lam is None else pr.lam.astype(np.float64),
                             alpha=pr.alpha, nu=pr.nu, lr=pr.lr, edge_weight=W)
    # The ReLU derivative is a discrete decision: take it where the FP32 forward took it,
    # after checking that every disagreement with the FP64 forward sits at Y ~ 0.
    active = sol.relu_active()
    Zo, terms_o, dZo, go, cache = otrain.loss_and_grads(ognn.to_f64(p_before), M, g, ocfg, gamma,
                                                        relu_active=active, return_cache=True)
    check_relu_decisions(active, [c["Y"] for c in cache[: len(active)]], preset)
    assert_close_array(sol.Z.cpu().numpy()[: g.n], Zo, what="Z")
    assert_close_array(sol.dZ.cpu().numpy()[: g.n], dZo, what="dZ")
    gg = sol.unpack(sol.grads)
    assert_close_array(gg["emb"], go["emb"], what="d emb")
    for k in range(pr.n_layers):
        for key in go["layers"][k]:
            assert_close_array(gg["layers"][k][key], go["layers"][k][key], what=f"d{key}{k}")
    T = sol.terms_host()
    worst = 0.0
    for gi, to in enumerate(terms_o):
        for s in range(pr.S):
            worst = max(worst, assert_close_scalar(T[gi, s], to["head"][s], abs(to["head"][s]) + 1.0,
                                                   what="l_s"))
        worst = max(worst, assert_close_scalar(T[gi, pr.S], to["entropy"], to["entropy"], what="S(P)"))
        worst = max(worst, assert_close_scalar(T[gi, pr.S + 1], to["psi"], abs(to["psi"]), what="Psi"))
    say(f"  worst loss-term error {worst:.3e} over {len(terms_o)} graph(s)")
    sol.close()


def test_full_size_per_graph_c3_sampled_graphs():
    """C3 with one network per graph (256 graphs, 710,241 nodes) in bench.py's launch
    configuration (the committed per-graph GEMM plans, a captured and replayed step):
    the graphs are independent problems, so sampled graphs -- the smallest, the largest
    and three more -- are each checked against the oracle run on that graph alone."""
    import json
    import os
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver, gamma_schedule
    from workloads import init_params_per_graph
    pr = get_preset("C3")
    g = pr.graph()
    G = g.n_graphs
    say(f"full-size C3 per graph: n={g.n} graphs={G}")
    table = os.path.join(os.path.dirname(api.__file__), "tuning", "c3_pergraph_mi355x.json")
    with open(table) as f:
        for e in json.load(f):
            api.autotune_set(e["key"], e["cfg"], e["splits"])
    try:
        dg = api.DeviceGraph.from_csr(g)
        cfg = CPRAConfig(problem=pr.problem, layer_kind=pr.layer_kind, n_layers=pr.n_layers,
                         hidden=pr.hidden, S=pr.S, alpha=pr.alpha, nu=pr.nu,
                         gamma_start=pr.gamma_start, gamma_end=pr.gamma_end, T=pr.T, lr=pr.lr,
                         per_graph_weights=True)
        sol = CPRASolver(dg, cfg, pr.lam)
        sol.load_params(init_params_per_graph(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S, G,
                                              seed=7))
        sol.step()
        torch.cuda.synchronize()
        t = sol.t
        p_before = ognn.to_f64(sol.unpack(sol.params))
        sol.capture()
        sol.replay(1)
        torch.cuda.synchronize()
        gamma = gamma_schedule(t, pr.T, pr.gamma_start, pr.gamma_end)
        gp = np.asarray(g.graph_ptr, dtype=np.int64)
        sizes = np.diff(gp)
        picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0, G // 2, G - 1})
        Z = sol.Z.cpu().numpy()
        dZ = sol.dZ.cpu().numpy()
        T = sol.terms_host()
        gg = sol.unpack(sol.grads)
        active = sol.relu_active()
        ocfg = otrain.StepConfig(problem=pr.problem, lam=None, alpha=pr.alpha, nu=pr.nu, lr=pr.lr)
        for b in picks:
            lo, hi = int(gp[b]), int(gp[b + 1])
            sub = oobj._slice_graph(g, lo, hi)
            M = ognn.mean_aggregation_matrix(sub.row_ptr, sub.col_idx)
            act_b = [a[lo:hi] for a in active]
            Zo, terms_o, dZo, go, cache = otrain.loss_and_grads(
                otrain.graph_params(p_before, b, lo, hi), M, sub, ocfg, gamma, relu_active=act_b,
                return_cache=True)
            say(f"  graph {b}: {hi - lo} nodes")
            check_relu_decisions(act_b, [c["Y"] for c in cache[: len(act_b)]], f"graph {b}")
            assert_close_array(Z[lo:hi], Zo, what=f"graph {b} Z")
            assert_close_array(dZ[lo:hi], dZo, what=f"graph {b} dZ")
            assert_close_array(gg["emb"][lo:hi], go["emb"], what=f"graph {b} d emb")
            for k in range(pr.n_layers):
                for key in go["layers"][k]:
                    assert_close_array(gg["layers"][k][key][b], go["layers"][k][key],
                                       what=f"graph {b} d{key}{k}")
            to = terms_o[0]
            for s in range(pr.S):
                assert_close_scalar(T[b, s], to["head"][s], abs(to["head"][s]) + 1.0, what="l_s")
            assert_close_scalar(T[b, pr.S], to["entropy"], to["entropy"], what="S(P)")
            assert_close_scalar(T[b, pr.S + 1], to["psi"], abs(to["psi"]), what="Psi")
        sol.close()
    finally:
        api.autotune_reset()


def test_c4_backward_on_1k_subgraph_matches_finite_differences():
    """Hand-written backward (GPU) vs the oracle's analytic gradient vs FP64 central
    differences, on the subgraph induced by a 1,000-node BFS ball of the
    100,000-node 20-regular workload graph (relabelled in BFS order)."""
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    pr = get_preset("C4")
    big = pr.graph()
    sub = induced_subgraph(big, bfs_ball(big, 1000, root=0))
    say(f"subgraph n={sub.n} edges={sub.n_edges}")
    dg = api.DeviceGraph.from_csr(sub)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=3, hidden=128, S=64, recompute=True)
    sol = CPRASolver(dg, cfg, pr.lam)
    p = init_params("gcn", sub.n, 3, 128, 64, seed=3)
    sol.load_params(p)
    gamma = -0.3
    from paper_2402_02190_amd.autograd import CPRALoss
    params = sol.params.clone().requires_grad_(True)
    R = CPRALoss.apply(params, sol, gamma)
    R.backward()
    gg = sol.unpack(params.grad)
    p64 = ognn.to_f64(p)
    M = ognn.mean_aggregation_matrix(sub.row_ptr, sub.col_idx)
    ocfg = otrain.StepConfig(problem="mis", lam=pr.lam.astype(np.float64))
    _, terms, _, go = otrain.loss_and_grads(p64, M, sub, ocfg, gamma)
    assert abs(float(R.detach()) - terms[0]["total"]) <= 1e-5 * (np.abs(terms[0]["head"]).sum() +
                                                                   abs(gamma) * terms[0]["entropy"])
    assert_close_array(gg["emb"], go["emb"], what="GPU vs oracle d emb")
    for k in range(3):
        assert_close_array(gg["layers"][k]["Ws"], go["layers"][k]["Ws"], what=f"GPU vs oracle dWs{k}")
        assert_close_array(gg["layers"][k]["Wn"], go["layers"][k]["Wn"], what=f"GPU vs oracle dWn{k}")

    def total(pp):
        Z, _ = ognn.forward(pp, M)
        return oobj.loss_terms(Z, sub, "mis", ocfg.lam, gamma, 2)["total"]

    # Central differences along sparse random directions with a small step, so that
    # no ReLU of the (nearly tree-shaped) subgraph changes side within the step.
    rng = np.random.default_rng(0)
    h = 1e-8
    for key in [("emb",), ("layers", 0, "Wn"), ("layers", 1, "Ws"), ("layers", 2, "Ws")]:
        arr = p64["emb"] if key == ("emb",) else p64["layers"][key[1]][key[2]]
        gpu_g = gg["emb"] if key == ("emb",) else gg["layers"][key[1]][key[2]]
        D = rng.standard_normal(arr.shape) * (rng.random(arr.shape) < 0.01)
        arr += h * D
        fp = total(p64)
        arr -= 2 * h * D
        fm = total(p64)
        arr += h * D
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(gpu_g.astype(np.float64) * D))
        say(f"  FD {key}: fd={fd:.8e} gpu={an:.8e} rel={abs(fd - an) / max(1.0, abs(fd)):.2e}")
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(fd))
