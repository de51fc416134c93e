"""Per-graph weights in batched mode (one network per graph of a block-diagonal
batch): the grouped GEMMs through the C ABI against per-graph float64 products,
and the training step against the oracle that solves each graph alone."""

import numpy as np
import pytest
import torch

from helpers import N_GEMM_CFGS, assert_close_array, assert_close_scalar, assert_update_close, \
    check_relu_decisions, need_gpu, say, to_dev
from oracle import gnn as ognn
from oracle import train as otrain
from workloads import CSRGraph, disjoint_union, erdos_renyi_graph, init_params_per_graph, \
    random_regular_graph

pytestmark = pytest.mark.gpu



@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def api():
    from paper_2402_02190_amd import api as a
    return a


def edgeless(n):
    return CSRGraph(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), None)


# graph sizes straddle every row-tile height (32, 64, 128), with an empty and a one-node graph
SIZES = [37, 130, 0, 64, 1, 257, 5, 96]


def ragged_batch(with_edges=True):
    if not with_edges:
        return disjoint_union([edgeless(n) for n in SIZES])
    return disjoint_union([random_regular_graph(38, 3, 1), erdos_renyi_graph(130, 0.05, 2),
                           edgeless(0), random_regular_graph(64, 4, 3), edgeless(1),
                           erdos_renyi_graph(257, 0.02, 4), random_regular_graph(6, 3, 5),
                           erdos_renyi_graph(96, 0.06, 6)])


def graph_rows(g):
    gp = np.asarray(g.graph_ptr, dtype=np.int64)
    return [(int(gp[b]), int(gp[b + 1])) for b in range(gp.size - 1)]


def per_graph_preacts(p64, g, n_hidden):
    """The FP64 pre-activations of the hidden layers, graph by graph (each graph
    its own network), stacked in the batch's row order."""
    out = [np.zeros((g.n, 0))] * n_hidden
    parts = [[] for _ in range(n_hidden)]
    for b, (lo, hi) in enumerate(graph_rows(g)):
        if hi == lo:
            continue
        sub = otrain.objective._slice_graph(g, lo, hi)
        M = ognn.mean_aggregation_matrix(sub.row_ptr, sub.col_idx)
        _, cache = ognn.forward(otrain.graph_params(p64, b, lo, hi), M)
        for k in range(n_hidden):
            parts[k].append(cache[k]["Y"])
    for k in range(n_hidden):
        out[k] = np.vstack(parts[k])
    return out


@pytest.mark.parametrize("cfg", range(N_GEMM_CFGS))
def test_grouped_rows_gemm_every_tile_config(cfg):
    """C[rows of g] = relu(A[rows of g] op(B_g) + bias_g) for both B layouts, with every
    tile configuration forced, on ragged graph sizes and unaligned widths."""
    a = api()
    g = ragged_batch(with_edges=False)
    dg = a.DeviceGraph.from_csr(g)
    G, n = g.n_graphs, g.n
    rng = np.random.default_rng(cfg)
    try:
        for tb in (False, True):
            for K, N in ((24, 40), (128, 64), (7, 3)):
                key = f"{'NT' if tb else 'NN'}|g1:{G}|{n}x{N}x{K}"
                a.autotune_reset()
                a.autotune_set(key, cfg, 1)
                A = rng.standard_normal((n, K)).astype(np.float32)
                B = rng.standard_normal((G, N, K) if tb else (G, K, N)).astype(np.float32)
                bias = rng.standard_normal((G, N)).astype(np.float32)
                C = torch.full((n, N), np.nan, dtype=torch.float32, device="cuda")
                a.gemm_grouped_rows(dg, to_dev(A), to_dev(B), C, tb, to_dev(bias), relu=True)
                torch.cuda.synchronize()
                ref = np.zeros((n, N))
                for b, (lo, hi) in enumerate(graph_rows(g)):
                    Bg = B[b].T if tb else B[b]
                    ref[lo:hi] = np.maximum(A[lo:hi].astype(np.float64) @ Bg + bias[b], 0.0)
                assert_close_array(C.cpu().numpy(), ref, 2e-6, f"cfg {cfg} {key}")
    finally:
        a.autotune_reset()


@pytest.mark.parametrize("cfg", range(N_GEMM_CFGS))
def test_grouped_k_gemm_every_tile_config(cfg):
    """C_g = A[rows of g]^T B[rows of g] and the per-graph column sums of A (the bias
    gradient), with every tile configuration and split-K forced; empty graphs give 0."""
    a = api()
    g = ragged_batch(with_edges=False)
    dg = a.DeviceGraph.from_csr(g)
    G, n = g.n_graphs, g.n
    rng = np.random.default_rng(100 + cfg)
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    try:
        for M, N in ((40, 24), (64, 128), (3, 5)):
            for with_bg in (False, True):
                for splits in (1, 3, 16):
                    key = f"TN|g2:{G}|{M}x{N + int(with_bg)}x{n}"
                    a.autotune_reset()
                    a.autotune_set(key, cfg, splits)
                    A = rng.standard_normal((n, M)).astype(np.float32)
                    B = rng.standard_normal((n, N)).astype(np.float32)
                    C = torch.full((G, M, N), np.nan, dtype=torch.float32, device="cuda")
                    bg = torch.full((G, M), np.nan, dtype=torch.float32, device="cuda") if with_bg else None
                    a.gemm_grouped_k(dg, to_dev(A), to_dev(B), C, bg, ws=ws)
                    torch.cuda.synchronize()
                    ref = np.zeros((G, M, N))
                    rbg = np.zeros((G, M))
                    for b, (lo, hi) in enumerate(graph_rows(g)):
                        ref[b] = A[lo:hi].T.astype(np.float64) @ B[lo:hi]
                        rbg[b] = A[lo:hi].astype(np.float64).sum(axis=0)
                    what = f"cfg {cfg} {key} splits {splits}"
                    assert_close_array(C.cpu().numpy(), ref, 2e-6, what)
                    if with_bg:
                        assert_close_array(bg.cpu().numpy(), rbg, 2e-6, what + " bias grad")
    finally:
        a.autotune_reset()


def _solver(g, kind, L, in_dim, H, S, problem, nu=0.0, recompute=False, seed=3):
    a = api()
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    dg = a.DeviceGraph.from_csr(g)
    lam = np.linspace(0.5, 3.0, S).astype(np.float32) if problem == "mis" else None
    cfg = CPRAConfig(problem=problem, layer_kind=kind, n_layers=L, hidden=H, S=S, in_dim=in_dim,
                     nu=nu, recompute=recompute, per_graph_weights=True, T=100)
    sol = CPRASolver(dg, cfg, lam)
    p = init_params_per_graph(kind, g.n, L, H, S, g.n_graphs, seed=seed, in_dim=in_dim)
    if kind == "sage":
        rng = np.random.default_rng(seed)
        for Ly in p["layers"]:
            Ly["b"] = (0.1 * rng.standard_normal(Ly["b"].shape)).astype(np.float32)
    sol.load_params(p)
    return sol, cfg, lam


STEP_CASES = [
    # name, kind, layers, in_dim, hidden, S, problem, nu, recompute
    ("gcn2_lf_last_maxcut", "gcn", 2, 16, 16, 8, "maxcut", 0.1, False),
    ("sage2_af_last_mis", "sage", 2, 16, 16, 24, "mis", 0.0, False),
    ("sage3_lf_first_recompute", "sage", 3, 24, 16, 8, "mis", 0.1, True),
    ("gcn2_h64_s32_c3_shape", "gcn", 2, 64, 64, 32, "maxcut", 0.1, False),
]


@pytest.mark.parametrize("case", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_per_graph_train_step_matches_oracle(case):
    """Two training steps with one network per graph: Z, dZ, the per-graph loss terms,
    every gradient (embedding and each graph's layers) and the Adam update against the
    oracle that solves each graph alone (ReLU decisions taken from the GPU's forward)."""
    name, kind, L, in_dim, H, S, problem, nu, recompute = case
    g = ragged_batch()
    say(f"per-graph step {name} n={g.n} graphs={g.n_graphs}")
    sol, cfg, lam = _solver(g, kind, L, in_dim, H, S, problem, nu, recompute)
    ocfg = otrain.StepConfig(problem=problem, lam=None if lam is None else lam.astype(np.float64),
                             nu=nu, lr=cfg.lr)
    from paper_2402_02190_amd.solver import gamma_schedule
    for _ in range(2):
        t = sol.t
        p_before = sol.unpack(sol.params)
        m_before, v_before = sol.unpack(sol.m), sol.unpack(sol.v)
        sol.step()
        torch.cuda.synchronize()
        gamma = gamma_schedule(t, cfg.T, cfg.gamma_start, cfg.gamma_end)
        active = sol.relu_active()
        check_relu_decisions(active, per_graph_preacts(ognn.to_f64(p_before), g, len(active)),
                             f"t={t}")
        Zo, terms_o, dZo, go = otrain.loss_and_grads_per_graph(
            ognn.to_f64(p_before), g, ocfg, gamma, relu_active=active)
        assert_close_array(sol.Z.cpu().numpy()[: g.n], Zo, what=f"[{t}] Z")
        assert_close_array(sol.dZ.cpu().numpy()[: g.n], dZo, what=f"[{t}] dZ")
        T_gpu = sol.terms.cpu().numpy()
        assert len(terms_o) == g.n_graphs
        for gi, to in enumerate(terms_o):
            for s in range(S):
                assert_close_scalar(T_gpu[gi, s], to["head"][s], abs(to["head"][s]) + 1.0, what="l_s")
            assert_close_scalar(T_gpu[gi, S], to["entropy"], to["entropy"] + 1e-9, what="S(P)")
        gg = sol.unpack(sol.grads)
        assert_close_array(gg["emb"], go["emb"], what=f"[{t}] d emb")
        for k in range(L):
            for key in go["layers"][k]:
                assert gg["layers"][k][key].shape == go["layers"][k][key].shape
                for b in range(g.n_graphs):
                    ref = go["layers"][k][key][b]
                    got = gg["layers"][k][key][b]
                    if not np.any(ref):  # the empty graph: exactly zero
                        assert not np.any(got), f"{key}{k} graph {b}"
                    else:
                        assert_close_array(got, ref, what=f"[{t}] d{key}{k} graph {b}")
        # Adam from the GPU's gradient in FP64, on the last layer of every graph
        pn = ognn.to_f64(p_before)
        g64 = ognn.to_f64(gg)
        mo, vo = ognn.to_f64(m_before), ognn.to_f64(v_before)
        after = sol.unpack(sol.params)
        otrain.adam_update(pn["layers"][-1]["Wn"], g64["layers"][-1]["Wn"], mo["layers"][-1]["Wn"],
                           vo["layers"][-1]["Wn"], t + 1, cfg.lr)
        assert_update_close(after["layers"][-1]["Wn"], p_before["layers"][-1]["Wn"],
                            pn["layers"][-1]["Wn"], what=f"[{t}] Wn update")
    sol.close()


def test_per_graph_forward_and_standalone_backward():
    """cpra_model_forward / cpra_model_backward (the backward builds its own row
    maps) against per-graph oracle forwards and backwards with an arbitrary dZ."""
    a = api()
    g = ragged_batch()
    S = 12
    sol, cfg, _ = _solver(g, "sage", 2, 20, 20, S, "maxcut")
    p64 = ognn.to_f64(sol.unpack(sol.params))
    sol.forward()
    torch.cuda.synchronize()
    dZ = np.random.default_rng(5).standard_normal((g.n, S)).astype(np.float32)
    grads = torch.zeros_like(sol.params)
    a.model_backward(sol.graph, sol.model_cfg, sol.params, to_dev(dZ), grads, sol.ws)
    torch.cuda.synchronize()
    gg = sol.unpack(grads)
    Z = sol.Z.cpu().numpy()
    relu = sol.relu_active()
    for b, (lo, hi) in enumerate(graph_rows(g)):
        if hi == lo:
            continue
        sub = otrain.objective._slice_graph(g, lo, hi)
        M = ognn.mean_aggregation_matrix(sub.row_ptr, sub.col_idx)
        pb = otrain.graph_params(p64, b, lo, hi)
        Zo, cache = ognn.forward(pb, M)
        check_relu_decisions([r[lo:hi] for r in relu], [c["Y"] for c in cache[: len(relu)]],
                             f"graph {b}")
        assert_close_array(Z[lo:hi], Zo, what=f"Z graph {b}")
        go = ognn.backward(pb, M, cache, dZ[lo:hi].astype(np.float64), [r[lo:hi] for r in relu])
        assert_close_array(gg["emb"][lo:hi], go["emb"], what=f"d emb graph {b}")
        for k in range(2):
            for key in go["layers"][k]:
                assert_close_array(gg["layers"][k][key][b], go["layers"][k][key],
                                   what=f"d{key}{k} graph {b}")
    sol.close()


def test_per_graph_graph_replay_is_bit_identical_to_eager():
    """The captured step (row maps built inside the graph) replays to the same bits."""
    g = ragged_batch()
    a_sol, _, _ = _solver(g, "gcn", 2, 16, 16, 8, "mis")
    b_sol, _, _ = _solver(g, "gcn", 2, 16, 16, 8, "mis")
    a_sol.run(7, use_graph=False)
    b_sol.run(3, use_graph=True)
    b_sol.run(4, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(a_sol.params, b_sol.params)
    assert torch.equal(a_sol.terms, b_sol.terms)
    a_sol.close()
    b_sol.close()


def test_per_graph_rejects_a_mismatched_group_count():
    a = api()
    from paper_2402_02190_amd._lib import CpraError
    g = ragged_batch()
    dg = a.DeviceGraph.from_csr(g)
    cfg = a.make_model_cfg(a.GCN, 2, 8, 8, 4, weight_groups=g.n_graphs + 1)
    Z = torch.zeros((g.n, 4), device="cuda")
    params = torch.zeros(a.model_param_count(cfg, g.n), device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(CpraError):
        a.model_forward(dg, cfg, params, Z, ws)


def test_shared_vs_per_graph_comparison_runs():
    """The quality comparison (pergraph.py) on a small batch: both arms train, and each
    graph's best value is a valid cut of that graph (between 0 and its edge count)."""
    from paper_2402_02190_amd import pergraph
    from workloads.presets import Preset
    g = ragged_batch()
    pr = Preset("small", "maxcut", "gcn", 2, 16, 8, None, -2.0, 0.1, 40, nu=0.1)
    a = api()
    dg = a.DeviceGraph.from_csr(g)
    for per_graph in (False, True):
        best, seconds = pergraph.train_arm(pr, g, dg, per_graph, seed=1, T=40)
        assert best.shape == (g.n_graphs,) and seconds > 0
        for b, (lo, hi) in enumerate(graph_rows(g)):
            m = int(g.row_ptr[hi] - g.row_ptr[lo]) // 2
            assert 0 <= best[b] <= m
