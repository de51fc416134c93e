"""Parity of the multi-instance path (one instance per head: per-head edge
weights on the graph's pattern) against the FP64 oracle, through the C ABI:
the fused loss and its gradient, the rounding/evaluation on each head's own
instance, and whole training steps (also on a block-diagonal batch and in a
replayed graph)."""

import numpy as np
import pytest
import torch

from helpers import assert_close_array, assert_close_scalar, check_relu_decisions, need_gpu, say, to_dev
from oracle import evaluate as oev
from oracle import gnn as ognn
from oracle import objective as oobj
from oracle import train as otrain
from workloads import (csr_from_edges, disjoint_union, erdos_renyi_graph, init_params,
                       instance_edge_weights, random_regular_graph)
from workloads.params import random_logits

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def api():
    from paper_2402_02190_amd import api as a
    return a


def weighted_er(n, p, seed):
    g = erdos_renyi_graph(n, p, seed)
    u, v, _ = g.edge_list()
    w = np.random.default_rng(seed).uniform(0.25, 3.0, size=u.size).astype(np.float32)
    return csr_from_edges(n, u, v, w)


GRAPHS = {
    "rrg3_100": lambda: random_regular_graph(100, 3, 1),        # tail chunk of 3 neighbours
    "er_sparse_300": lambda: erdos_renyi_graph(300, 1.5 / 299, 2),  # isolated nodes, ragged degrees
    "rrg20_500": lambda: random_regular_graph(500, 20, 3),      # full chunks only
    "weighted_er_400": lambda: weighted_er(400, 0.02, 4),       # graph weights, replaced per head
    "batch": lambda: disjoint_union([erdos_renyi_graph(37, 0.1, 5), erdos_renyi_graph(1, 0.0, 6),
                                     erdos_renyi_graph(250, 0.02, 7), random_regular_graph(90, 5, 8)]),
}

LOSS_CASES = [
    # graph, S, problem, weight kind, drop, alpha, nu
    ("rrg3_100", 10, "mis", "uniform", 0.3, 2, 0.0),
    ("er_sparse_300", 1, "maxcut", "signed", 0.0, 2, 0.0),
    ("rrg20_500", 130, "mis", "integer", 0.5, 4, 0.2),
    ("weighted_er_400", 64, "maxcut", "signed", 0.2, 2, 0.1),
    ("batch", 32, "maxcut", "uniform", 0.1, 2, 0.1),
    ("batch", 7, "mis", "signed", 0.25, 6, 0.3),
]


def head_scale(Z, g, ew, problem, lam):
    """Sum of the absolute summands of each head's loss (the tolerance's scale)."""
    P, _ = oobj.sigmoid_pair(Z)
    n = len(g.row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    up = rows < g.col_idx
    ei, ej, w = rows[up], g.col_idx[up].astype(np.int64), np.abs(ew[up]).astype(np.float64)
    pair = np.sum(w * P[ei] * P[ej], axis=0)
    if problem == "mis":
        return P.sum(0) + np.abs(lam) * pair
    return 2 * pair + np.sum(w * (P[ei] + P[ej]), axis=0)


@pytest.mark.parametrize("case", LOSS_CASES, ids=[f"{c[0]}_S{c[1]}_{c[2]}_{c[3]}" for c in LOSS_CASES])
def test_multi_instance_loss_matches_oracle(case):
    a = api()
    gname, S, problem, kind, drop, alpha, nu = case
    g = GRAPHS[gname]()
    ew = instance_edge_weights(g, S, seed=S + 3, kind=kind, drop=drop)
    say(f"multi-instance loss {gname} S={S} {problem} {kind} drop={drop}")
    dg = a.DeviceGraph.from_csr(g)
    Z = random_logits(g.n, S, seed=S + alpha)
    lam = np.logspace(-1, 1, S).astype(np.float32)
    gamma = -0.6
    pid = a.MIS if problem == "mis" else a.MAXCUT
    ewd = to_dev(ew)
    lam_d = to_dev(lam) if problem == "mis" else None  # held: the config keeps only its address
    cfg = a.make_loss_cfg(pid, S, lam_d, alpha, gamma, nu, edge_weight=ewd)
    ws = torch.empty(a.loss_workspace_bytes(dg, cfg), dtype=torch.uint8, device="cuda")
    Zd = to_dev(Z)
    dZ = torch.empty_like(Zd)
    terms = torch.empty((dg.n_graphs, S + 2), dtype=torch.float64, device="cuda")
    a.loss_fwd_bwd(dg, cfg, Zd, dZ, terms, ws)
    torch.cuda.synchronize()
    T = terms.cpu().numpy()
    dZh = dZ.cpu().numpy()
    Z64 = Z.astype(np.float64)
    gp = g.graph_ptr
    lam64 = lam.astype(np.float64)
    for gi in range(len(gp) - 1):
        lo, hi = int(gp[gi]), int(gp[gi + 1])
        sub = oobj._slice_graph(g, lo, hi) if len(gp) > 2 else g
        ea, eb = oobj.entry_range(g, lo, hi)
        ref = oobj.loss_terms(Z64[lo:hi], sub, problem, lam64, gamma, alpha, nu, 0, None, ew[ea:eb])
        scale = head_scale(Z64[lo:hi], sub, ew[ea:eb], problem, lam64) if hi > lo else np.zeros(S)
        for s in range(S):
            assert_close_scalar(T[gi, s], ref["head"][s], scale[s], what=f"graph {gi} l_{s}")
        assert_close_scalar(T[gi, S], ref["entropy"], abs(ref["entropy"]) + 1e-30, what="S(P)")
        assert_close_scalar(T[gi, S + 1], ref["psi"], abs(ref["psi"]) + 1e-30, what="Psi")
        if hi > lo:
            gref = oobj.grad_wrt_Z(Z64[lo:hi], sub, problem, lam64, gamma, alpha, nu, 0, None,
                                   ew[ea:eb])
            assert_close_array(dZh[lo:hi], gref, what=f"dZ graph {gi}")
    # deterministic: a second call gives identical bits
    dZ2, terms2 = torch.empty_like(dZ), torch.empty_like(terms)
    a.loss_fwd_bwd(dg, cfg, Zd, dZ2, terms2, ws)
    torch.cuda.synchronize()
    assert torch.equal(dZ, dZ2) and torch.equal(terms, terms2)


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
def test_equal_columns_match_the_plain_path(problem):
    """Every head given the graph's own weights: the per-head path reproduces the
    plain one (same gather order; MaxCut's degree summed in the pass instead of
    read from wdeg)."""
    a = api()
    g = weighted_er(400, 0.02, 4)
    S = 24
    ew = np.repeat(g.weight[:, None], S, axis=1)
    dg = a.DeviceGraph.from_csr(g)
    Zd = to_dev(random_logits(g.n, S, seed=9))
    lam = to_dev(np.logspace(-1, 1, S).astype(np.float32)) if problem == "mis" else None
    pid = a.MIS if problem == "mis" else a.MAXCUT
    ewd = to_dev(ew)
    c1 = a.make_loss_cfg(pid, S, lam, 2, -0.3, 0.1)
    c2 = a.make_loss_cfg(pid, S, lam, 2, -0.3, 0.1, edge_weight=ewd)
    ws = torch.empty(a.loss_workspace_bytes(dg, c1), dtype=torch.uint8, device="cuda")
    d1, d2 = torch.empty_like(Zd), torch.empty_like(Zd)
    t1 = torch.empty((1, S + 2), dtype=torch.float64, device="cuda")
    t2 = torch.empty_like(t1)
    a.loss_fwd_bwd(dg, c1, Zd, d1, t1, ws)
    a.loss_fwd_bwd(dg, c2, Zd, d2, t2, ws)
    torch.cuda.synchronize()
    assert_close_array(d2.cpu().numpy(), d1.cpu().numpy(), 1e-6, "dZ")
    assert_close_array(t2.cpu().numpy(), t1.cpu().numpy(), 1e-6, "terms")
    if problem == "mis":  # no degree involved: the same sums in the same order
        assert torch.equal(d1, d2)


EVAL_CASES = [("rrg3_100", 10, "mis", "integer", 0.3), ("er_sparse_300", 1, "maxcut", "signed", 0.2),
              ("rrg20_500", 130, "mis", "uniform", 0.6), ("weighted_er_400", 64, "maxcut", "signed", 0.0),
              ("batch", 32, "maxcut", "uniform", 0.4), ("batch", 5, "mis", "integer", 0.5)]


@pytest.mark.parametrize("case", EVAL_CASES, ids=[f"{c[0]}_S{c[1]}_{c[2]}" for c in EVAL_CASES])
def test_multi_instance_eval_matches_oracle(case):
    a = api()
    gname, S, problem, kind, drop = case
    g = GRAPHS[gname]()
    ew = instance_edge_weights(g, S, seed=S + 11, kind=kind, drop=drop)
    say(f"multi-instance eval {gname} S={S} {problem}")
    dg = a.DeviceGraph.from_csr(g)
    Z = random_logits(g.n, S, seed=S + 1)
    Zd = to_dev(Z)
    G = dg.n_graphs
    val = torch.empty(G * S, dtype=torch.int64, device="cuda")
    vio = torch.empty(G * S, dtype=torch.int64, device="cuda")
    wv = torch.empty(G * S, dtype=torch.float64, device="cuda")
    X = torch.empty((g.n, S), dtype=torch.uint8, device="cuda")
    a.round_eval(dg, a.MIS if problem == "mis" else a.MAXCUT, Zd, X, val, vio, wv,
                 edge_weight=to_dev(ew))
    torch.cuda.synchronize()
    Xo = oev.round_solutions(Z.astype(np.float64))
    assert np.array_equal(X.cpu().numpy(), Xo)
    ev = oev.evaluate(Xo, g, problem, None, ew)
    val, vio, wv = (t.cpu().numpy().reshape(G, S) for t in (val, vio, wv))
    for gi, e in enumerate(ev):
        if problem == "mis":
            assert np.array_equal(val[gi], e["size"])
            assert np.array_equal(vio[gi], e["violations"])
        else:
            assert np.array_equal(val[gi], e["cut_edges"])
            np.testing.assert_allclose(wv[gi], e["cut"], rtol=1e-12, atol=1e-9)


STEP_CASES = [
    # name, graph fn, problem, kind, layers, hidden, S, weight kind, drop, nu
    ("gcn2_mis_rrg", lambda: random_regular_graph(300, 4, 2), "mis", "gcn", 2, 32, 12, "integer", 0.3, 0.0),
    ("sage2_maxcut_signed", lambda: erdos_renyi_graph(400, 0.015, 3), "maxcut", "sage", 2, 32, 20,
     "signed", 0.1, 0.1),
    ("gcn2_maxcut_batch", lambda: disjoint_union([erdos_renyi_graph(80, 0.06, 4), random_regular_graph(60, 3, 5),
                                                  erdos_renyi_graph(3, 0.0, 6)]),
     "maxcut", "gcn", 2, 16, 8, "uniform", 0.2, 0.1),
]


@pytest.mark.parametrize("case", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_multi_instance_train_step_matches_oracle(case):
    """One training step with one instance per head: Z, dZ, the loss terms and every
    gradient against the oracle; then the captured graph replays bit-identically to
    eager steps from the same state."""
    from paper_2402_02190_amd import api as A
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    name, gfn, problem, kind, L, H, S, wkind, drop, nu = case
    g = gfn()
    ew = instance_edge_weights(g, S, seed=7, kind=wkind, drop=drop)
    say(f"multi-instance step {name} n={g.n} S={S}")
    dg = A.DeviceGraph.from_csr(g)
    lam = np.linspace(0.5, 3.0, S).astype(np.float32) if problem == "mis" else None
    cfg = CPRAConfig(problem=problem, layer_kind=kind, n_layers=L, hidden=H, S=S, nu=nu, T=200)
    sol = CPRASolver(dg, cfg, lam, edge_weight=ew)
    p = init_params(kind, g.n, L, H, S, seed=5)
    sol.load_params(p)
    sol.step()
    torch.cuda.synchronize()
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ocfg = otrain.StepConfig(problem=problem, lam=None if lam is None else lam.astype(np.float64),
                             nu=nu, edge_weight=ew)
    active = sol.relu_active()
    Zo, terms_o, dZo, go, cache = otrain.loss_and_grads(ognn.to_f64(p), M, g, ocfg, cfg.gamma_start,
                                                        relu_active=active, return_cache=True)
    check_relu_decisions(active, [c["Y"] for c in cache[: len(active)]], "instances")
    assert_close_array(sol.Z.cpu().numpy()[: g.n], Zo, what="Z")
    assert_close_array(sol.dZ.cpu().numpy()[: g.n], dZo, what="dZ")
    gg = sol.unpack(sol.grads)
    assert_close_array(gg["emb"], go["emb"], what="d emb")
    for k in range(L):
        for key in go["layers"][k]:
            assert_close_array(gg["layers"][k][key], go["layers"][k][key], what=f"d{key}{k}")
    T_gpu = sol.terms.cpu().numpy()
    for gi, to in enumerate(terms_o):
        for s in range(S):
            assert_close_scalar(T_gpu[gi, s], to["head"][s], np.abs(to["head"]).sum() + 1.0,
                                what=f"graph {gi} l_{s}")
    ev = sol.evaluate()
    Xo = oev.round_solutions(sol.Z.cpu().numpy()[: g.n].astype(np.float64))
    evo = oev.evaluate(Xo, g, problem, None, ew)
    for gi, e in enumerate(evo):
        key = "size" if problem == "mis" else "cut_edges"
        assert np.array_equal(ev["value"][gi], e[key])
        if problem == "mis":
            assert np.array_equal(ev["violations"][gi], e["violations"])
    sol.close()
    # a replayed graph reproduces eager steps bit for bit
    ea, gr = CPRASolver(dg, cfg, lam, edge_weight=ew), CPRASolver(dg, cfg, lam, edge_weight=ew)
    ea.load_params(p)
    gr.load_params(p)
    ea.run(6, use_graph=False)
    gr.run(6, use_graph=True)
    torch.cuda.synchronize()
    assert torch.equal(ea.params, gr.params) and torch.equal(ea.terms, gr.terms)
    ea.close()
    gr.close()


@pytest.mark.parametrize("problem", ["maxcut", "mis"])
def test_together_vs_one_by_one_driver_runs(problem):
    """The comparison driver on tiny instances: both arms train and score every instance."""
    from paper_2402_02190_amd import multiinstance
    res = multiinstance.run(problem, instances=3, n=60, degree=3, hidden=8, T=40, seed=1)
    assert res["instances"] == 3
    assert res["together_seconds"] > 0 and res["one_by_one_seconds"] > 0
    assert res["together_better"] + res["equal"] + res["one_by_one_better"] == 3
    assert res["mean_score_together"] >= 0 and res["mean_score_one_by_one"] >= 0
