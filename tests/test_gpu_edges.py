"""Degenerate and extreme inputs through the C ABI: an empty graph, a graph
without edges, a batch with an empty member graph, one very high-degree node,
and the maximum head count, each against the oracle."""

import numpy as np
import pytest
import torch

from helpers import assert_close_array, assert_close_scalar, need_gpu, say, to_dev
from oracle import evaluate as oev
from oracle import gnn as ognn
from oracle import objective as oobj
from oracle import train as otrain
from oracle import warmstart as W
from workloads import CSRGraph, csr_from_edges, disjoint_union, init_params, random_channels, \
    random_regular_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def mods():
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    return api, CPRAConfig, CPRASolver


def edgeless(n):
    return CSRGraph(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), None)


def star(leaves):
    return csr_from_edges(leaves + 1, np.zeros(leaves, np.int64), np.arange(1, leaves + 1))


def _head_scale(Z, g, problem, lam):
    """Sum of |summands| of each head's relaxed objective (its conditioning scale)."""
    P, _ = oobj.sigmoid_pair(Z)
    ei, ej, w = oobj.edges_of(g.row_ptr, g.col_idx, g.weight)
    pair = np.sum(np.abs(w)[:, None] * P[ei] * P[ej], axis=0)
    if problem == "mis":
        return P.sum(axis=0) + np.abs(np.asarray(lam, dtype=np.float64)) * pair
    return 2.0 * pair + np.sum(np.abs(w)[:, None] * (P[ei] + P[ej]), axis=0)


def _step_vs_oracle(g, kind="sage", L=2, H=32, S=8, problem="mis", what=""):
    api, CPRAConfig, CPRASolver = mods()
    dg = api.DeviceGraph.from_csr(g)
    lam = np.linspace(0.5, 3, S).astype(np.float32) if problem == "mis" else None
    cfg = CPRAConfig(problem=problem, layer_kind=kind, n_layers=L, hidden=H, S=S)
    sol = CPRASolver(dg, cfg, lam)
    p = init_params(kind, g.n, L, H, S, seed=3)
    sol.load_params(p)
    sol.step()
    torch.cuda.synchronize()
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ocfg = otrain.StepConfig(problem=problem, lam=None if lam is None else lam.astype(np.float64))
    Zo, terms, dZo, go = otrain.loss_and_grads(ognn.to_f64(p), M, g, ocfg, cfg.gamma_start)
    if g.n:
        assert_close_array(sol.Z.cpu().numpy()[: g.n], Zo, what=f"{what} Z")
        assert_close_array(sol.dZ.cpu().numpy()[: g.n], dZo, what=f"{what} dZ")
    gg = sol.unpack(sol.grads)
    for k in range(L):
        for key in go["layers"][k]:
            ref = go["layers"][k][key]
            if np.linalg.norm(ref) == 0:
                assert np.all(gg["layers"][k][key] == 0), f"{what} d{key}{k}"
            else:
                assert_close_array(gg["layers"][k][key], ref, what=f"{what} d{key}{k}")
    T = sol.terms_host()
    gp = np.asarray(g.graph_ptr, dtype=np.int64)
    for gi, t in enumerate(terms):
        # every head's term on its own, against the sum of its summands' magnitudes
        lo, hi = int(gp[gi]), int(gp[gi + 1])
        sub = oobj._slice_graph(g, lo, hi) if gp.size > 2 else g
        scale = _head_scale(Zo[lo:hi], sub, problem, lam) + 1e-30
        for s in range(S):
            assert_close_scalar(T[gi, s], t["head"][s], scale[s], what=f"{what} l_{s} graph {gi}")
        assert_close_scalar(T[gi, S], t["entropy"], abs(t["entropy"]) + 1e-30, what=f"{what} S(P)")
        assert_close_scalar(T[gi, S + 1], t["psi"], abs(t["psi"]) + 1e-30, what=f"{what} Psi")
    ev = sol.evaluate()
    Xo = oev.round_solutions(Zo)
    ref_ev = oev.evaluate(Xo, g, problem)
    for gi, e in enumerate(ref_ev):
        if problem == "mis":
            assert np.array_equal(ev["value"][gi], e["size"])
            assert np.array_equal(ev["violations"][gi], e["violations"])
    sol.close()


def test_empty_graph_is_a_no_op():
    api, CPRAConfig, CPRASolver = mods()
    g = CSRGraph(0, np.zeros(1, np.int32), np.zeros(0, np.int32), None)
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem="mis", layer_kind="gcn", n_layers=2, hidden=16, S=4)
    sol = CPRASolver(dg, cfg, np.ones(4, np.float32))
    sol.step()
    sol.forward()
    ev = sol.evaluate()
    torch.cuda.synchronize()
    assert np.all(ev["value"] == 0) and np.all(ev["violations"] == 0)
    say("  empty graph: step, forward and evaluation return without work")
    sol.close()


def test_edgeless_graph_step_matches_oracle():
    _step_vs_oracle(edgeless(70), what="edgeless")


def test_batch_with_an_empty_member_graph():
    g = disjoint_union([random_regular_graph(40, 3, 1), CSRGraph(0, np.zeros(1, np.int32),
                        np.zeros(0, np.int32), None), random_regular_graph(30, 4, 2), edgeless(5)])
    assert g.n_graphs == 4
    _step_vs_oracle(g, kind="gcn", what="batch with empty member")


def test_one_very_high_degree_node():
    _step_vs_oracle(star(5000), kind="sage", S=16, what="star 5000")


def test_maximum_head_count_step_and_eval():
    _step_vs_oracle(random_regular_graph(60, 3, 4), kind="gcn", H=64, S=1024, what="S=1024")


def test_star_triangles_and_features():
    from paper_2402_02190_amd.warmstart import WarmStartNet
    api, _, _ = mods()
    for g in (star(5000), edgeless(37)):
        dg = api.DeviceGraph.from_csr(g)
        net = WarmStartNet(3, 16, 64, 32, 14)
        rand = random_channels(g.n, 14, seed=1)
        feat, tri = net.features(dg, rand, triangles=True)
        torch.cuda.synchronize()
        fo, to = W.node_features(g, rand, 16)
        assert np.array_equal(tri.cpu().numpy()[: g.n], to)
        assert np.array_equal(feat.cpu().numpy()[: g.n].view(np.uint16), W.bf16_bits(fo))


def test_single_node_graph_step_matches_oracle():
    _step_vs_oracle(edgeless(1), kind="sage", what="N=1")


def test_one_head_step_matches_oracle():
    _step_vs_oracle(random_regular_graph(80, 3, 7), kind="gcn", H=16, S=1, what="S=1")
    _step_vs_oracle(random_regular_graph(80, 3, 7), kind="sage", H=16, S=1, problem="maxcut",
                    what="S=1 maxcut")
