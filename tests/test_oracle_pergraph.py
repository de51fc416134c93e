"""Pins of the per-graph-weights oracle (one network per graph of a
block-diagonal batch): identical weights reproduce the shared-weight batch,
graphs do not interact, and the stitched gradients match finite differences."""

import copy

import numpy as np
import pytest

from oracle import gnn, train
from workloads import CSRGraph, disjoint_union, erdos_renyi_graph, init_params_per_graph, \
    random_regular_graph


def batch():
    return disjoint_union([random_regular_graph(30, 3, 1), erdos_renyi_graph(23, 0.2, 2),
                           CSRGraph(0, np.zeros(1, np.int32), np.zeros(0, np.int32), None),
                           random_regular_graph(18, 4, 3)])


def cfg_for(problem, S, nu=0.1):
    lam = np.linspace(0.5, 3.0, S) if problem == "mis" else None
    return train.StepConfig(problem=problem, lam=lam, nu=nu)


@pytest.mark.parametrize("kind,problem", [("gcn", "mis"), ("sage", "maxcut"), ("sage", "mis")])
def test_identical_weights_reproduce_the_shared_weight_batch(kind, problem):
    """Every graph given the same network = the shared-weight batch: Z, dZ, terms
    and the embedding gradient agree, and the per-graph layer gradients add up to
    the shared gradient (the shared weight's gradient sums over the graphs)."""
    g = batch()
    G, S = g.n_graphs, 6
    pg = gnn.to_f64(init_params_per_graph(kind, g.n, 2, 8, S, G, seed=4))
    if kind == "sage":
        for L in pg["layers"]:
            L["b"][:] = np.linspace(-0.2, 0.3, L["b"].shape[1])[None, :]
    for L in pg["layers"]:
        for k in L:
            L[k][:] = L[k][0]
    shared = {"emb": pg["emb"], "layers": [{k: v[0] for k, v in L.items()} for L in pg["layers"]]}
    cfg = cfg_for(problem, S)
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    Zs, ts, dZs, gs = train.loss_and_grads(shared, M, g, cfg, 0.3)
    Zp, tp, dZp, gpg = train.loss_and_grads_per_graph(pg, g, cfg, 0.3)
    np.testing.assert_allclose(Zp, Zs, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dZp, dZs, rtol=1e-12, atol=1e-12)
    assert len(tp) == len(ts) == G
    for a, b in zip(tp, ts):
        np.testing.assert_allclose(a["head"], b["head"], rtol=1e-12, atol=1e-12)
        assert a["total"] == pytest.approx(b["total"], rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(gpg["emb"], gs["emb"], rtol=1e-12, atol=1e-12)
    for Lp, Ls in zip(gpg["layers"], gs["layers"]):
        for k in Ls:
            np.testing.assert_allclose(Lp[k].sum(axis=0), Ls[k], rtol=1e-10, atol=1e-12)


def test_graphs_do_not_interact():
    """Changing graph 0's network leaves every other graph's outputs and gradients unchanged."""
    g = batch()
    G, S = g.n_graphs, 5
    pg = gnn.to_f64(init_params_per_graph("sage", g.n, 2, 8, S, G, seed=5))
    cfg = cfg_for("mis", S)
    Z0, _, dZ0, g0 = train.loss_and_grads_per_graph(pg, g, cfg, -0.5)
    pert = copy.deepcopy(pg)
    for L in pert["layers"]:
        for k in L:
            L[k][0] += 0.25
    Z1, _, dZ1, g1 = train.loss_and_grads_per_graph(pert, g, cfg, -0.5)
    n0 = int(g.graph_ptr[1])
    assert not np.allclose(Z1[:n0], Z0[:n0])
    assert np.array_equal(Z1[n0:], Z0[n0:]) and np.array_equal(dZ1[n0:], dZ0[n0:])
    for L0, L1 in zip(g0["layers"], g1["layers"]):
        for k in L0:
            assert np.array_equal(L0[k][1:], L1[k][1:])


@pytest.mark.parametrize("which", [("Wn", 1, 0), ("Ws", 3, 1), ("b", 1, 1)])
def test_per_graph_gradient_finite_differences(which):
    key, b, layer = which
    g = batch()
    G, S = g.n_graphs, 4
    pg = gnn.to_f64(init_params_per_graph("sage", g.n, 2, 8, S, G, seed=6))
    cfg = cfg_for("mis", S)
    _, _, _, grads = train.loss_and_grads_per_graph(pg, g, cfg, 0.2)
    rng = np.random.default_rng(7)
    D = rng.standard_normal(pg["layers"][layer][key][b].shape)

    def total(h):
        p = copy.deepcopy(pg)
        p["layers"][layer][key][b] += h * D
        _, t, _, _ = train.loss_and_grads_per_graph(p, g, cfg, 0.2)
        return sum(x["total"] for x in t)

    h = 1e-6
    fd = (total(h) - total(-h)) / (2 * h)
    an = float(np.sum(grads["layers"][layer][key][b] * D))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd))
