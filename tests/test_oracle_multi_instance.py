"""Pins of the multi-instance oracle (one instance per head: per-head edge
weights on a shared pattern, Sec. 3.1 with a different C_s for every head, as
in the multi-instance appendix).  Each pin is computed by code other than the
oracle's: explicit loops over edges, discrete objectives on binary points, a
rebuilt graph without the zero-weight edges, and finite differences."""

import itertools

import numpy as np
import pytest

from oracle import evaluate as oev
from oracle import objective as obj
from workloads import csr_from_edges, disjoint_union, erdos_renyi_graph, instance_edge_weights, \
    random_regular_graph


def loops_head_losses(P, g, ew, problem, lam, nw=None):
    """sum over unordered edges of each head's own weight, written as plain loops."""
    N, S = P.shape
    out = np.zeros(S)
    for s in range(S):
        tot = 0.0
        for i in range(N):
            for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
                j = int(g.col_idx[k])
                if j <= i:
                    continue
                w = float(ew[k, s])
                if problem == "mis":
                    tot += lam[s] * w * P[i, s] * P[j, s]
                else:
                    tot += w * (2 * P[i, s] * P[j, s] - P[i, s] - P[j, s])
        if problem == "mis":
            for i in range(N):
                tot -= (1.0 if nw is None else nw[i, s]) * P[i, s]
        out[s] = tot
    return out


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
@pytest.mark.parametrize("kind", ["uniform", "signed", "integer"])
def test_head_losses_match_loops_over_each_heads_edges(problem, kind):
    g = erdos_renyi_graph(9, 0.45, 3)
    S = 4
    ew = instance_edge_weights(g, S, 7, kind, drop=0.25)
    rng = np.random.default_rng(1)
    Z = rng.normal(0, 2, (g.n, S))
    lam = np.array([0.5, 1.0, 2.0, 3.5])
    nw = rng.uniform(0, 1, (g.n, S)) if problem == "mis" else None
    t = obj.loss_terms(Z, g, problem, lam, 0.3, 2, 0.0, 0, nw, ew)
    P, _ = obj.sigmoid_pair(Z)
    np.testing.assert_allclose(t["head"], loops_head_losses(P, g, ew, problem, lam, nw),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
def test_relaxed_equals_discrete_on_every_binary_point(problem):
    """On binary P the relaxed loss of head s is the discrete objective of instance s
    (relaxation of Sec. 2.2), for all 2^N points of a 7-node graph."""
    g = erdos_renyi_graph(7, 0.5, 5)
    S = 3
    ew = instance_edge_weights(g, S, 11, "integer", drop=0.3)
    lam = np.array([1.0, 2.0, 0.5])
    for bits in itertools.product((0, 1), repeat=g.n):
        x = np.array(bits, dtype=np.float64)
        Z = np.repeat(np.where(x > 0, 40.0, -40.0)[:, None], S, axis=1)
        head = obj.loss_terms(Z, g, problem, lam, 0.0, 2, 0.0, 0, None, ew)["head"]
        for s in range(S):
            inst = obj.head_instance(g, np.asarray(ew, dtype=np.float64), s)
            ei, ej, w = obj.edges_of(inst.row_ptr, inst.col_idx, inst.weight)
            d = obj.discrete_mis(x, ei, ej, w, lam[s]) if problem == "mis" \
                else obj.discrete_maxcut(x, ei, ej, w)
            assert abs(head[s] - d) < 1e-9, (bits, s)


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
def test_zero_weight_is_the_edge_removed(problem):
    """A head whose weight on some edges is 0 equals the plain objective on the graph
    rebuilt without those edges (and with the head's weights on the rest)."""
    g = random_regular_graph(12, 3, 2)
    S = 3
    ew = instance_edge_weights(g, S, 4, "uniform", drop=0.4)
    rng = np.random.default_rng(2)
    Z = rng.normal(0, 1.5, (g.n, S))
    lam = np.array([0.7, 1.3, 2.2])
    t = obj.loss_terms(Z, g, problem, lam, 0.0, 2, 0.0, 0, None, ew)
    gz = obj.grad_wrt_Z(Z, g, problem, lam, 0.0, 2, 0.0, 0, None, ew)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for s in range(S):
        keep = (rows < g.col_idx) & (ew[:, s] != 0)
        h = csr_from_edges(g.n, rows[keep], g.col_idx[keep], ew[keep, s])
        ts = obj.loss_terms(Z[:, [s]], h, problem, lam[[s]], 0.0, 2)
        np.testing.assert_allclose(t["head"][s], ts["head"][0], rtol=1e-12, atol=1e-12)
        gs = obj.grad_wrt_Z(Z[:, [s]], h, problem, lam[[s]], 0.0, 2)
        np.testing.assert_allclose(gz[:, [s]], gs, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
def test_equal_columns_reproduce_the_single_instance_loss(problem):
    g = erdos_renyi_graph(40, 0.1, 8)
    S = 5
    w = np.random.default_rng(3).uniform(0.5, 2, g.nnz)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    # symmetrise: both entries of an edge take the value of its upper entry
    up = {(int(i), int(j)): w[k] for k, (i, j) in enumerate(zip(rows, g.col_idx)) if i < j}
    wsym = np.array([up[(min(i, j), max(i, j))] for i, j in zip(rows, g.col_idx)], np.float32)
    g.weight = wsym
    ew = np.repeat(wsym[:, None], S, axis=1)
    Z = np.random.default_rng(4).normal(0, 2, (g.n, S))
    lam = np.linspace(0.5, 2, S)
    a = obj.loss_terms(Z, g, problem, lam, 0.4, 4, 0.2, 0, None, ew)
    b = obj.loss_terms(Z, g, problem, lam, 0.4, 4, 0.2, 0)
    np.testing.assert_allclose(a["head"], b["head"], rtol=1e-12)
    assert abs(a["total"] - b["total"]) <= 1e-12 * abs(b["total"])
    np.testing.assert_allclose(obj.grad_wrt_Z(Z, g, problem, lam, 0.4, 4, 0.2, 0, None, ew),
                               obj.grad_wrt_Z(Z, g, problem, lam, 0.4, 4, 0.2, 0),
                               rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
def test_gradient_matches_central_differences(problem):
    g = erdos_renyi_graph(10, 0.35, 6)
    S = 3
    ew = instance_edge_weights(g, S, 9, "signed", drop=0.2)
    rng = np.random.default_rng(5)
    Z = rng.normal(0, 1.5, (g.n, S))
    lam = np.array([0.8, 1.6, 2.4])
    nw = rng.uniform(0.2, 1.0, (g.n, S)) if problem == "mis" else None
    args = (problem, lam, 0.35, 4, 0.15, 0, nw, ew)
    G = obj.grad_wrt_Z(Z, g, *args)
    h = 1e-6
    for i in range(g.n):
        for s in range(S):
            Zp, Zm = Z.copy(), Z.copy()
            Zp[i, s] += h
            Zm[i, s] -= h
            fd = (obj.loss_terms(Zp, g, *args)["total"] - obj.loss_terms(Zm, g, *args)["total"]) / (2 * h)
            assert abs(fd - G[i, s]) <= 1e-6 * max(1.0, abs(G[i, s])), (i, s, fd, G[i, s])


def test_evaluation_counts_each_heads_own_edges():
    g = erdos_renyi_graph(30, 0.2, 12)
    S = 6
    ew = instance_edge_weights(g, S, 13, "signed", drop=0.35)
    X = (np.random.default_rng(6).random((g.n, S)) < 0.4).astype(np.uint8)
    mis = oev.evaluate_one(X, g, "mis", None, ew)
    cut = oev.evaluate_one(X, g, "maxcut", None, ew)
    for s in range(S):
        viol = cut_edges = 0
        cutw = 0.0
        for i in range(g.n):
            for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
                j = int(g.col_idx[k])
                if j <= i or ew[k, s] == 0:
                    continue
                viol += int(X[i, s] and X[j, s])
                if X[i, s] != X[j, s]:
                    cut_edges += 1
                    cutw += float(ew[k, s])
        assert mis["violations"][s] == viol
        assert cut["cut_edges"][s] == cut_edges
        assert cut["cut"][s] == pytest.approx(cutw, abs=1e-12)
        assert mis["size"][s] == int(X[:, s].sum())


def test_batch_terms_are_the_members_terms():
    parts = [random_regular_graph(14, 3, 1), erdos_renyi_graph(9, 0.3, 2), random_regular_graph(8, 4, 3)]
    S = 4
    ews = [instance_edge_weights(p, S, 20 + b, "uniform", drop=0.2) for b, p in enumerate(parts)]
    g = disjoint_union(parts)
    ew = np.concatenate(ews, axis=0)
    rng = np.random.default_rng(7)
    Z = rng.normal(0, 2, (g.n, S))
    lam = np.linspace(0.5, 2.0, S)
    tb = obj.batched_loss_terms(Z, g, "mis", lam, 0.2, 2, 0.1, 0, None, ew)
    off = 0
    for p, e, t in zip(parts, ews, tb):
        ts = obj.loss_terms(Z[off:off + p.n], p, "mis", lam, 0.2, 2, 0.1, 0, None, e)
        np.testing.assert_allclose(t["head"], ts["head"], rtol=1e-12)
        off += p.n


def test_asymmetric_weights_are_rejected():
    g = random_regular_graph(8, 3, 1)
    ew = instance_edge_weights(g, 2, 1, "uniform")
    ew[0, 1] += 1.0  # entry (i, j) of head 1 no longer equals entry (j, i)
    with pytest.raises(ValueError):
        obj.loss_terms(np.zeros((g.n, 2)), g, "maxcut", None, 0.0, 2, 0.0, 0, None, ew)
