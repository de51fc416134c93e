"""Pins of the weighted-MIS objective (node weights per node or per head, the
tasks of the two-stage appendix) against networkx, brute force and finite
differences."""

import itertools

import networkx as nx
import numpy as np
import pytest

from oracle import evaluate, objective
from workloads import erdos_renyi_graph, random_regular_graph


def nx_graph(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    ei, ej, _ = g.edge_list()
    G.add_edges_from(zip(ei.tolist(), ej.tolist()))
    return G


@pytest.mark.parametrize("per_head", [False, True])
def test_weighted_relaxation_equals_discrete_networkx(per_head):
    g = erdos_renyi_graph(40, 0.15, 3)
    G = nx_graph(g)
    rng = np.random.default_rng(0)
    S = 6
    W = rng.uniform(0, 1, (g.n, S)) if per_head else rng.uniform(0, 1, g.n)
    X = (rng.random((g.n, S)) < 0.4).astype(np.float64)
    lam = rng.uniform(0.1, 5.0, S)
    ei, ej, w = objective.edges_of(g.row_ptr, g.col_idx, None)
    got = objective.relaxed_head_losses(X, ei, ej, w, "mis", lam, W)
    for s in range(S):
        chosen = [i for i in range(g.n) if X[i, s] == 1]
        ws = sum((W[i, s] if per_head else W[i]) for i in chosen)
        assert got[s] == pytest.approx(-ws + lam[s] * G.subgraph(chosen).number_of_edges(), abs=1e-12)
        assert got[s] == pytest.approx(objective.discrete_mis(X[:, s], ei, ej, w, lam[s],
                                                              W[:, s] if per_head else W), abs=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_penalty_minimisers_are_maximum_weight_independent_sets(seed):
    """lambda > max w: removing one endpoint of a violated edge always lowers the
    objective, so the brute-force minimiser is an independent set of maximum
    weight -- the weight networkx finds as a maximum-weight clique of the complement."""
    g = erdos_renyi_graph(12, 0.3, 10 + seed)
    rng = np.random.default_rng(seed)
    wi = rng.integers(1, 10, g.n)
    lam = float(wi.max()) + 0.5
    ei, ej, w = objective.edges_of(g.row_ptr, g.col_idx, None)
    best = min(objective.discrete_mis(np.array(x), ei, ej, w, lam, wi)
               for x in itertools.product([0, 1], repeat=g.n))
    C = nx.complement(nx_graph(g))
    nx.set_node_attributes(C, {i: int(wi[i]) for i in range(g.n)}, "w")
    _, mw = nx.max_weight_clique(C, weight="w")
    assert best == pytest.approx(-mw)


@pytest.mark.parametrize("per_head", [False, True])
def test_weighted_gradient_finite_differences(per_head):
    g = random_regular_graph(30, 3, 5)
    rng = np.random.default_rng(1)
    S = 5
    W = rng.uniform(0, 1, (g.n, S)) if per_head else rng.uniform(0, 1, g.n)
    lam = np.linspace(0.5, 3, S)
    Z = rng.standard_normal((g.n, S)) * 2
    gZ = objective.grad_wrt_Z(Z, g, "mis", lam, 0.3, 2, 0.1, 0, W)
    h = 1e-6
    D = rng.standard_normal(Z.shape)
    fp = objective.loss_terms(Z + h * D, g, "mis", lam, 0.3, 2, 0.1, 0, W)["total"]
    fm = objective.loss_terms(Z - h * D, g, "mis", lam, 0.3, 2, 0.1, 0, W)["total"]
    fd = (fp - fm) / (2 * h)
    assert abs(fd - np.sum(gZ * D)) <= 1e-7 * max(1.0, abs(fd))


def test_unit_weights_reduce_to_plain_mis():
    g = erdos_renyi_graph(50, 0.1, 7)
    Z = np.random.default_rng(2).standard_normal((g.n, 4))
    lam = np.array([0.5, 1, 2, 4.0])
    a = objective.loss_terms(Z, g, "mis", lam, 0.2, 2)
    b = objective.loss_terms(Z, g, "mis", lam, 0.2, 2, node_weight=np.ones(g.n))
    assert np.array_equal(a["head"], b["head"])


def test_evaluate_reports_set_weight():
    g = erdos_renyi_graph(30, 0.2, 9)
    rng = np.random.default_rng(3)
    W = rng.uniform(0, 1, (g.n, 3))
    X = (rng.random((g.n, 3)) < 0.5).astype(np.uint8)
    ev = evaluate.evaluate_one(X, g, "mis", W)
    for s in range(3):
        assert ev["weight"][s] == pytest.approx(sum(W[i, s] for i in range(g.n) if X[i, s]))


# ---------------------------------------------------------------------------
# Solution-diversity analytics (pairwise Hamming matrix, histogram, unique count)
def test_diversity_stats_against_brute_force_and_proposition_3_2():
    rng = np.random.default_rng(4)
    N, S = 37, 9
    X = (rng.random((N, S)) < 0.4).astype(np.uint8)
    X[:, 5] = X[:, 2]  # two duplicated solutions
    X[:, 7] = X[:, 2]
    st = evaluate.diversity_stats(X)
    for s in range(S):
        for l in range(S):
            assert st["D"][s, l] == int(np.sum(X[:, s] != X[:, l]))
    assert st["unique"] == S - 2
    # total over pairs = sum_i k_i (S - k_i) (Proposition 3.2's counting identity)
    k = X.astype(np.int64).sum(axis=1)
    assert st["hist"].dot(np.arange(N + 1)) == int(np.sum(k * (S - k)))
    assert st["hist"].sum() == S * (S - 1) // 2 and st["hist"][0] == 3  # pairs among {2, 5, 7}
