"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test ties an oracle function to something other than its own formula:
networkx's independent-set and cut computations, finite differences,
torch's autograd and optimizers on the CPU, brute-force enumeration, closed
forms on textbook graphs, Lemma A.1, Theorem 3.1, Proposition 3.2 and the
parameter counts printed in the paper's result tables.
"""

import json
import os

import networkx as nx
import numpy as np
import pytest
import torch

from oracle import evaluate, exact, gnn, objective, train
from workloads import csr_from_edges, erdos_renyi_graph, init_params, random_regular_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def nx_graph(g, weighted=False):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    ei, ej, w = g.edge_list()
    for k, (a, b) in enumerate(zip(ei, ej)):
        G.add_edge(int(a), int(b), weight=float(w[k]) if (weighted and w is not None) else 1.0)
    return G


def weighted_graph(n, p, seed):
    g = erdos_renyi_graph(n, p, seed)
    ei, ej, _ = g.edge_list()
    rng = np.random.default_rng(seed + 100)
    w = rng.uniform(0.5, 2.0, size=ei.size).astype(np.float32)
    return csr_from_edges(n, ei, ej, w)


# ---------------------------------------------------------------------------
# Relaxation exactness (Sec. 2.2): l_hat(x) = l(x) on {0,1}^N
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_relaxed_mis_equals_discrete_networkx(seed):
    g = erdos_renyi_graph(40, 0.15, seed)
    G = nx_graph(g)
    rng = np.random.default_rng(seed)
    S = 7
    X = (rng.random((g.n, S)) < 0.4).astype(np.float64)
    lam = rng.uniform(0.1, 5.0, size=S)
    ei, ej, w = objective.edges_of(g.row_ptr, g.col_idx, None)
    got = objective.relaxed_head_losses(X, ei, ej, w, "mis", lam)
    for s in range(S):
        chosen = [i for i in range(g.n) if X[i, s] == 1]
        inside = G.subgraph(chosen).number_of_edges()
        assert got[s] == pytest.approx(-len(chosen) + lam[s] * inside, abs=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_relaxed_maxcut_equals_negative_cut_networkx(seed):
    g = weighted_graph(30, 0.2, seed)
    G = nx_graph(g, weighted=True)
    rng = np.random.default_rng(seed)
    X = (rng.random((g.n, 5)) < 0.5).astype(np.float64)
    ei, ej, w = objective.edges_of(g.row_ptr, g.col_idx, g.weight)
    got = objective.relaxed_head_losses(X, ei, ej, w, "maxcut", None)
    for s in range(5):
        part = [i for i in range(g.n) if X[i, s] == 1]
        assert got[s] == pytest.approx(-nx.cut_size(G, part, weight="weight"), rel=1e-12)


def test_loss_terms_at_saturated_logits_are_integers():
    g = random_regular_graph(50, 3, 7)
    rng = np.random.default_rng(3)
    Z = np.where(rng.random((50, 6)) < 0.5, -60.0, 60.0)
    lam = np.arange(1, 7, dtype=np.float64)
    t = objective.loss_terms(Z, g, "mis", lam, gamma=0.7, alpha=2, nu=0.0)
    X = (Z > 0).astype(np.float64)
    G = nx_graph(g)
    for s in range(6):
        chosen = [i for i in range(50) if X[i, s]]
        assert t["head"][s] == -len(chosen) + lam[s] * G.subgraph(chosen).number_of_edges()
    # 1 - (2P-1)^2 = 4 sigma(60) sigma(-60) ~ 3.5e-26 per entry: tiny but not rounded away
    assert 0.0 < t["entropy"] < 300 * 4 * np.exp(-60.0) * 1.01


# ---------------------------------------------------------------------------
# Lemma A.1 and the annealing term
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [2, 4, 6])
def test_entropy_endpoints_lemma_a1(alpha):
    N, S = 13, 5
    half = np.full((N, S), 0.5)
    assert objective.entropy_term(half, 1 - half, alpha) == pytest.approx(N * S, abs=1e-12)
    rng = np.random.default_rng(alpha)
    X = (rng.random((N, S)) < 0.5).astype(np.float64)
    assert objective.entropy_term(X, 1 - X, alpha) == 0.0
    P = rng.random((N, S))
    phi = objective.one_minus_t_pow(P, 1 - P, alpha)
    assert np.all(phi >= 0) and np.all(phi <= 1)
    np.testing.assert_allclose(phi, 1 - (2 * P - 1) ** alpha, rtol=0, atol=1e-14)


def test_alpha_must_be_even():
    with pytest.raises(ValueError):
        objective.check_alpha(3)
    with pytest.raises(ValueError):
        objective.check_alpha(0)


# ---------------------------------------------------------------------------
# Proposition 3.2 and the diversity term
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_proposition_3_2_binary(seed):
    rng = np.random.default_rng(seed)
    N, S = 17, 9
    X = (rng.random((N, S)) < rng.uniform(0.1, 0.9)).astype(np.uint8)
    brute = sum(int(np.sum(X[:, s] != X[:, l])) for s in range(S) for l in range(s + 1, S))
    var = np.var(X.astype(np.float64), axis=1)  # population variance (Notation section)
    assert S * S * var.sum() == pytest.approx(brute, abs=1e-9)
    assert evaluate.pairwise_hamming_sum(X) == brute
    k = X.astype(np.int64).sum(axis=1)
    assert int(np.sum(k * (S - k))) == brute
    # Psi at a binary point: -S * sum_i sqrt(k_i (S - k_i)) / S
    psi = objective.diversity_term(X.astype(np.float64))
    assert psi == pytest.approx(-np.sum(np.sqrt(k * (S - k))), abs=1e-9)


def test_proposition_3_2_real_squared_form():
    rng = np.random.default_rng(9)
    P = rng.random((11, 6))
    lhs = 36 * np.sum(objective.row_std(P) ** 2)
    rhs = sum(np.sum((P[:, s] - P[:, l]) ** 2) for s in range(6) for l in range(s + 1, 6))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_std_matches_numpy_ddof():
    rng = np.random.default_rng(1)
    P = rng.random((20, 8))
    np.testing.assert_allclose(objective.row_std(P, 0), np.std(P, axis=1), rtol=1e-13)
    np.testing.assert_allclose(objective.row_std(P, 1), np.std(P, axis=1, ddof=1), rtol=1e-13)


def _psi_grad(P, ddof=0, nu=1.0):
    """nu * dPsi/dP alone: MaxCut on an edgeless graph at gamma = 0 has no other term."""
    from workloads import csr_from_edges
    N = P.shape[0]
    g = csr_from_edges(N, np.zeros(0, np.int64), np.zeros(0, np.int64))
    return objective.grad_wrt_P(P, 1.0 - P, g, "maxcut", None, 0.0, 2, nu, ddof)


@pytest.mark.parametrize("ddof", [0, 1])
def test_psi_gradient_sums_to_zero_over_heads(ddof):
    """sigma_i does not change when one constant is added to every head of node i,
    so every (sub)gradient of Psi sums to zero over the heads of each node."""
    rng = np.random.default_rng(11 + ddof)
    for S in (2, 3, 7, 32, 100):
        P = rng.random((40, S))
        P[::5] = P[::5, :1]  # every fifth row: all heads equal
        G = _psi_grad(P, ddof, nu=0.7)
        scale = np.abs(G).sum(axis=1)
        assert np.all(np.abs(G.sum(axis=1)) <= 1e-12 * np.maximum(scale, 1e-300))
        assert np.all(scale[1::5] > 0)  # the other rows do carry a gradient


@pytest.mark.parametrize("S", [3, 7, 100])
def test_psi_identical_heads_give_exact_zero(S):
    """Heads that coincide at a node: sigma_i = 0, Psi_i = 0 and dPsi_i = 0 exactly,
    for non-dyadic values whose rounded mean differs from the value itself."""
    rng = np.random.default_rng(S)
    vals = np.concatenate([[0.3, 0.1, 0.7, 1.0 / 3.0], rng.random(60)])
    P = np.repeat(vals[:, None], S, axis=1)
    mean_off = np.sum(P.sum(axis=1) / S != vals)
    assert mean_off > 0  # the two-pass mean alone would leave sigma > 0 on these rows
    for ddof in (0, 1):
        assert np.all(objective.row_std(P, ddof) == 0.0)
        assert objective.diversity_term(P, ddof) == 0.0
        assert np.all(_psi_grad(P, ddof) == 0.0)
    # the same rows among distinct ones: only the distinct rows move
    Q = np.vstack([P, rng.random((10, S))])
    G = _psi_grad(Q, 0)
    assert np.all(G[: vals.size] == 0.0) and np.all(np.abs(G[vals.size:]).sum(axis=1) > 0)
    np.testing.assert_allclose(objective.row_std(Q[vals.size:]), np.std(Q[vals.size:], axis=1),
                               rtol=1e-13)


def test_dscore_definition():
    X = np.array([[1, 0, 1], [0, 0, 1], [1, 1, 1], [0, 1, 0]], dtype=np.uint8)
    # columns 1010, 0011, 1110: d_H(0,1)=2, d_H(0,2)=1, d_H(1,2)=3 -> 6 ; DScore = 2*6/(4*3*2)
    assert evaluate.pairwise_hamming_sum(X) == 6
    assert evaluate.dscore(X) == pytest.approx(12 / 24)


# ---------------------------------------------------------------------------
# Gradients: finite differences and torch autograd
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("problem,alpha,nu,ddof,weighted", [
    ("mis", 2, 0.0, 0, False), ("mis", 4, 0.3, 0, False), ("maxcut", 2, 0.5, 0, True),
    ("maxcut", 6, 0.2, 1, False)])
def test_grad_wrt_Z_finite_differences(problem, alpha, nu, ddof, weighted):
    g = weighted_graph(25, 0.2, 4) if weighted else erdos_renyi_graph(25, 0.2, 4)
    rng = np.random.default_rng(5)
    S = 6
    Z = 1.5 * rng.standard_normal((g.n, S))
    lam = rng.uniform(0.2, 4, size=S)
    gamma = -0.7
    G = objective.grad_wrt_Z(Z, g, problem, lam, gamma, alpha, nu, ddof)
    f = lambda z: objective.loss_terms(z, g, problem, lam, gamma, alpha, nu, ddof)["total"]
    h = 1e-6
    for _ in range(5):
        D = rng.standard_normal(Z.shape)
        fd = (f(Z + h * D) - f(Z - h * D)) / (2 * h)
        an = float(np.sum(G * D))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))
    # single coordinates
    for (i, s) in [(0, 0), (3, 2), (g.n - 1, S - 1)]:
        E = np.zeros_like(Z)
        E[i, s] = 1
        fd = (f(Z + h * E) - f(Z - h * E)) / (2 * h)
        assert abs(fd - G[i, s]) <= 1e-6 * max(1.0, abs(G[i, s]))


def _torch_loss(Zt, g, problem, lam, gamma, alpha, nu, ddof):
    """The loss written directly in torch ops (dense adjacency), for autograd."""
    n = g.n
    A = torch.zeros((n, n), dtype=torch.float64)
    ei, ej, w = g.edge_list()
    wt = torch.ones(ei.size, dtype=torch.float64) if w is None else torch.tensor(w, dtype=torch.float64)
    A[torch.tensor(ei), torch.tensor(ej)] = wt
    A[torch.tensor(ej), torch.tensor(ei)] = wt
    P = torch.sigmoid(Zt)
    if problem == "mis":
        head = -P.sum(0) + torch.tensor(lam) * 0.5 * (P * (A @ P)).sum(0)
    else:
        head = (P * (A @ P)).sum(0) - (A.sum(1)[:, None] * P).sum(0)
    ent = (1 - (2 * P - 1) ** alpha).sum()
    psi = -P.shape[1] * torch.std(P, dim=1, correction=ddof).sum()
    return head.sum() + gamma * ent + nu * psi


@pytest.mark.parametrize("problem", ["mis", "maxcut"])
def test_grad_wrt_Z_matches_torch_autograd(problem):
    g = erdos_renyi_graph(30, 0.15, 8)
    rng = np.random.default_rng(2)
    Z = rng.standard_normal((30, 5))
    lam = rng.uniform(0.5, 3, size=5)
    Zt = torch.tensor(Z, requires_grad=True)
    _torch_loss(Zt, g, problem, lam, 0.4, 2, 0.25, 0).backward()
    G = objective.grad_wrt_Z(Z, g, problem, lam, 0.4, 2, 0.25, 0)
    np.testing.assert_allclose(G, Zt.grad.numpy(), rtol=1e-10, atol=1e-12)
    t = objective.loss_terms(Z, g, problem, lam, 0.4, 2, 0.25, 0)
    assert t["total"] == pytest.approx(float(_torch_loss(torch.tensor(Z), g, problem, lam, 0.4,
                                                          2, 0.25, 0)), rel=1e-12)


@pytest.mark.parametrize("kind,n_layers", [("gcn", 2), ("sage", 2), ("gcn", 3)])
def test_gnn_backward_finite_differences(kind, n_layers):
    g = erdos_renyi_graph(20, 0.2, 1)  # has isolated/low-degree nodes
    params = gnn.to_f64(init_params(kind, g.n, n_layers, 6, 4, seed=3))
    if kind == "sage":
        for L in params["layers"]:
            L["b"] = np.random.default_rng(0).standard_normal(L["b"].shape) * 0.1
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    rng = np.random.default_rng(4)
    W = rng.standard_normal((g.n, 4))  # loss = sum(W * Z), so dZ = W

    def loss(p):
        Z, _ = gnn.forward(p, M)
        return float(np.sum(W * Z))

    Z, cache = gnn.forward(params, M)
    grads = gnn.backward(params, M, cache, W)

    def leaves(p):
        yield ("emb",), p["emb"]
        for k, L in enumerate(p["layers"]):
            for name in L:
                yield ("layers", k, name), L[name]

    h = 1e-6
    for key, arr in leaves(params):
        gk = grads["emb"] if key == ("emb",) else grads["layers"][key[1]][key[2]]
        D = rng.standard_normal(arr.shape)
        arr += h * D
        fp = loss(params)
        arr -= 2 * h * D
        fm = loss(params)
        arr += h * D
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(gk * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), key


def test_gnn_forward_matches_torch_dense():
    g = random_regular_graph(24, 3, 2)
    p32 = init_params("sage", g.n, 2, 8, 3, seed=5)
    params = gnn.to_f64(p32)
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    Z, _ = gnn.forward(params, M)
    A = torch.zeros((g.n, g.n), dtype=torch.float64)
    ei, ej, _ = g.edge_list()
    A[torch.tensor(ei), torch.tensor(ej)] = 1
    A[torch.tensor(ej), torch.tensor(ei)] = 1
    H = torch.tensor(params["emb"])
    for k, L in enumerate(params["layers"]):
        lin_n = torch.nn.Linear(8, L["Wn"].shape[0], bias=True, dtype=torch.float64)
        lin_s = torch.nn.Linear(8, L["Ws"].shape[0], bias=False, dtype=torch.float64)
        with torch.no_grad():
            lin_n.weight.copy_(torch.tensor(L["Wn"]))
            lin_n.bias.copy_(torch.tensor(L["b"]))
            lin_s.weight.copy_(torch.tensor(L["Ws"]))
        meanH = (A @ H) / A.sum(1, keepdim=True)
        H = lin_n(meanH) + lin_s(H)
        if k == 0:
            H = torch.relu(H)
    np.testing.assert_allclose(Z, H.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_gnn_permutation_equivariance():
    g = erdos_renyi_graph(30, 0.2, 6)
    params = gnn.to_f64(init_params("gcn", g.n, 2, 5, 3, seed=1))
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    Z, _ = gnn.forward(params, M)
    perm = np.random.default_rng(0).permutation(g.n)
    inv = np.argsort(perm)
    ei, ej, _ = g.edge_list()
    gp = csr_from_edges(g.n, inv[ei], inv[ej])  # node v becomes inv[v]
    pp = {"emb": params["emb"][perm], "layers": params["layers"]}
    Zp, _ = gnn.forward(pp, gnn.mean_aggregation_matrix(gp.row_ptr, gp.col_idx))
    np.testing.assert_allclose(Zp, Z[perm], rtol=1e-12, atol=1e-13)


def test_gnn_edgeless_graph_is_mlp():
    g = csr_from_edges(6, np.zeros(0, np.int64), np.zeros(0, np.int64))
    params = gnn.to_f64(init_params("gcn", 6, 2, 4, 2, seed=2))
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    Z, _ = gnn.forward(params, M)
    L1, L2 = params["layers"]
    ref = np.maximum(params["emb"] @ L1["Ws"].T, 0) @ L2["Ws"].T
    np.testing.assert_allclose(Z, ref, rtol=1e-13)


# ---------------------------------------------------------------------------
# Parameter counts printed in the result tables
# ---------------------------------------------------------------------------

def test_param_count_identities_from_paper_tables():
    with open(os.path.join(GOLDEN, "param_counts.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        H0, S = c["H0"], c["S"]
        assert gnn.param_count("sage", [(H0, H0), (H0, S)]) == c["params"], c
    # The oracle's forward consumes exactly these arrays (embedding excluded).
    p = init_params("sage", 10, 2, 12, 3, seed=0)
    n = sum(a.size for L in p["layers"] for a in L.values())
    assert n == gnn.param_count("sage", [(12, 12), (12, 3)])


# ---------------------------------------------------------------------------
# Theorem 3.1 limits
# ---------------------------------------------------------------------------

def _descend_in_P(P0, g, lam, gamma, steps=4000, lr=1e-3):
    """Projected gradient descent on R(P) directly (no GNN), P kept in [0, 1]."""
    P = P0.copy()
    for _ in range(steps):
        G = objective.grad_wrt_P(P, 1 - P, g, "mis", lam, gamma, 2)
        P = np.clip(P - lr * G, 0.0, 1.0)
    return P


def test_theorem_3_1_gamma_to_minus_infinity_gives_half():
    g = random_regular_graph(10, 3, 0)
    lam = np.array([0.5, 2.0, 4.0])
    rng = np.random.default_rng(0)
    ends = [_descend_in_P(rng.random((10, 3)), g, lam, gamma=-1e4, steps=300, lr=1e-6)
            for _ in range(3)]
    for P in ends:
        assert np.max(np.abs(P - 0.5)) < 1e-3
    assert np.max(np.abs(ends[0] - ends[1])) < 1e-9


def test_theorem_3_1_gamma_to_plus_infinity_gives_binary_optima():
    g = random_regular_graph(8, 3, 1)
    lam = np.array([2.0])
    best, _ = exact.bruteforce_min(g, "mis", lam=2.0)
    rng = np.random.default_rng(1)
    vals = []
    for _ in range(30):
        P = _descend_in_P(rng.random((8, 1)), g, lam, gamma=20.0, steps=400, lr=1e-2)
        assert objective.entropy_term(P, 1 - P, 2) < 1e-9  # every limit is a vertex
        ei, ej, w = objective.edges_of(g.row_ptr, g.col_idx, None)
        vals.append(objective.relaxed_head_losses(P, ei, ej, w, "mis", lam)[0])
    assert min(vals) == pytest.approx(best)


# ---------------------------------------------------------------------------
# Exact solvers on textbook graphs; penalty argmin = maximum independent sets
# ---------------------------------------------------------------------------

def _cycle(n):
    return csr_from_edges(n, np.arange(n), (np.arange(n) + 1) % n)


def _complete(n):
    iu = np.triu_indices(n, 1)
    return csr_from_edges(n, iu[0], iu[1])


def _from_nx(G):
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(G.number_of_nodes(), e[:, 0], e[:, 1])


def test_textbook_independence_numbers():
    for n in (5, 6, 9):
        assert exact.mis_size_bruteforce(_cycle(n)) == n // 2
        assert exact.mis_size_milp(_cycle(n)) == n // 2
    assert exact.mis_size_bruteforce(_complete(7)) == 1
    assert exact.mis_size_bruteforce(_from_nx(nx.petersen_graph())) == 4
    assert exact.mis_size_bruteforce(_from_nx(nx.complete_bipartite_graph(3, 5))) == 5
    empty = csr_from_edges(6, np.zeros(0, np.int64), np.zeros(0, np.int64))
    assert exact.mis_size_bruteforce(empty) == 6


def test_textbook_maxcuts():
    assert exact.maxcut_bruteforce(_cycle(7)) == 6
    assert exact.maxcut_bruteforce(_cycle(8)) == 8
    assert exact.maxcut_bruteforce(_complete(7)) == 49 // 4
    kb = nx.complete_bipartite_graph(3, 4)
    assert exact.maxcut_bruteforce(_from_nx(kb)) == kb.number_of_edges()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_penalty_minimisers_are_maximum_independent_sets(seed):
    g = random_regular_graph(14, 3, seed)
    G = nx_graph(g)
    alpha_nx = len(nx.max_weight_clique(nx.complement(G), weight=None)[0])
    best, argmins = exact.bruteforce_min(g, "mis", lam=2.0)
    assert best == -alpha_nx
    for code in argmins:
        x = exact.code_to_x(int(code), g.n)
        chosen = [i for i in range(g.n) if x[i]]
        assert G.subgraph(chosen).number_of_edges() == 0 and len(chosen) == alpha_nx
    assert exact.mis_size_milp(g) == alpha_nx


# ---------------------------------------------------------------------------
# Evaluation, rounding, optimizer, schedule
# ---------------------------------------------------------------------------

def test_rounding_tie_goes_to_zero():
    Z = np.array([[0.0, -0.0, 1e-300, -1e-300, 3.0]])
    assert evaluate.round_solutions(Z).tolist() == [[0, 0, 1, 0, 1]]


def test_rounding_matches_exact_sigmoid_threshold():
    """x = [sigmoid(z) > 1/2] decided in exact decimal arithmetic (2,000 digits,
    enough to hold 1 - 2^-1074 exactly) for logits at and around the tie,
    subnormals included: the rule P <= 0.5 -> 0, P > 0.5 -> 1 of the
    training-setting appendix, with sigmoid evaluated without rounding."""
    from decimal import Decimal, localcontext
    zs = [0.0, -0.0, 5e-324, -5e-324, 1e-320, 1e-300, -1e-300, 1e-20, 1e-17, 1e-16, 1.1e-16,
          2.3e-16, -2.3e-16, 1e-8, -1e-8, 0.5, -7.0, 40.0]
    with localcontext() as ctx:
        ctx.prec = 2000
        exact = [int(Decimal(1) / (1 + (-Decimal(z)).exp()) > Decimal("0.5")) for z in zs]
    got = evaluate.round_solutions(np.array([zs])).tolist()[0]
    assert got == exact
    assert exact[:4] == [0, 0, 1, 0]


def test_evaluate_against_networkx():
    g = erdos_renyi_graph(60, 0.08, 3)
    G = nx_graph(g)
    rng = np.random.default_rng(0)
    X = (rng.random((60, 4)) < 0.3).astype(np.uint8)
    ev = evaluate.evaluate(X, g, "mis")[0]
    ev_c = evaluate.evaluate(X, g, "maxcut")[0]
    for s in range(4):
        chosen = [i for i in range(60) if X[i, s]]
        assert ev["size"][s] == len(chosen)
        assert ev["violations"][s] == G.subgraph(chosen).number_of_edges()
        assert ev_c["cut_edges"][s] == nx.cut_size(G, chosen)


@pytest.mark.parametrize("wd", [0.0, 1e-2])
def test_adam_matches_torch_optim(wd):
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tt = torch.tensor(theta.copy(), requires_grad=True)
    cls = torch.optim.AdamW if wd else torch.optim.Adam
    opt = cls([tt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    for t in range(1, 8):
        g = rng.standard_normal(50)
        train.adam_update(theta, g, m, v, t, 1e-2, weight_decay=wd)
        opt.zero_grad()
        tt.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(theta, tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_first_adam_step_moves_by_lr_times_sign():
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.3, -5.0, 1e-3])
    train.adam_update(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    np.testing.assert_allclose(theta, [0.9, -1.9, 2.9], atol=1e-6)


def test_early_stop_rule_special_cases():
    """The stopping rule on sequences whose answer is fixed by hand: constant
    values stall from step 1 on; a loss that keeps falling by more than the
    tolerance never stops; a fall inside the tolerance, or any rise, counts as
    stalled; one monitored value falling is enough to reset the count."""
    es = lambda h, p, tol, pat: train.early_stop_step(h, p, tol, pat, relative=True)  # noqa: E731
    const = [5.0] * 30
    assert es(const, const, 1e-5, 10) == 10
    assert es(const, const, 1e-5, 1) == 1
    assert es(const[:10], const[:10], 1e-5, 10) is None
    falling = [100.0 * 0.99 ** t for t in range(200)]  # 1% per step > tol
    flat = [5.0] * len(falling)
    assert es(falling, flat, 1e-3, 5) is None
    assert es(flat, falling, 1e-3, 5) is None
    slow = [100.0 * (1 - 1e-6) ** t for t in range(50)]  # falls by 1e-6 < tol = 1e-5
    assert es(slow, slow, 1e-5, 20) == 20
    rising = [float(t) for t in range(50)]
    assert es(rising, rising, 0.0, 3) == 3
    # steps 1-5 stall, the loss falls at step 6 (reset), steps 7-12 stall: fires at 12
    L = [1.0] * 6 + [0.5] * 30
    assert es(L, [2.0] * 36, 1e-5, 6) == 12
    assert es(L, [2.0] * 36, 1e-5, 5) == 5
    # negative values: "falling" means moving towards -inf
    neg = [-1.0 - 0.01 * t for t in range(40)]
    assert es(neg, [-3.0] * 40, 1e-3, 4) is None
    assert es([-1.0] * 40, [-3.0] * 40, 1e-3, 4) == 4


def test_early_stop_rule_absolute_tolerance():
    """The paper's plain (absolute) tolerance: a fall of 1e-6 per step is within a
    tolerance of 1e-5 whatever the values' magnitude; 1e-4 is not; and a value
    that decays towards 0 geometrically stalls once its steps drop below tol."""
    es = train.early_stop_step
    small_fall = [1e6 - 1e-6 * t for t in range(40)]
    big_fall = [1.0 - 1e-4 * t for t in range(40)]
    flat = [0.0] * 40
    assert es(small_fall, flat, 1e-5, 10) == 10
    assert es(big_fall, flat, 1e-5, 10) is None
    decay = [0.5 ** t for t in range(60)]  # step t falls by 0.5^t: <= 1e-5 from t = 17 on
    first = next(t for t in range(1, 60) if decay[t - 1] - decay[t] <= 1e-5)
    assert first == 17
    assert es(flat, decay, 1e-5, 8) == first + 7
    assert es(flat, decay, 1e-5, 8, relative=True) is None  # halves every step: never stalls


def test_gamma_schedule_endpoints():
    assert train.gamma_at(0, 2000, -2.0, 0.1) == -2.0
    assert train.gamma_at(1999, 2000, -2.0, 0.1) == pytest.approx(0.1)
    assert train.gamma_at(1, 2000, -2.0, 0.1) - train.gamma_at(0, 2000, -2.0, 0.1) == \
        pytest.approx(2.1 / 1999)
    assert train.gamma_paper(1000, -20.0, 1e-3) == pytest.approx(-19.0)


def test_batched_terms_equal_per_graph_terms():
    from workloads import disjoint_union
    gs = [erdos_renyi_graph(20, 0.2, 1), erdos_renyi_graph(15, 0.3, 2), random_regular_graph(12, 3, 3)]
    u = disjoint_union(gs)
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((u.n, 4))
    bt = objective.batched_loss_terms(Z, u, "maxcut", None, 0.3, 2, 0.1)
    off = 0
    for g, t in zip(gs, bt):
        ref = objective.loss_terms(Z[off:off + g.n], g, "maxcut", None, 0.3, 2, 0.1)
        np.testing.assert_allclose(t["head"], ref["head"], rtol=1e-13)
        assert t["psi"] == pytest.approx(ref["psi"], rel=1e-13)
        off += g.n
