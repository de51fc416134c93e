"""Pins of the warm-start oracle (oracle/warmstart.py) against facts that do
not come from its own formulas: torch's float32 -> bfloat16 conversion,
networkx's triangle counts and clustering coefficients, closed forms on
textbook graphs, a dense torch implementation of the network with torch's
own bfloat16 rounding, torch autograd, and central finite differences."""

import networkx as nx
import numpy as np
import pytest
import torch

from oracle import gnn, objective
from oracle import warmstart as W
from workloads import (csr_from_edges, erdos_renyi_graph, init_mpnn_params, random_channels,
                       random_regular_graph)


def nx_graph(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    ei, ej, _ = g.edge_list()
    G.add_edges_from(zip(ei.tolist(), ej.tolist()))
    return G


def graph_from_nx(G):
    n = G.number_of_nodes()
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(n, e[:, 0], e[:, 1])


# ------------------------------------------------------------------ bfloat16
def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        rng.uniform(-1, 1, 5000), [0.0, -0.0, 1.0, -2.5, 3e38, 1e-40]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = W.bf16_round(x)
    assert np.array_equal(got, ref)
    bits = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy() \
        .astype(np.uint16)
    assert np.array_equal(W.bf16_bits(x), bits)
    assert np.array_equal(W.from_bf16_bits(bits), ref)


def test_bf16_ties_round_to_even():
    # 8 significant bits: the spacing just above 1 is 2^-7
    assert W.bf16_round(1.0 + 2.0 ** -8)[()] == 1.0                      # tie -> even (1.0)
    assert W.bf16_round(1.0 + 3 * 2.0 ** -8)[()] == 1.0 + 2.0 ** -6      # tie -> even (up)
    assert W.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20)[()] == 1.0 + 2.0 ** -7
    assert W.bf16_round(-(1.0 + 2.0 ** -8))[()] == -1.0
    assert np.array_equal(W.bf16_round(W.bf16_round([0.1, 0.3, 7.77])), W.bf16_round([0.1, 0.3, 7.77]))


# ------------------------------------------------------------------ features
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_triangles_and_clustering_match_networkx(seed):
    g = erdos_renyi_graph(60, 0.2, seed)
    G = nx_graph(g)
    tri = W.triangles(g.row_ptr, g.col_idx)
    assert tri.dtype == np.int64
    assert [int(t) for t in tri] == [nx.triangles(G, i) for i in range(g.n)]
    c = W.clustering(g.degrees(), tri)
    ref = nx.clustering(G)
    assert np.allclose(c, [ref[i] for i in range(g.n)], rtol=0, atol=1e-15)


def test_triangles_closed_forms():
    cases = [
        (nx.complete_graph(6), lambda i: 10),                      # C(5, 2)
        (nx.cycle_graph(7), lambda i: 0),
        (nx.petersen_graph(), lambda i: 0),                        # girth 5
        (nx.complete_bipartite_graph(3, 3), lambda i: 0),
        (nx.wheel_graph(9), lambda i: 8 if i == 0 else 2),         # hub + 8-cycle rim
    ]
    for G, expect in cases:
        g = graph_from_nx(G)
        tri = W.triangles(g.row_ptr, g.col_idx)
        assert [int(t) for t in tri] == [expect(i) for i in range(g.n)]
        # sum_i T_i = 3 x (number of triangles) = trace(A^3) / 2
        A = nx.to_numpy_array(G, nodelist=range(g.n))
        assert int(tri.sum()) == int(round(np.trace(A @ A @ A) / 2))


def test_clustering_closed_forms():
    g = graph_from_nx(nx.wheel_graph(9))
    c = W.clustering(g.degrees(), W.triangles(g.row_ptr, g.col_idx))
    assert c[0] == pytest.approx(2 * 8 / (8 * 7))
    assert np.allclose(c[1:], 2 * 2 / (3 * 2))
    star = graph_from_nx(nx.star_graph(5))
    assert np.all(W.clustering(star.degrees(), W.triangles(star.row_ptr, star.col_idx)) == 0)
    k5 = graph_from_nx(nx.complete_graph(5))
    assert np.all(W.clustering(k5.degrees(), W.triangles(k5.row_ptr, k5.col_idx)) == 1.0)


def test_node_features_layout():
    g = erdos_renyi_graph(50, 0.15, 4)
    r = random_channels(g.n, 5, seed=1)
    feat, tri = W.node_features(g, r, 16)
    deg = g.degrees()
    G = nx_graph(g)
    cl = nx.clustering(G)
    # column 0: degree / 16 (exact); column 1: clustering in bf16; 2..6: channels; rest 0
    assert np.array_equal(feat[:, 0], deg / 16.0)
    ref_c = torch.tensor([cl[i] for i in range(g.n)], dtype=torch.float64).to(torch.float32) \
        .to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(feat[:, 1], ref_c)
    assert np.array_equal(feat[:, 2:7], torch.tensor(r).to(torch.bfloat16).to(torch.float64).numpy())
    assert np.all(feat[:, 7:] == 0)
    assert [int(t) for t in tri] == [nx.triangles(G, i) for i in range(g.n)]


# ------------------------------------------------------------------ network
def _torch_mpnn(params, feat, g, bf16):
    """Dense torch implementation with torch's own bfloat16 rounding."""
    A = torch.tensor(nx.to_numpy_array(nx_graph(g), nodelist=range(g.n)), dtype=torch.float64)
    deg = A.sum(1, keepdim=True)
    Mt = torch.where(deg > 0, A / deg.clamp(min=1), torch.zeros_like(A))
    r = (lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64)) if bf16 else (lambda t: t)
    H = r(torch.tensor(feat, dtype=torch.float64))
    L = params["layers"]
    for k, layer in enumerate(L):
        Ws = r(torch.tensor(layer["Ws"], dtype=torch.float64))
        Wn = r(torch.tensor(layer["Wn"], dtype=torch.float64))
        Ag = r(Mt @ H)
        Y = H @ Ws.T + Ag @ Wn.T + torch.tensor(layer["b"], dtype=torch.float64)
        H = r(torch.relu(Y)) if k < len(L) - 1 else Y
    return H


@pytest.mark.parametrize("bf16", [False, True])
def test_mpnn_forward_matches_dense_torch(bf16):
    g = erdos_renyi_graph(70, 0.08, 5)
    p = init_mpnn_params(16, 32, 8, 3, seed=2)
    for L in p["layers"]:
        L["b"][:] = np.random.default_rng(3).uniform(-0.2, 0.2, L["b"].shape)
    feat, _ = W.node_features(g, random_channels(g.n, 14, seed=3), 16)
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    Z, cache = W.mpnn_forward(p, feat, M, bf16=bf16)
    ref = _torch_mpnn(p, feat, g, bf16).numpy()
    # identical rounding points; the only differences are float64 summation order
    # (and, with bf16, a value pushed across a rounding boundary by it -- none here)
    assert np.allclose(Z, ref, rtol=1e-12, atol=1e-12)
    if bf16:
        for c in cache:
            for key in ("H", "A", "Ws", "Wn"):
                assert np.array_equal(W.bf16_round(c[key]), c[key])


def test_mpnn_backward_matches_torch_autograd_exact_mode():
    g = erdos_renyi_graph(40, 0.1, 6)
    p = init_mpnn_params(16, 32, 8, 3, seed=4)
    feat, _ = W.node_features(g, random_channels(g.n, 14, seed=5), 16)
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    dZ = np.random.default_rng(7).standard_normal((g.n, 8))
    Z, cache = W.mpnn_forward(p, feat, M, bf16=False)
    grads = W.mpnn_backward(cache, M, dZ, bf16=False)
    tp = [{k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in L.items()}
          for L in p["layers"]]
    A = torch.tensor(nx.to_numpy_array(nx_graph(g), nodelist=range(g.n)), dtype=torch.float64)
    deg = A.sum(1, keepdim=True)
    Mt = torch.where(deg > 0, A / deg.clamp(min=1), torch.zeros_like(A))
    H = torch.tensor(feat)
    for k, L in enumerate(tp):
        Y = H @ L["Ws"].T + (Mt @ H) @ L["Wn"].T + L["b"]
        H = torch.relu(Y) if k < len(tp) - 1 else Y
    (H * torch.tensor(dZ)).sum().backward()
    for k, L in enumerate(tp):
        for key in ("Ws", "Wn", "b"):
            assert np.allclose(grads["layers"][k][key], L[key].grad.numpy(), rtol=1e-10, atol=1e-12)


def test_mpnn_backward_finite_differences_exact_mode():
    g = random_regular_graph(30, 3, seed=8)
    p = {"layers": [{k: v.astype(np.float64) for k, v in L.items()}
                    for L in init_mpnn_params(16, 32, 8, 3, seed=6)["layers"]]}
    feat, _ = W.node_features(g, random_channels(g.n, 14, seed=9), 16)
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    dZ = np.random.default_rng(1).standard_normal((g.n, 8))
    _, cache = W.mpnn_forward(p, feat, M, bf16=False)
    grads = W.mpnn_backward(cache, M, dZ, bf16=False)
    rng = np.random.default_rng(2)
    h = 1e-7
    for k in range(3):
        for key in ("Ws", "Wn", "b"):
            arr = p["layers"][k][key]
            D = rng.standard_normal(arr.shape)
            arr += h * D
            fp = np.sum(W.mpnn_forward(p, feat, M, bf16=False)[0] * dZ)
            arr -= 2 * h * D
            fm = np.sum(W.mpnn_forward(p, feat, M, bf16=False)[0] * dZ)
            arr += h * D
            fd = (fp - fm) / (2 * h)
            an = np.sum(grads["layers"][k][key] * D)
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, key, fd, an)


def test_mpnn_single_layer_is_neighbour_mean():
    # Ws = 0, Wn = I, b = 0: Z = M X, the per-node mean of the neighbours' rows
    g = erdos_renyi_graph(25, 0.2, 11)
    X = np.random.default_rng(0).standard_normal((g.n, 16))
    p = {"layers": [{"Ws": np.zeros((16, 16)), "Wn": np.eye(16), "b": np.zeros(16)}]}
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    Z, _ = W.mpnn_forward(p, X, M, bf16=False)
    for i in range(g.n):
        nb = g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]
        ref = X[nb].mean(axis=0) if nb.size else np.zeros(16)
        assert np.allclose(Z[i], ref, rtol=1e-13, atol=1e-14)


def test_mpnn_permutation_equivariance():
    g = erdos_renyi_graph(40, 0.12, 12)
    perm = np.random.default_rng(3).permutation(g.n)
    inv = np.argsort(perm)
    ei, ej, _ = g.edge_list()
    gp = csr_from_edges(g.n, inv[ei], inv[ej])
    p = init_mpnn_params(16, 32, 8, 3, seed=7)
    feat, _ = W.node_features(g, random_channels(g.n, 14, seed=1), 16)
    featp, _ = W.node_features(gp, random_channels(g.n, 14, seed=1)[perm], 16)
    Z, _ = W.mpnn_forward(p, feat, gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx))
    Zp, _ = W.mpnn_forward(p, featp, gnn.mean_aggregation_matrix(gp.row_ptr, gp.col_idx))
    assert np.allclose(Zp, Z[perm], rtol=1e-12, atol=1e-12)


def test_bce_gradient_finite_differences():
    rng = np.random.default_rng(4)
    Z = rng.standard_normal((20, 6)) * 3
    X = (rng.random((20, 6)) < 0.4).astype(np.float64)
    g = W.bce_grad(Z, X, 0.7)
    h = 1e-6
    D = rng.standard_normal(Z.shape)
    fd = (W.bce_value(Z + h * D, X, 0.7) - W.bce_value(Z - h * D, X, 0.7)) / (2 * h)
    assert abs(fd - np.sum(g * D)) <= 1e-8 * max(1.0, abs(fd))
    # BCE against the textbook -[x log p + (1-x) log(1-p)]
    P = 1 / (1 + np.exp(-Z))
    ref = -np.sum(X * np.log(P) + (1 - X) * np.log(1 - P))
    assert W.bce_value(Z, X, 1.0) == pytest.approx(ref, rel=1e-12)


def test_warm_training_gradient_finite_differences_exact_mode():
    g = random_regular_graph(40, 3, seed=13)
    S = 8
    p = {"layers": [{k: v.astype(np.float64) for k, v in L.items()}
                    for L in init_mpnn_params(16, 32, S, 3, seed=8)["layers"]]}
    feat, _ = W.node_features(g, random_channels(g.n, 14, seed=2), 16)
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    lam = np.logspace(-1, 1, S)
    X = (np.random.default_rng(5).random((g.n, S)) < 0.4).astype(np.float64)
    gamma, beta = 0.05, 0.3

    def total(pp):
        Z, _ = W.mpnn_forward(pp, feat, M, bf16=False)
        return objective.loss_terms(Z, g, "mis", lam, gamma, 2)["total"] + W.bce_value(Z, X, beta)

    _, _, _, grads = W.warm_loss_and_grads(p, feat, M, g, "mis", lam, gamma, X, beta, bf16=False)
    rng = np.random.default_rng(6)
    h = 1e-7
    for k in range(3):
        for key in ("Ws", "Wn", "b"):
            arr = p["layers"][k][key]
            D = rng.standard_normal(arr.shape)
            arr += h * D
            fp = total(p)
            arr -= 2 * h * D
            fm = total(p)
            arr += h * D
            fd = (fp - fm) / (2 * h)
            an = np.sum(grads["layers"][k][key] * D)
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, key, fd, an)


def test_z_offset_shifts_the_logits_and_keeps_gradients_exact():
    from oracle import train
    from workloads import init_params
    g = random_regular_graph(30, 3, seed=3)
    S = 6
    p = gnn.to_f64(init_params("gcn", g.n, 2, 8, S, seed=1))
    M = gnn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    off = np.random.default_rng(0).standard_normal((g.n, S)) * 2
    Z0, _ = gnn.forward(p, M)
    Z1, _ = gnn.forward(p, M, off)
    assert np.array_equal(Z1, Z0 + off)
    cfg = train.StepConfig(problem="mis", lam=np.linspace(0.5, 3, S))
    _, terms, _, grads = train.loss_and_grads(p, M, g, cfg, 0.1, z_offset=off)
    rng = np.random.default_rng(1)
    h = 1e-7
    for key in ("Ws", "Wn"):
        arr = p["layers"][1][key]
        D = rng.standard_normal(arr.shape)
        arr += h * D
        fp = train.loss_and_grads(p, M, g, cfg, 0.1, z_offset=off)[1][0]["total"]
        arr -= 2 * h * D
        fm = train.loss_and_grads(p, M, g, cfg, 0.1, z_offset=off)[1][0]["total"]
        arr += h * D
        fd = (fp - fm) / (2 * h)
        assert abs(fd - np.sum(grads["layers"][1][key] * D)) <= 1e-6 * max(1.0, abs(fd))
