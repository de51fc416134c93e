"""Learned warm start for CPRA, in float64.  TEST INFRASTRUCTURE ONLY.

The paper's background section describes a family of learned solvers that
train one network over many instances and use it on a new instance, and a
meta-learned initialisation for new instances (paragraph on learning
generalized heuristics from data).  The warm start here is that idea applied
to CPRA's own outputs: a small message-passing network (the GraphSAGE form of
the GNN appendix, with a bias) maps per-node features to S logits Z_w, and
CPRA then trains on P = sigmoid(GNN_theta(G) + Z_w).

Features of node i (all stored in bfloat16):
  f_0 = d_i / 16                       (degree, an exact scaling)
  f_1 = c_i = 2 T_i / (d_i (d_i - 1))  (local clustering; 0 when d_i < 2)
  f_2 .. f_{1+R} = given random channels (they break the symmetry of
                   regular graphs, on which degree and clustering are constant)
  remaining columns up to in_dim = 0
T_i is the number of triangles through i: pairs of neighbours of i that are
themselves adjacent.  c_i is formed in float64, rounded to float32 and then to
bfloat16.

Network (n_layers layers, widths in_dim -> hidden -> ... -> S):
  A_k = bf16(M H_{k-1})                            mean over neighbours
  Y_k = H_{k-1} bf16(Ws_k)^T + A_k bf16(Wn_k)^T + b_k
  H_k = bf16(relu(Y_k)) for hidden layers;  Z_w = Y_L (float32 on the device)
Weights are kept in float32 and rounded to bfloat16 for every forward; the
bias stays in float32.  Each bf16(.) above is a point where the device stores
a bfloat16 tensor; the oracle rounds at exactly those points so that the two
differ only by the order of float32 versus float64 sums (and the rare value
that this difference moves across a bfloat16 rounding boundary).

Backward (upstream gradient dZ_w):
  dY_L = bf16(dZ_w)
  dWs_k = dY_k^T H_{k-1},  dWn_k = dY_k^T A_k,  db_k = sum over rows of dY_k
  G = dY_k [bf16(Ws_k) | bf16(Wn_k)]   (float32)
  dY_{k-1} = bf16((G_s + M^T G_n) * [H_{k-1} > 0])

Training objective on a graph with a converged CPRA solution X* [N, S]:
  the CPRA loss of P = sigmoid(Z_w) (``objective.loss_terms`` at a fixed gamma)
  + beta * sum_{i,s} BCE(sigmoid(Z_w[i,s]), X*[i,s])
whose gradient in Z_w is the CPRA gradient + beta * (sigmoid(Z_w) - X*).
"""

from __future__ import annotations

from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp

from . import objective


# ---------------------------------------------------------------- bfloat16
def bf16_round(x) -> np.ndarray:
    """Round to float32 (nearest even), then keep the top 16 bits of the float32
    pattern with round-to-nearest-even on the dropped 16 bits.  Returns float64
    values that are exactly representable in bfloat16.  (Finite inputs; a value
    that rounds past the largest bfloat16 becomes inf.)"""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """The uint16 bit patterns of bf16_round(x)."""
    f = bf16_round(x).astype(np.float32)
    return (f.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32) \
        .astype(np.float64)


# ---------------------------------------------------------------- features
def adjacency(row_ptr, col_idx) -> sp.csr_matrix:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = row_ptr.size - 1
    nnz = int(row_ptr[-1])
    return sp.csr_matrix((np.ones(nnz, dtype=np.int64), np.asarray(col_idx, dtype=np.int64),
                          row_ptr), shape=(n, n))


def triangles(row_ptr, col_idx) -> np.ndarray:
    """T_i = (1/2) sum_j A_ij (A^2)_ij: each triangle {i, j, k} is seen from i
    once through j and once through k."""
    A = adjacency(row_ptr, col_idx)
    A2 = A @ A
    twice = np.asarray(A.multiply(A2).sum(axis=1)).ravel().astype(np.int64)
    return twice // 2


def clustering(deg: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """c_i = 2 T_i / (d_i (d_i - 1)) in float64; 0 where d_i < 2."""
    deg = np.asarray(deg, dtype=np.float64)
    den = deg * (deg - 1.0)
    return np.divide(2.0 * np.asarray(tri, dtype=np.float64), den, out=np.zeros_like(den),
                     where=den > 0)


def node_features(graph, rand: Optional[np.ndarray], in_dim: int):
    """(features [N, in_dim] as bf16 values in float64, triangles int64 [N])."""
    n = graph.n
    R = 0 if rand is None else rand.shape[1]
    if 2 + R > in_dim:
        raise ValueError("in_dim too small for 2 + random channels")
    deg = np.diff(np.asarray(graph.row_ptr, dtype=np.int64))
    tri = triangles(graph.row_ptr, graph.col_idx)
    feat = np.zeros((n, in_dim))
    feat[:, 0] = bf16_round(deg.astype(np.float64) / 16.0)
    feat[:, 1] = bf16_round(clustering(deg, tri).astype(np.float32))
    if R:
        feat[:, 2:2 + R] = bf16_round(np.asarray(rand, dtype=np.float32))
    return feat, tri


# ---------------------------------------------------------------- network
def mpnn_dims(in_dim: int, hidden: int, S: int, n_layers: int):
    dims = []
    d = in_dim
    for k in range(n_layers):
        out = S if k == n_layers - 1 else hidden
        dims.append((d, out))
        d = out
    return dims


def mpnn_forward(params: Dict[str, object], feat: np.ndarray, M: sp.csr_matrix,
                 bf16: bool = True):
    """Z_w and the cache for the backward.  bf16=False: exact float64 (no
    rounding points), for finite-difference checks."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    H = rnd(feat)
    layers = params["layers"]
    cache: List[Dict[str, np.ndarray]] = []
    for k, L in enumerate(layers):
        A = rnd(M @ H)
        Ws, Wn = rnd(L["Ws"]), rnd(L["Wn"])
        Y = H @ Ws.T + A @ Wn.T + np.asarray(L["b"], dtype=np.float64)[None, :]
        cache.append({"H": H, "A": A, "Ws": Ws, "Wn": Wn})
        if k < len(layers) - 1:
            H = rnd(np.maximum(Y, 0.0))
        else:
            H = Y
    return H, cache


def mpnn_backward(cache, M: sp.csr_matrix, dZ: np.ndarray, bf16: bool = True):
    """Gradients of every layer's Ws, Wn, b for upstream gradient dZ = dLoss/dZ_w."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    MT = M.T.tocsr()
    n_layers = len(cache)
    grads: List[Optional[Dict[str, np.ndarray]]] = [None] * n_layers
    dY = rnd(dZ)
    for k in range(n_layers - 1, -1, -1):
        c = cache[k]
        grads[k] = {"Ws": dY.T @ c["H"], "Wn": dY.T @ c["A"], "b": dY.sum(axis=0)}
        if k == 0:
            break
        Gs = dY @ c["Ws"]
        Gn = dY @ c["Wn"]
        dH = Gs + MT @ Gn
        dY = rnd(dH * (c["H"] > 0.0))
    return {"layers": grads}


def bce_grad(Z: np.ndarray, target: np.ndarray, beta: float) -> np.ndarray:
    """d/dZ of beta * sum BCE(sigmoid(Z), target) = beta * (sigmoid(Z) - target)."""
    P, _ = objective.sigmoid_pair(Z)
    return beta * (P - np.asarray(target, dtype=np.float64))


def bce_value(Z: np.ndarray, target: np.ndarray, beta: float) -> float:
    """beta * sum [softplus(Z) - target * Z], the BCE of sigmoid(Z) with logits."""
    Z = np.asarray(Z, dtype=np.float64)
    sp_ = np.maximum(Z, 0.0) + np.log1p(np.exp(-np.abs(Z)))
    return float(beta * np.sum(sp_ - np.asarray(target, dtype=np.float64) * Z))


def warm_loss_and_grads(params, feat, M, graph, problem: str, lam, gamma: float,
                        target=None, beta: float = 0.0, alpha: int = 2, bf16: bool = True):
    """One training evaluation of the warm-start network: (Z_w, loss terms per
    graph, dZ_w, grads).  The CPRA part is computed per graph of a batch."""
    Zw, cache = mpnn_forward(params, feat, M, bf16)
    gp = np.asarray(graph.graph_ptr, dtype=np.int64)
    dZ = np.zeros_like(Zw)
    terms = []
    for g in range(gp.size - 1):
        sub = objective._slice_graph(graph, int(gp[g]), int(gp[g + 1])) if gp.size > 2 else graph
        Zg = Zw[gp[g]:gp[g + 1]]
        terms.append(objective.loss_terms(Zg, sub, problem, lam, gamma, alpha))
        dZ[gp[g]:gp[g + 1]] = objective.grad_wrt_Z(Zg, sub, problem, lam, gamma, alpha)
    if target is not None and beta != 0.0:
        dZ = dZ + bce_grad(Zw, target, beta)
    grads = mpnn_backward(cache, M, dZ, bf16)
    return Zw, terms, dZ, grads
