"""Relaxed CPRA objective and its gradient, in float64.  TEST INFRASTRUCTURE ONLY.

Notation follows the paper: P in [0,1]^{N x S} holds S relaxed solutions
(heads) as columns; P = sigmoid(Z) with Z the GNN output logits (GNN
appendix, sigmoid after the last layer).

Discrete objectives (problem-specification appendix, objective table):
  MIS:    l(x; G, lam) = -sum_i w_i x_i + lam * sum_{(i,j) in E} x_i x_j
          (node weights w_i = 1 for plain MIS; weighted MIS takes one weight
          vector per head -- the weighted-MIS tasks of the two-stage appendix)
  MaxCut: l(x; G)      = sum_{i<j} A_ij (2 x_i x_j - x_i - x_j)
Each edge {i, j} is counted once (i < j).  The relaxation (Sec. 2.2) keeps
the same multilinear polynomial with p in [0,1]^N, so it equals the
discrete objective on every binary point.

Multiple instances (Sec. 3.1 lets every head s carry its own instance C_s;
the multi-instance appendix solves 27 instances of one structure at once):
with per-head edge weights ``edge_weight`` [nnz, S] (one value per CSR entry
and head, symmetric), head s is the objective above on the graph whose edge
weights are column s -- a zero weight leaves the edge out of that head's
instance.  The annealing and diversity terms do not depend on the instances.

CPRA loss (Sec. 3.1, Eq. CPRA-loss-function-GNN, and Sec. 3.3,
Eq. CPRA-loss-function-GNN-variation):
  R(P) = sum_s l(P[:, s]; lam_s) + gamma * S(P) + nu * Psi(P)
  S(P) = sum_{i,s} (1 - (2 P_is - 1)^alpha),  alpha even
  Psi(P) = -S * sum_i STD_s[P_is]
with STD the empirical (population, 1/K) standard deviation of the Notation
section; ``ddof=1`` selects the sample form mentioned at the end of Sec. 3.3.

Numerics: wherever 1 - P appears it is evaluated as sigmoid(-Z), and
1 - t^alpha with t = 2P - 1 is evaluated through the exact factorisation
1 - t^alpha = (1 - t)(1 + t) * sum_{k < alpha/2} t^(2k) = 4 P Q * sum t^(2k)
with Q = 1 - P, so that saturated entries keep their relative accuracy.
"""

from __future__ import annotations

from typing import Dict, Optional

import numpy as np

PROBLEMS = ("mis", "maxcut")


def sigmoid_pair(Z: np.ndarray):
    """(P, Q) = (sigmoid(Z), sigmoid(-Z)), each without cancellation."""
    Z = np.asarray(Z, dtype=np.float64)
    e = np.exp(-np.abs(Z))
    inv = 1.0 / (1.0 + e)
    P = np.where(Z >= 0, inv, e * inv)
    Q = np.where(Z >= 0, e * inv, inv)
    return P, Q


def edges_of(row_ptr: np.ndarray, col_idx: np.ndarray, weight: Optional[np.ndarray] = None):
    """Undirected edge list (i < j) with weights A_ij (1 where no weights are given)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    cols = np.asarray(col_idx, dtype=np.int64)
    keep = rows < cols
    w = np.ones(int(keep.sum()), dtype=np.float64) if weight is None else \
        np.asarray(weight, dtype=np.float64)[keep]
    return rows[keep], cols[keep], w


# ---------------------------------------------------------------------------
# Discrete objectives (objective table)
# ---------------------------------------------------------------------------

def discrete_mis(x: np.ndarray, ei, ej, w, lam: float, node_w=None) -> float:
    """-sum_i w_i x_i + lam * sum_{(i,j) in E} A_ij x_i x_j for one binary vector."""
    x = np.asarray(x, dtype=np.float64)
    lin = x.sum() if node_w is None else float(np.sum(np.asarray(node_w, dtype=np.float64) * x))
    return float(-lin + lam * np.sum(w * x[ei] * x[ej]))


def node_weights(node_weight, N: int, S: int) -> np.ndarray:
    """Node weights as [N, S] float64: None -> ones; [N] -> shared by every head."""
    if node_weight is None:
        return np.ones((N, S))
    w = np.asarray(node_weight, dtype=np.float64)
    if w.ndim == 1:
        w = np.repeat(w[:, None], S, axis=1)
    if w.shape != (N, S):
        raise ValueError("node weights must be [N] or [N, S]")
    return w


def instance_weights(graph, edge_weight, S: int) -> np.ndarray:
    """Per-head edge weights as [nnz, S] float64, checked to be symmetric
    (entry (i, j) of head s equals entry (j, i))."""
    rp = np.asarray(graph.row_ptr, dtype=np.int64)
    ci = np.asarray(graph.col_idx, dtype=np.int64)
    w = np.asarray(edge_weight, dtype=np.float64)
    if w.shape != (ci.size, S):
        raise ValueError("per-head edge weights must be [nnz, S]")
    n = rp.size - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    # entry (j, i) of every entry (i, j): the CSR keys i * n + j are sorted
    keys = rows * n + ci
    back = np.searchsorted(keys, ci * n + rows)
    if back.size and not np.array_equal(w, w[back]):
        raise ValueError("per-head edge weights must be symmetric")
    return w


def head_instance(graph, edge_weight: np.ndarray, s: int):
    """Instance C_s of head s: the graph's pattern with edge weights edge_weight[:, s]."""
    return _Sub(np.asarray(graph.row_ptr), np.asarray(graph.col_idx), edge_weight[:, s])


def discrete_maxcut(x: np.ndarray, ei, ej, w) -> float:
    """sum_{i<j} A_ij (2 x_i x_j - x_i - x_j) for one binary vector."""
    x = np.asarray(x, dtype=np.float64)
    return float(np.sum(w * (2.0 * x[ei] * x[ej] - x[ei] - x[ej])))


# ---------------------------------------------------------------------------
# Relaxed objective per head, annealing term, diversity term
# ---------------------------------------------------------------------------

def relaxed_head_losses(P: np.ndarray, ei, ej, w, problem: str,
                        lam: Optional[np.ndarray], node_weight=None) -> np.ndarray:
    """l_hat(P[:, s]; C, lam_s) for every head s (the relaxation of Sec. 2.2)."""
    P = np.asarray(P, dtype=np.float64)
    if problem == "mis":
        lam = np.asarray(lam, dtype=np.float64)
        pair = np.sum(w[:, None] * P[ei] * P[ej], axis=0)
        nw = node_weights(node_weight, *P.shape)
        return -(nw * P).sum(axis=0) + lam * pair
    if problem == "maxcut":
        return np.sum(w[:, None] * (2.0 * P[ei] * P[ej] - P[ei] - P[ej]), axis=0)
    raise ValueError(problem)


def one_minus_t_pow(P: np.ndarray, Q: np.ndarray, alpha: int) -> np.ndarray:
    """phi(P) = 1 - (2P - 1)^alpha elementwise (Lemma A.1's phi), alpha even."""
    check_alpha(alpha)
    t = P - Q
    series = np.zeros_like(P)
    for k in range(alpha // 2):
        series = series + t ** (2 * k)
    return 4.0 * P * Q * series


def check_alpha(alpha: int) -> None:
    if int(alpha) != alpha or alpha < 2 or alpha % 2:
        raise ValueError("alpha must be an even integer >= 2")


def entropy_term(P: np.ndarray, Q: np.ndarray, alpha: int) -> float:
    """S(P) = sum_{i,s} (1 - (2 P_is - 1)^alpha)   (Sec. 3.1)."""
    return float(np.sum(one_minus_t_pow(P, Q, alpha)))


def identical_rows(P: np.ndarray) -> np.ndarray:
    """Nodes whose S heads hold one and the same value (max == min over the row)."""
    return P.max(axis=1) == P.min(axis=1)


def row_std(P: np.ndarray, ddof: int = 0) -> np.ndarray:
    """STD_s[P_is] per node i, two-pass: mean first, then squared deviations.

    A row whose heads are all equal has STD exactly 0.  The rounded mean of S
    equal values need not equal them (e.g. ten copies of 0.3 sum to
    2.9999999999999996), which would leave a spurious sigma of ~1e-17, so such
    rows are set to 0 by their definition rather than by the two passes."""
    S = P.shape[1]
    mu = P.sum(axis=1) / S
    dev = P - mu[:, None]
    sig = np.sqrt(np.sum(dev * dev, axis=1) / (S - ddof))
    return np.where(identical_rows(P), 0.0, sig)


def diversity_term(P: np.ndarray, ddof: int = 0) -> float:
    """Psi(P) = -S * sum_i STD_s[P_is]   (Sec. 3.3)."""
    S = P.shape[1]
    return float(-S * np.sum(row_std(P, ddof)))


# ---------------------------------------------------------------------------
# Total loss and gradient
# ---------------------------------------------------------------------------

def loss_terms(Z: np.ndarray, graph, problem: str, lam, gamma: float, alpha: int,
               nu: float = 0.0, ddof: int = 0, node_weight=None,
               edge_weight=None) -> Dict[str, object]:
    """All loss terms of one graph at logits Z [N, S].

    Returns {"head": l_hat_s [S], "entropy": S(P), "psi": Psi(P), "total": R}.
    ``graph`` provides row_ptr, col_idx and weight (None = unweighted);
    ``edge_weight`` [nnz, S], when given, replaces the graph's weights with one
    instance per head (head s alone on the graph weighted by column s).
    """
    P, Q = sigmoid_pair(Z)
    if edge_weight is None:
        ei, ej, w = edges_of(graph.row_ptr, graph.col_idx, graph.weight)
        head = relaxed_head_losses(P, ei, ej, w, problem, lam, node_weight)
    else:
        N, S = P.shape
        ew = instance_weights(graph, edge_weight, S)
        nw = None if node_weight is None else node_weights(node_weight, N, S)
        head = np.zeros(S)
        for s in range(S):
            ei, ej, w = edges_of(graph.row_ptr, graph.col_idx, ew[:, s])
            head[s] = relaxed_head_losses(P[:, [s]], ei, ej, w, problem,
                                          None if problem != "mis" else np.asarray(lam)[[s]],
                                          None if nw is None else nw[:, [s]])[0]
    ent = entropy_term(P, Q, alpha)
    psi = diversity_term(P, ddof) if P.shape[1] > 1 else 0.0
    total = float(head.sum() + gamma * ent + nu * psi)
    return {"head": head, "entropy": ent, "psi": psi, "total": total}


def _problem_grad(P: np.ndarray, graph, weight, problem: str, lam, node_weight) -> np.ndarray:
    """d/dP of sum_s l_hat_s for the heads (columns) of P on one weighted graph."""
    ei, ej, w = edges_of(graph.row_ptr, graph.col_idx, weight)
    N, S = P.shape
    # Neighbour sums by scattering each undirected edge to both endpoints.
    nb = np.zeros((N, S), dtype=np.float64)
    np.add.at(nb, ei, w[:, None] * P[ej])
    np.add.at(nb, ej, w[:, None] * P[ei])
    if problem == "mis":
        return -node_weights(node_weight, N, S) + np.asarray(lam, dtype=np.float64)[None, :] * nb
    if problem == "maxcut":
        wdeg = np.zeros(N, dtype=np.float64)
        np.add.at(wdeg, ei, w)
        np.add.at(wdeg, ej, w)
        return 2.0 * nb - wdeg[:, None]
    raise ValueError(problem)


def grad_wrt_P(P: np.ndarray, Q: np.ndarray, graph, problem: str, lam, gamma: float,
               alpha: int, nu: float = 0.0, ddof: int = 0, node_weight=None,
               edge_weight=None) -> np.ndarray:
    """dR/dP [N, S] (derived by hand from the loss above).

    problem part: MIS    -w_is + lam_s * sum_{j in N(i)} A_ij P_js
                  MaxCut sum_{j in N(i)} A_ij (2 P_js - 1)
    annealing:    gamma * d/dP (1 - (2P-1)^alpha) = -2 alpha gamma (2P-1)^(alpha-1)
    diversity:    nu * dPsi/dP_is = -nu * S (P_is - mu_i) / ((S - ddof) sigma_i),
                  taken as 0 where sigma_i = 0, i.e. where all heads of node i are
                  equal (0 is a subgradient of the norm there; any subgradient sums
                  to 0 over the heads, as the gradient does wherever sigma_i > 0).
    """
    N, S = P.shape
    if edge_weight is None:
        g = _problem_grad(P, graph, graph.weight, problem, lam, node_weight)
    else:  # head s on its own instance
        ew = instance_weights(graph, edge_weight, S)
        nw = None if node_weight is None else node_weights(node_weight, N, S)
        g = np.zeros((N, S))
        for s in range(S):
            g[:, [s]] = _problem_grad(P[:, [s]], graph, ew[:, s], problem,
                                      None if problem != "mis" else np.asarray(lam)[[s]],
                                      None if nw is None else nw[:, [s]])
    check_alpha(alpha)
    t = P - Q
    g = g - 2.0 * alpha * gamma * t ** (alpha - 1)
    if nu != 0.0 and S > 1:
        mu = P.sum(axis=1) / S
        sig = row_std(P, ddof)
        dev = P - mu[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            dpsi = np.where(sig[:, None] > 0, -S * dev / ((S - ddof) * sig[:, None]), 0.0)
        g = g + nu * dpsi
    return g


def grad_wrt_Z(Z: np.ndarray, graph, problem: str, lam, gamma: float, alpha: int,
               nu: float = 0.0, ddof: int = 0, node_weight=None, edge_weight=None) -> np.ndarray:
    """dR/dZ = dR/dP * P * (1 - P), with 1 - P taken as sigmoid(-Z)."""
    P, Q = sigmoid_pair(Z)
    return grad_wrt_P(P, Q, graph, problem, lam, gamma, alpha, nu, ddof, node_weight,
                      edge_weight) * P * Q


def entry_range(graph, lo: int, hi: int):
    """CSR entries [a, b) of rows lo..hi-1."""
    rp = np.asarray(graph.row_ptr, dtype=np.int64)
    return int(rp[lo]), int(rp[hi])


def batched_loss_terms(Z: np.ndarray, graph, problem, lam, gamma, alpha, nu=0.0, ddof=0,
                       node_weight=None, edge_weight=None):
    """Per-graph loss terms of a block-diagonal batch (graph.graph_ptr slices)."""
    out = []
    gp = np.asarray(graph.graph_ptr, dtype=np.int64)
    for g in range(gp.size - 1):
        lo, hi = int(gp[g]), int(gp[g + 1])
        sub = _slice_graph(graph, lo, hi)
        nw = None if node_weight is None else np.asarray(node_weight)[lo:hi]
        a, b = entry_range(graph, lo, hi)
        ew = None if edge_weight is None else np.asarray(edge_weight)[a:b]
        out.append(loss_terms(Z[lo:hi], sub, problem, lam, gamma, alpha, nu, ddof, nw, ew))
    return out


class _Sub:
    def __init__(self, row_ptr, col_idx, weight):
        self.row_ptr, self.col_idx, self.weight = row_ptr, col_idx, weight
        self.graph_ptr = np.array([0, row_ptr.size - 1], dtype=np.int64)  # one graph


def _slice_graph(graph, lo: int, hi: int):
    rp = np.asarray(graph.row_ptr, dtype=np.int64)
    a, b = rp[lo], rp[hi]
    w = None if graph.weight is None else graph.weight[a:b]
    return _Sub(rp[lo:hi + 1] - a, np.asarray(graph.col_idx[a:b], dtype=np.int64) - lo, w)
