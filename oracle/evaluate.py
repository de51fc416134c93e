"""Rounding and evaluation of the S solutions.  TEST INFRASTRUCTURE ONLY.

* Rounding (training-setting appendix): P_is <= 0.5 -> 0, P_is > 0.5 -> 1.
* MIS (problem-specification appendix): the set size sum_i x_i and the
  number of violated edges (both endpoints selected); a head is an
  independent set iff it violates no edge.
* MaxCut: cut value sum_{i<j} A_ij [x_i != x_j] (the negated QUBO objective).
* One instance per head (per-head edge weights [nnz, S]): head s is evaluated
  on its own instance -- the edges whose weight in column s is nonzero, with
  those weights; MIS violations and cut edges count those edges only.
* DScore (Sec. 4.1 Evaluation Metrics):
  2 / (N S (S-1)) * sum_{s<l} d_H(x_s, x_l), from the pairwise Hamming
  distances themselves.
All counts are exact integers (int64); weighted cuts are float64.
"""

from __future__ import annotations

from typing import Dict

import numpy as np

from .objective import edges_of


def round_solutions(Z: np.ndarray) -> np.ndarray:
    """X = [P > 1/2] with P = sigmoid(Z), as uint8 [N, S].

    sigmoid is strictly increasing with sigmoid(0) = 1/2, so P > 1/2 exactly
    when Z > 0; the decision is taken on Z itself.  (A rounded FP64
    sigmoid(Z) equals 0.5 for 0 < Z < ~1.1e-16 and would send those entries to
    0, against the rounding rule's exact meaning.)"""
    return (np.asarray(Z, dtype=np.float64) > 0.0).astype(np.uint8)


def pairwise_hamming_sum(X: np.ndarray) -> int:
    """sum_{s<l} d_H(X[:, s], X[:, l]) computed pair by pair through a Gram matrix."""
    Xi = X.astype(np.int64)
    ones = Xi.sum(axis=0)
    gram = Xi.T @ Xi
    D = ones[:, None] + ones[None, :] - 2 * gram  # d_H for every ordered pair
    return int(np.triu(D, k=1).sum())


def pairwise_hamming_matrix(X: np.ndarray) -> np.ndarray:
    """D[s, l] = d_H(X[:, s], X[:, l]) for every pair of heads (int64 [S, S])."""
    Xi = X.astype(np.int64)
    ones = Xi.sum(axis=0)
    return ones[:, None] + ones[None, :] - 2 * (Xi.T @ Xi)


def diversity_stats(X: np.ndarray):
    """Solution-diversity analytics of Sec. 4.1 / the diversity appendix figures:
    the distance matrix, the histogram of d_H over the S(S-1)/2 pairs (bins 0..N),
    and the number of distinct solutions among the heads."""
    N, S = X.shape
    D = pairwise_hamming_matrix(X)
    iu = np.triu_indices(S, k=1)
    hist = np.bincount(D[iu], minlength=N + 1).astype(np.int64)
    unique = int(np.unique(X.T.astype(np.uint8), axis=0).shape[0]) if S else 0
    return {"D": D, "hist": hist, "unique": unique}


def dscore(X: np.ndarray) -> float:
    N, S = X.shape
    if S < 2 or N == 0:
        return 0.0
    return 2.0 * pairwise_hamming_sum(X) / (N * S * (S - 1))


def evaluate_one(X: np.ndarray, graph, problem: str, node_weight=None,
                 edge_weight=None) -> Dict[str, object]:
    """node_weight ([N] or [N, S], MIS only): also the total weight of each head's set.
    edge_weight ([nnz, S]): head s is evaluated on its own instance."""
    Xi = X.astype(np.int64)
    N, S = X.shape
    if edge_weight is None:
        ei, ej, w = edges_of(graph.row_ptr, graph.col_idx, graph.weight)
        W = np.repeat(w[:, None], S, axis=1)   # every head on the graph itself
        present = np.ones_like(W, dtype=bool)
    else:
        from .objective import instance_weights
        ew = instance_weights(graph, edge_weight, S)
        ei, ej, _ = edges_of(graph.row_ptr, graph.col_idx)
        rp = np.asarray(graph.row_ptr, dtype=np.int64)
        rows = np.repeat(np.arange(N, dtype=np.int64), np.diff(rp))
        W = ew[rows < np.asarray(graph.col_idx, dtype=np.int64)]
        present = W != 0
    out = {"pair_hamming": pairwise_hamming_sum(X)}
    if problem == "mis":
        out["size"] = Xi.sum(axis=0)
        out["violations"] = (Xi[ei] * Xi[ej] * present).sum(axis=0)
        from .objective import node_weights
        out["weight"] = (node_weights(node_weight, *X.shape) * Xi).sum(axis=0)
    elif problem == "maxcut":
        differ = (Xi[ei] != Xi[ej]) & present
        out["cut_edges"] = differ.sum(axis=0).astype(np.int64)
        out["cut"] = (W * differ).sum(axis=0)
    else:
        raise ValueError(problem)
    return out


def evaluate(X: np.ndarray, graph, problem: str, node_weight=None, edge_weight=None):
    """Per-graph evaluation; a single graph gives a one-element list."""
    from .objective import _slice_graph, entry_range
    gp = np.asarray(graph.graph_ptr, dtype=np.int64)
    res = []
    for g in range(gp.size - 1):
        lo, hi = int(gp[g]), int(gp[g + 1])
        sub = _slice_graph(graph, lo, hi)
        nw = None if node_weight is None else np.asarray(node_weight)[lo:hi]
        a, b = entry_range(graph, lo, hi)
        ew = None if edge_weight is None else np.asarray(edge_weight)[a:b]
        res.append(evaluate_one(X[lo:hi], sub, problem, nw, ew))
    return res


def best_feasible_mis(ev: Dict[str, object]) -> int:
    """Largest independent set among the heads (0 if none is feasible)."""
    ok = ev["violations"] == 0
    return int(ev["size"][ok].max()) if np.any(ok) else 0
