"""The GNN that parameterises P, in float64.  TEST INFRASTRUCTURE ONLY.

GNN appendix (aggregate/combine; the GCN equation):
  h_v^k = act( W^k * mean_{u in N(v)} h_u^{k-1} + B^k h_v^{k-1} )
Here W^k is the neighbour weight ``Wn`` and B^k the self weight ``Ws``.
The GraphSAGE layers of the experiments add one bias per layer; that form
is fixed by the parameter counts printed in the MIS and DBM result tables
(2 H0^2 + H0 + (2 H0 + 1) S for a two-layer network with H1 = H0, H2 = S,
the node embedding not counted).

Architecture appendix: the input is a trainable per-node embedding h^0;
ReLU follows every layer but the last; the last layer has S outputs and is
followed by the sigmoid (applied in ``objective``).

Mean aggregation is M = D^-1 A over the neighbour set (structure only,
ignoring edge weights); an isolated node aggregates to 0.  The oracle
aggregates first and multiplies second, literally as the equation reads.
"""

from __future__ import annotations

from typing import Dict, List

import numpy as np
import scipy.sparse as sp


def mean_aggregation_matrix(row_ptr: np.ndarray, col_idx: np.ndarray) -> sp.csr_matrix:
    """M = D^-1 A as a sparse matrix (rows of isolated nodes are zero)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = row_ptr.size - 1
    deg = np.diff(row_ptr).astype(np.float64)
    vals = np.repeat(np.divide(1.0, deg, out=np.zeros_like(deg), where=deg > 0), np.diff(row_ptr))
    return sp.csr_matrix((vals, np.asarray(col_idx, dtype=np.int64), row_ptr), shape=(n, n))


def to_f64(params: Dict[str, object]) -> Dict[str, object]:
    return {"emb": np.asarray(params["emb"], dtype=np.float64),
            "layers": [{k: np.asarray(v, dtype=np.float64) for k, v in L.items()}
                       for L in params["layers"]]}


def forward(params: Dict[str, object], M: sp.csr_matrix, z_offset=None):
    """Returns (Z, cache).  cache holds each layer's input, aggregate and pre-activation.

    z_offset (optional, [N, S]): fixed logits added to the network's output, so
    that P = sigmoid(GNN(G) + z_offset) -- the warm start of a learned proposal."""
    H = params["emb"]
    cache: List[Dict[str, np.ndarray]] = []
    n_layers = len(params["layers"])
    for k, L in enumerate(params["layers"]):
        agg = M @ H
        Y = agg @ L["Wn"].T + H @ L["Ws"].T
        if "b" in L:
            Y = Y + L["b"][None, :]
        cache.append({"H": H, "agg": agg, "Y": Y})
        H = np.maximum(Y, 0.0) if k < n_layers - 1 else Y
    if z_offset is not None:
        H = H + np.asarray(z_offset, dtype=np.float64)
    return H, cache


def backward(params: Dict[str, object], M: sp.csr_matrix, cache, dZ: np.ndarray,
             relu_active=None):
    """Gradients of a scalar loss with dLoss/dZ = dZ, by the chain rule through ``forward``.

    ``relu_active`` (optional): per hidden layer k (0-based, all but the last), a
    boolean array [N, out_k] of the units on the positive side of their ReLU.
    By default the oracle's own pre-activations decide (Y > 0); a comparison
    with a lower-precision forward passes that forward's decisions instead, so
    that both sides take the ReLU's derivative at the same (discrete) point.
    """
    grads = {"layers": [None] * len(params["layers"])}
    dY = np.asarray(dZ, dtype=np.float64)
    MT = M.T.tocsr()
    for k in range(len(params["layers"]) - 1, -1, -1):
        L = params["layers"][k]
        c = cache[k]
        if k < len(params["layers"]) - 1:
            active = (c["Y"] > 0.0) if relu_active is None else relu_active[k]
            dY = dY * active
        g = {"Ws": dY.T @ c["H"], "Wn": dY.T @ c["agg"]}
        if "b" in L:
            g["b"] = dY.sum(axis=0)
        grads["layers"][k] = g
        dY = dY @ L["Ws"] + MT @ (dY @ L["Wn"])
    grads["emb"] = dY
    return grads


def param_count(kind: str, dims, include_embedding: bool = False, n_nodes: int = 0,
                in_dim: int = 0) -> int:
    """Number of trainable weights: two [out, in] matrices per layer (+ out biases for SAGE)."""
    total = 0
    for d_in, d_out in dims:
        total += 2 * d_in * d_out + (d_out if kind == "sage" else 0)
    if include_embedding:
        total += n_nodes * in_dim
    return total
