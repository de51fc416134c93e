"""Seeded initial parameters of the GNN that parameterises the relaxed solutions.

The paper leaves the initialisation unstated.  The project fixes it here and
hands the same float32 bytes to every consumer:

* trainable node embedding ``emb`` [n, in_dim] with entries ~ N(0, 1);
* per layer k: self weight ``Ws`` and neighbour weight ``Wn``, both
  [out_k, in_k] row-major with entries ~ U(-1/sqrt(in_k), 1/sqrt(in_k)), and
  (GraphSAGE layers only) a bias ``b`` [out_k] initialised to zero.

Layer widths: in_0 = in_dim (= hidden unless stated), every hidden layer
maps to ``hidden``, the last layer maps to S (one output per relaxed
solution).
"""

from __future__ import annotations

from typing import Dict, List

import numpy as np

LAYER_KINDS = ("gcn", "sage")


def layer_dims(n_layers: int, in_dim: int, hidden: int, S: int):
    """[(in_k, out_k)] for k = 1..n_layers."""
    if n_layers < 1:
        raise ValueError("need at least one layer")
    dims = []
    d_in = in_dim
    for k in range(n_layers):
        d_out = S if k == n_layers - 1 else hidden
        dims.append((d_in, d_out))
        d_in = d_out
    return dims


def param_shapes(kind: str, n_nodes: int, n_layers: int, hidden: int, S: int,
                 in_dim: int = None) -> Dict[str, object]:
    in_dim = hidden if in_dim is None else in_dim
    shapes = {"emb": (n_nodes, in_dim), "layers": []}
    for d_in, d_out in layer_dims(n_layers, in_dim, hidden, S):
        layer = {"Ws": (d_out, d_in), "Wn": (d_out, d_in)}
        if kind == "sage":
            layer["b"] = (d_out,)
        shapes["layers"].append(layer)
    return shapes


def init_params(kind: str, n_nodes: int, n_layers: int, hidden: int, S: int,
                seed: int, in_dim: int = None) -> Dict[str, object]:
    """Seeded float32 parameters: {"emb": array, "layers": [{"Ws","Wn"[,"b"]}]}."""
    if kind not in LAYER_KINDS:
        raise ValueError(f"layer kind must be one of {LAYER_KINDS}")
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = param_shapes(kind, n_nodes, n_layers, hidden, S, in_dim)
    emb = rng.standard_normal(shapes["emb"], dtype=np.float32)
    layers: List[Dict[str, np.ndarray]] = []
    for sh in shapes["layers"]:
        d_out, d_in = sh["Ws"]
        bound = 1.0 / np.sqrt(d_in)
        layer = {
            "Ws": rng.uniform(-bound, bound, size=(d_out, d_in)).astype(np.float32),
            "Wn": rng.uniform(-bound, bound, size=(d_out, d_in)).astype(np.float32),
        }
        if kind == "sage":
            layer["b"] = np.zeros(d_out, dtype=np.float32)
        layers.append(layer)
    return {"emb": emb, "layers": layers}


def init_params_per_graph(kind: str, n_nodes: int, n_layers: int, hidden: int, S: int,
                          n_graphs: int, seed: int, in_dim: int = None) -> Dict[str, object]:
    """Seeded float32 parameters with one network per graph of a batch: the
    embedding as in init_params, and every layer's Ws, Wn [G, out_k, in_k] and
    b [G, out_k] with the same per-entry distributions, graph g's matrices drawn
    after graph g-1's."""
    if kind not in LAYER_KINDS:
        raise ValueError(f"layer kind must be one of {LAYER_KINDS}")
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = param_shapes(kind, n_nodes, n_layers, hidden, S, in_dim)
    emb = rng.standard_normal(shapes["emb"], dtype=np.float32)
    layers: List[Dict[str, np.ndarray]] = []
    for sh in shapes["layers"]:
        d_out, d_in = sh["Ws"]
        bound = 1.0 / np.sqrt(d_in)
        layer = {"Ws": np.empty((n_graphs, d_out, d_in), np.float32),
                 "Wn": np.empty((n_graphs, d_out, d_in), np.float32)}
        for g in range(n_graphs):
            layer["Ws"][g] = rng.uniform(-bound, bound, size=(d_out, d_in))
            layer["Wn"][g] = rng.uniform(-bound, bound, size=(d_out, d_in))
        if kind == "sage":
            layer["b"] = np.zeros((n_graphs, d_out), dtype=np.float32)
        layers.append(layer)
    return {"emb": emb, "layers": layers}


def random_logits(n: int, S: int, seed: int, scale: float = 2.0,
                  near_binary: bool = False) -> np.ndarray:
    """Logit matrices for kernel-level tests and benchmarks.

    ``near_binary`` draws |Z| in [10, 20] with random signs, the saturated
    regime that annealing drives the relaxed solutions into.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if near_binary:
        mag = rng.uniform(10.0, 20.0, size=(n, S))
        sgn = np.where(rng.random((n, S)) < 0.5, -1.0, 1.0)
        return (mag * sgn).astype(np.float32)
    return (scale * rng.standard_normal((n, S))).astype(np.float32)


def init_mpnn_params(in_dim: int, hidden: int, S: int, n_layers: int, seed: int):
    """Seeded float32 weights of the warm-start network (GraphSAGE form with bias):
    per layer Ws, Wn [out_k, in_k] ~ U(-1/sqrt(in_k), 1/sqrt(in_k)), b [out_k] = 0."""
    rng = np.random.default_rng(seed)
    layers: List[Dict[str, np.ndarray]] = []
    for d_in, d_out in layer_dims(n_layers, in_dim, hidden, S):
        bound = 1.0 / np.sqrt(d_in)
        layers.append({"Ws": rng.uniform(-bound, bound, (d_out, d_in)).astype(np.float32),
                       "Wn": rng.uniform(-bound, bound, (d_out, d_in)).astype(np.float32),
                       "b": np.zeros(d_out, dtype=np.float32)})
    return {"layers": layers}


def random_channels(n: int, R: int, seed: int) -> np.ndarray:
    """Seeded per-node random input channels ~ U(-1, 1), float32 [n, R]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (n, R)).astype(np.float32)
