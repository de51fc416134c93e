"""Named workloads: graph recipe, model shape, penalty grid and schedule.

Each preset fixes everything a run needs except the implementation:

* C1 -- MIS, random 3-regular graph, N=100, 2-layer GCN (hidden 32), S=10,
  lambda_s = linspace(0.5, 5, 10), gamma linear -2 -> +0.1 over 2000 steps.
* C2 -- MIS, random 5-regular graph, N=10,000 (25,000 edges), 2-layer
  GraphSAGE (hidden 256), S=100, lambda_s = logspace(-1, 1, 100), gamma
  -2 -> +0.1 over 5000 steps.
* C3 -- MaxCut, block-diagonal batch of 256 Erdos-Renyi graphs with
  N_b ~ U{500..5000} and mean degree ~ U[4, 10], 2-layer GCN (hidden 64),
  S=32, diversity weight nu=0.1, gamma -2 -> +0.1 over 2000 steps.  C3s is
  one GPU's eighth of it (32 graphs).
* C4 -- MIS, random 20-regular graph, N=100,000 (1,000,000 edges), 3-layer
  GCN (hidden 128), S=64, lambda_s = logspace(-1, 1, 64).
* C5 -- warm-start test graphs: random d-regular, N=50,000, S=32,
  lambda_s = logspace(-1, 1, 32), 2-layer GCN (hidden 64).

All use alpha=2 and Adam (lr 1e-3, betas 0.9/0.999, eps 1e-8, no weight decay).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, Optional

import numpy as np

from .graphs import CSRGraph, disjoint_union, erdos_renyi_graph, random_regular_graph


@dataclass
class Preset:
    name: str
    problem: str  # "mis" or "maxcut"
    layer_kind: str  # "gcn" or "sage"
    n_layers: int
    hidden: int
    S: int
    lam: Optional[np.ndarray]  # float32 [S] (MIS) or None (MaxCut)
    gamma_start: float
    gamma_end: float
    T: int
    alpha: int = 2
    nu: float = 0.0
    lr: float = 1e-3
    recompute: bool = False
    side_first: bool = False  # capture each backward fork's side work first (CPRA_SIDE_FIRST=1)
    graph_fn: Callable[[], CSRGraph] = field(default=None, repr=False)
    description: str = ""

    def graph(self) -> CSRGraph:
        return self.graph_fn()


def _c3_graph(n_graphs: int, seed: int) -> CSRGraph:
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(500, 5001, size=n_graphs)
    degs = rng.uniform(4.0, 10.0, size=n_graphs)
    seeds = rng.integers(0, 2 ** 31 - 1, size=n_graphs)
    graphs = [erdos_renyi_graph(int(n), float(d) / (int(n) - 1), int(s))
              for n, d, s in zip(sizes, degs, seeds)]
    return disjoint_union(graphs)


def _logspace(S: int) -> np.ndarray:
    return np.logspace(-1.0, 1.0, S).astype(np.float32)


PRESETS: Dict[str, Preset] = {
    "C1": Preset(
        "C1", "mis", "gcn", 2, 32, 10,
        np.linspace(0.5, 5.0, 10).astype(np.float32), -2.0, 0.1, 2000,
        graph_fn=lambda: random_regular_graph(100, 3, seed=1),
        description="MIS on a random 3-regular graph, N=100, 2-layer GCN hidden 32, S=10"),
    "C2": Preset(
        "C2", "mis", "sage", 2, 256, 100, _logspace(100), -2.0, 0.1, 5000,
        graph_fn=lambda: random_regular_graph(10_000, 5, seed=2),
        description="MIS on a random 5-regular graph, N=10000, 2-layer GraphSAGE hidden 256, S=100"),
    "C3": Preset(
        "C3", "maxcut", "gcn", 2, 64, 32, None, -2.0, 0.1, 2000, nu=0.1, side_first=True,
        graph_fn=lambda: _c3_graph(256, seed=3),
        description="MaxCut on 256 Erdos-Renyi graphs (N~U{500..5000}, mean degree~U[4,10]), "
                    "2-layer GCN hidden 64, S=32, nu=0.1"),
    "C3s": Preset(
        "C3s", "maxcut", "gcn", 2, 64, 32, None, -2.0, 0.1, 2000, nu=0.1,
        graph_fn=lambda: _c3_graph(32, seed=33),
        description="one eighth of C3: 32 Erdos-Renyi graphs, MaxCut, S=32, nu=0.1"),
    "C4": Preset(
        "C4", "mis", "gcn", 3, 128, 64, _logspace(64), -2.0, 0.1, 5000, recompute=True,
        graph_fn=lambda: random_regular_graph(100_000, 20, seed=4),
        description="MIS on a random 20-regular graph, N=100000, 3-layer GCN hidden 128, S=64"),
    "C5": Preset(
        "C5", "mis", "gcn", 2, 64, 32, _logspace(32), -2.0, 0.1, 3000,
        graph_fn=lambda: random_regular_graph(50_000, 5, seed=5),
        description="warm-start test graph: random 5-regular, N=50000, S=32"),
}


def get_preset(name: str) -> Preset:
    return PRESETS[name]
