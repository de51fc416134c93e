"""K instances of one structure solved together, one per head, against the same
K instances solved one at a time (the multi-instance use of CPRA: Sec. 3.1
lets every head carry its own instance, and the multi-instance appendix solves
27 instances of one structure in a single run instead of 27 runs).

The instances are synthetic (the appendix's matching instances are not
available): K weightings of one random regular graph, from
``workloads.instance_edge_weights`` -- MaxCut with integer weights U{1..4}, or
MIS with each instance keeping a random 70% of the edges.

  together: one network with K heads, head k on instance k (per-head edge
            weights), one run of T steps;
  one by one: K runs of T steps, each a one-head network on its own instance
            (for MIS, on the graph of that instance's edges).

Both arms use the same kernels, schedule and optimiser, with GEMM plans tuned
outside the clock; the clock covers the training steps of every run (the joint
run may be given a longer schedule, ``together_T``, to compare at a smaller
time ratio).  Each instance is scored by its head's rounded solution: the cut
weight (MaxCut) or the independent-set size, 0 when infeasible (MIS).

    python -m paper_2402_02190_amd.multiinstance [--problem maxcut] [--instances 27]
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import api
from .solver import CPRAConfig, CPRASolver


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _score(ev, problem: str) -> np.ndarray:
    """Per head: the cut weight (MaxCut) or the set size of a feasible head (MIS)."""
    if problem == "maxcut":
        return ev["wvalue"][0].astype(np.float64)
    return np.where(ev["violations"][0] == 0, ev["value"][0], 0).astype(np.float64)


def _train(dg, cfg, lam, params, T, edge_weight=None):
    sol = CPRASolver(dg, cfg, lam, edge_weight=edge_weight)
    sol.load_params(params)
    sol.autotune()           # one tuned step outside the clock (reuses entries already tuned) ...
    sol.load_params(params)  # ... then training starts from the same parameters
    sol.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.replay(T)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    ev = sol.evaluate()
    sol.close()
    return ev, seconds


def run(problem: str = "maxcut", instances: int = 27, n: int = 2000, degree: int = 3,
        hidden: int = 64, T: int = 2000, seed: int = 0, together_T: int = None):
    from workloads import csr_from_edges, init_params, instance_edge_weights, random_regular_graph
    g = random_regular_graph(n, degree, seed + 1)
    K = instances
    if problem == "maxcut":
        W = instance_edge_weights(g, K, seed + 2, "integer")
        lam = None
    else:
        W = instance_edge_weights(g, K, seed + 2, "unit", drop=0.3)
        lam = np.full(K, 2.0, np.float32)
    base = dict(problem=problem, layer_kind="gcn", n_layers=2, hidden=hidden, alpha=2, nu=0.0,
                gamma_start=-2.0, gamma_end=0.1, T=T, lr=1e-3)
    api.autotune_reset()
    # together: K heads, head k on instance k
    dg = api.DeviceGraph.from_csr(g)
    Tj = T if together_T is None else together_T
    cfg = CPRAConfig(S=K, **dict(base, T=Tj))
    ev, t_together = _train(dg, cfg, lam, init_params("gcn", n, 2, hidden, K, seed=seed), Tj, W)
    together = _score(ev, problem)
    # one by one: a one-head network per instance, on that instance's own graph
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    upper = rows < g.col_idx
    single = np.zeros(K)
    t_single = 0.0
    cfg1 = CPRAConfig(S=1, **base)
    for k in range(K):
        keep = upper & (W[:, k] != 0)
        gk = csr_from_edges(n, rows[keep], g.col_idx[keep],
                            W[keep, k] if problem == "maxcut" else None)
        dgk = api.DeviceGraph.from_csr(gk)
        ev1, sec = _train(dgk, cfg1, None if lam is None else lam[:1],
                          init_params("gcn", n, 2, hidden, 1, seed=seed + 100 + k), T)
        single[k] = _score(ev1, problem)[0]
        t_single += sec
    api.autotune_reset()
    res = {"problem": problem, "instances": K, "nodes": n, "degree": degree, "T": T,
           "together_T": Tj, "seed": seed,
           "together_seconds": t_together, "one_by_one_seconds": t_single,
           "speedup": t_single / t_together,
           "mean_score_together": float(together.mean()), "mean_score_one_by_one": float(single.mean()),
           "together_better": int((together > single).sum()), "equal": int((together == single).sum()),
           "one_by_one_better": int((together < single).sum())}
    log(f"[multi-instance] {json.dumps(res)}")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description="K instances together (one per head) vs one by one")
    ap.add_argument("--problem", default="maxcut", choices=["maxcut", "mis"])
    ap.add_argument("--instances", type=int, default=27)
    ap.add_argument("--nodes", type=int, default=2000)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--hidden", type=int, default=64)
    ap.add_argument("--T", type=int, default=2000)
    ap.add_argument("--together-T", type=int, default=None,
                    help="schedule length of the joint run (default: --T)")
    ap.add_argument("--seeds", type=int, nargs="+", default=[0])
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = [run(a.problem, a.instances, a.nodes, a.degree, a.hidden, a.T, s, a.together_T)
           for s in a.seeds]
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
