"""Two-stage S' -> S training on weighted-MIS tasks (the last paragraph of
Sec. 3.1 and the two-stage appendix), on the library's kernels.

Tasks: S weighted-MIS instances on one graph; head s minimises
-sum_i w_is x_i + lam * sum_{(i,j) in E} x_i x_j with its own weight vector w_s
(seeded U(0, 1); the paper does not state the distribution) and lam = 2 > max w,
so the penalty minimisers are independent sets.

  stage 1 (warm-up): S' heads on the first S' tasks, gamma -2 -> +2 over T1
          steps, stopped once the annealing term per entry falls below eps;
  stage 2 (fine-tune): the encoder (embedding and every layer but the last)
          frozen, a fresh S-way output layer trained alone for up to T2 steps,
          same stopping rule; the frozen prefix's activations are computed once
          and reused.  The printed fine-tune schedule ("0.1 -> 0") leaves a fresh
          random head without a smoothing phase; the default here anneals
          gamma -2 -> +2 like the warm-up (both are options);
  baseline: S heads from scratch with stage 1's schedule.

    python -m paper_2402_02190_amd.twostage [--n 1000 --d 5 --S1 200 --S 500 ...]
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


def _run(sol: CPRASolver, T: int, eps: float, K: int = 50):
    """Steps until T or the stopping rule; returns (steps, seconds)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = sol.run_until_binary(T, eps, K)
    torch.cuda.synchronize()
    return done, time.perf_counter() - t0


def _quality(sol: CPRASolver):
    sol.forward()
    ev = sol.evaluate()
    feas = ev["violations"][0] == 0
    w = ev["wvalue"][0]
    return {"feasible": int(feas.sum()), "heads": int(feas.size),
            "mean_weight_feasible": float(w[feas].mean()) if feas.any() else 0.0,
            "mean_weight_all": float(np.where(feas, w, 0.0).mean())}


def run(n: int = 1000, d: int = 5, S1: int = 200, S: int = 500, hidden: int = 256,
        T1: int = 8000, T2: int = 2000, eps: float = 1e-4, lam: float = 2.0, seed: int = 0,
        ft_gamma=(-2.0, 2.0)):
    from workloads import init_params, random_regular_graph
    g = random_regular_graph(n, d, seed=seed + 100)
    dg = api.DeviceGraph.from_csr(g)
    W = np.random.default_rng(seed + 7).uniform(0.0, 1.0, (n, S)).astype(np.float32)
    base = dict(problem="mis", layer_kind="sage", n_layers=2, hidden=hidden, lr=1e-3)

    # stage 1: warm-up on the first S1 tasks
    c1 = CPRAConfig(S=S1, gamma_start=-2.0, gamma_end=2.0, T=T1, **base)
    s1 = CPRASolver(dg, c1, np.full(S1, lam, np.float32), node_weight=W[:, :S1])
    p1 = init_params("sage", n, 2, hidden, S1, seed=seed + 1)
    s1.load_params(p1)
    steps1, t1 = _run(s1, T1, eps)
    q1 = _quality(s1)
    enc = s1.unpack(s1.params)
    s1.close()
    log(f"[two-stage] warm-up: {steps1} steps, {t1:.3f} s, {q1}")

    # stage 2: frozen encoder, fresh S-way output layer
    c2 = CPRAConfig(S=S, gamma_start=ft_gamma[0], gamma_end=ft_gamma[1], T=T2, train_from_layer=1,
                    **base)
    s2 = CPRASolver(dg, c2, np.full(S, lam, np.float32), node_weight=W)
    fresh = init_params("sage", n, 2, hidden, S, seed=seed + 2)
    p2 = {"emb": enc["emb"], "layers": [enc["layers"][0], fresh["layers"][1]]}
    s2.load_params(p2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s2.step()                       # one full forward saves the frozen prefix ...
    s2.set_reuse_frozen_prefix(True)  # ... which later steps start from
    steps2, _ = _run(s2, T2 - 1, eps)
    torch.cuda.synchronize()
    t2 = time.perf_counter() - t0
    q2 = _quality(s2)
    s2.close()
    log(f"[two-stage] fine-tune: {steps2 + 1} steps, {t2:.3f} s, {q2}")

    # baseline: S heads from scratch
    c3 = CPRAConfig(S=S, gamma_start=-2.0, gamma_end=2.0, T=T1, **base)
    s3 = CPRASolver(dg, c3, np.full(S, lam, np.float32), node_weight=W)
    s3.load_params(init_params("sage", n, 2, hidden, S, seed=seed + 3))
    steps3, t3 = _run(s3, T1, eps)
    q3 = _quality(s3)
    s3.close()
    log(f"[two-stage] scratch: {steps3} steps, {t3:.3f} s, {q3}")
    return {"graph": f"random {d}-regular N={n}", "tasks": S, "warmup_tasks": S1, "lambda": lam,
            "weights": "U(0,1) per node and task, seeded", "model": f"SAGE 2x{hidden}",
            "finetune_gamma": list(ft_gamma),
            "two_stage": {"warmup_steps": steps1, "warmup_s": t1, "finetune_steps": steps2 + 1,
                          "finetune_s": t2, "total_s": t1 + t2, **q2},
            "scratch": {"steps": steps3, "seconds": t3, **q3}}


def main(argv=None):
    ap = argparse.ArgumentParser(description="two-stage S' -> S weighted-MIS experiment")
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--d", type=int, default=5)
    ap.add_argument("--S1", type=int, default=200)
    ap.add_argument("--S", type=int, default=500)
    ap.add_argument("--hidden", type=int, default=256)
    ap.add_argument("--T1", type=int, default=8000)
    ap.add_argument("--T2", type=int, default=2000)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--seeds", type=int, nargs="+", default=[0])
    ap.add_argument("--ft-gamma", type=float, nargs=2, default=[-2.0, 2.0],
                    help="fine-tune gamma schedule endpoints")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = [run(a.n, a.d, a.S1, a.S, a.hidden, a.T1, a.T2, a.eps, seed=s, ft_gamma=tuple(a.ft_gamma))
           for s in a.seeds]
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
