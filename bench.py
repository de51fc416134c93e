#!/usr/bin/env python3
"""Throughput of the CPRA training step on one MI355X.

A step is one full pass of the hot path over the workload: GNN forward,
sigmoid, the fused relaxed loss and its gradient, the hand-written backward
and Adam over every parameter (embedding included).  Steps are replayed
from a captured HIP graph; gamma follows the annealing schedule on the
device, so every timed step is a real training step.

Default workload (the 10,000-node configuration the throughput metric is
quoted on): MIS on a seeded random 5-regular graph (N = 10,000, 25,000
edges), 2-layer GraphSAGE with hidden width 256, S = 100 heads with
lambda_s = logspace(-1, 1, 100), alpha = 2, gamma -2 -> +0.1 over 5000
steps, Adam lr 1e-3, FP32.  value = S * |E| / seconds per step.

Besides the JSON line's throughput, the run measures per-kernel durations
with HIP events (the library's profiler: an event pair around every kernel
of eager steps queued behind a GPU sleep, so they run back to back), reports the dominant
kernel against its roofline, and times the FP64 CPU oracle on a bounded
sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
METRIC = "head·edges/s per CPRA step; time-to-target MIS size vs plain form"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name: str):
    from workloads import get_preset, init_params
    pr = get_preset(name)
    t0 = time.time()
    g = pr.graph()
    log(f"[bench] workload {name}: n={g.n} edges={g.n_edges} graphs={g.n_graphs} "
        f"({time.time() - t0:.1f}s to generate)")
    params = init_params(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S, seed=2024)
    return pr, g, params


def make_solver(pr, g, params):
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem=pr.problem, layer_kind=pr.layer_kind, n_layers=pr.n_layers,
                     hidden=pr.hidden, S=pr.S, alpha=pr.alpha, nu=pr.nu,
                     gamma_start=pr.gamma_start, gamma_end=pr.gamma_end, T=pr.T, lr=pr.lr,
                     recompute=pr.recompute)
    sol = CPRASolver(dg, cfg, pr.lam)
    sol.load_params(params)
    return sol


def roofline_entry(name, stats, workload):
    """The kernel family's achieved rate from the profiler (algorithmic work per
    launch / average launch time) and, when a counter record for this kernel
    source and workload exists under profiles/, its measured HBM bytes per launch."""
    from paper_2402_02190_amd.traffic import load_traffic
    launches, ms, flops, nbytes = stats
    avg_s = ms / 1e3 / launches
    try:
        traffic = load_traffic(name, workload)
    except ValueError:
        traffic = None
    if flops > 0:
        achieved = flops / launches / avg_s / 1e12
        return {"kernel": name, "bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                "avg_us": avg_s * 1e6, "launches": launches,
                "work_per_launch": flops / launches, "work_unit": "FLOP"}
    achieved = nbytes / launches / avg_s / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "avg_us": avg_s * 1e6, "launches": launches,
            "work_per_launch": nbytes / launches, "work_unit": "B"}


def default_tuning_file(workload: str):
    p = os.path.join(ROOT, "paper_2402_02190_amd", "tuning", f"{workload.lower()}_mi355x.json")
    return p if os.path.exists(p) else None


def pmc_pass(sol, steps: int):
    """The short deterministic run that the counter passes profile: a calibration
    copy of a known size, then eager training steps."""
    import torch
    from paper_2402_02190_amd.traffic import CALIBRATION_BYTES
    src = torch.empty(CALIBRATION_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    for _ in range(steps):
        sol.step()
    torch.cuda.synchronize()
    log(f"[bench] pmc pass: calibration copy + {steps} steps done")


def cpu_baseline(pr, g, params, seconds: float):
    """The FP64 oracle's training step timed on the host, on a bounded number of steps."""
    from oracle import gnn as ognn
    from oracle import train as otrain
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    p64 = ognn.to_f64(params)
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    cfg = otrain.StepConfig(problem=pr.problem, lam=None if pr.lam is None else pr.lam.astype(np.float64),
                            alpha=pr.alpha, nu=pr.nu, lr=pr.lr)
    opt = otrain.AdamState(p64)
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        gamma = otrain.gamma_at(len(times), pr.T, pr.gamma_start, pr.gamma_end)
        _, _, _, grads = otrain.loss_and_grads(p64, M, g, cfg, gamma)
        opt.step(p64, grads, cfg)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > seconds or len(times) >= 200:
            break
    t_step = float(np.median(times))
    return {"value": pr.S * g.n_edges / t_step, "unit": "head·edges/s", "cores": int(cores),
            "kind": "oracle", "ms_per_step": t_step * 1e3,
            "sample": f"{len(times)} full FP64 oracle training steps (forward, loss, gradient, Adam) "
                      f"of the same workload; median step time"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning-file", default=None,
                    help="GEMM tuning table: loaded if it exists, else written after autotuning "
                         "(default: the committed MI355X table of the workload, if any)")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="run only the short sequence the HBM counter passes profile")
    args = ap.parse_args()
    if args.tuning_file is None and not args.no_autotune:
        args.tuning_file = default_tuning_file(args.workload)
    if args.gpus != 1:
        log("bench.py measures one GPU: this build has no multi-GPU path (each GPU would run its "
            "own share of graphs; see the sharding note in DESIGN.md). Run with --gpus 1.")
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    from paper_2402_02190_amd import api

    pr, g, params = build_workload(args.workload)
    sol = make_solver(pr, g, params)
    torch.cuda.synchronize()
    log(f"[bench] params={sol.n_params} workspace={sol.ws.numel() / 2**20:.1f} MiB")

    # GEMM tile shapes: load a saved tuning table, or autotune on this workload's
    # shapes (one real training step) and save the table
    if args.tuning_file and os.path.exists(args.tuning_file):
        with open(args.tuning_file) as f:
            for e in json.load(f):
                api.autotune_set(e["key"], e["cfg"], e["splits"])
        log(f"[bench] loaded GEMM tuning table {args.tuning_file}")
    elif not args.no_autotune:
        table = sol.autotune()
        for key, choice, us, hus in table:
            log(f"[bench] autotune {key:40s} -> {choice:26s} {us:8.2f} us (heuristic {hus:8.2f} us)")
        if args.tuning_file:
            with open(args.tuning_file, "w") as f:
                json.dump(api.autotune_table(), f, indent=1)
    if args.pmc_pass:
        pmc_pass(sol, 5)
        sol.close()
        return
    # warm-up: capture once, replay W steps
    sol.capture()
    sol.replay(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")

    # timed region: K replayed steps, synchronised on both sides
    stream = sol._stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        api.graph_launch(sol._graph, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sol.t += args.steps
    ms_event = ev0.elapsed_time(ev1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    value = pr.S * g.n_edges / (ms_per_step / 1e3)
    log(f"[bench] {args.steps} steps: {ms_per_step:.4f} ms/step wall ({ms_event:.4f} ms by events)")
    terms = sol.terms_host()
    if not np.all(np.isfinite(terms)):
        raise RuntimeError("non-finite loss terms")

    result = {
        "metric": METRIC, "value": value, "unit": "head·edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{pr.name}: {pr.description}", "n_nodes": g.n,
                   "n_edges": g.n_edges, "n_graphs": g.n_graphs, "S": pr.S,
                   "layer": pr.layer_kind, "layers": pr.n_layers, "hidden": pr.hidden,
                   "problem": pr.problem, "hip_graph_replay": True,
                   "autotuned_gemm": not args.no_autotune,
                   "ms_per_step_events": ms_event},
    }

    if not args.no_profile:
        # per-kernel durations: eager steps with an event pair around every kernel,
        # queued behind a GPU sleep so that the host runs ahead of the GPU and the
        # kernels execute back to back as in the replayed graph
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            torch.cuda._sleep(int(2.4e9 * 0.004 * args.profile_steps))  # ~4 ms per step
            api.profile_begin()
            for _ in range(args.profile_steps):
                sol.step(stream)
            api.profile_stop()
        torch.cuda.synchronize()
        stats = api.profile_end()
        total = sum(v[1] for v in stats.values())
        kernels = {k: {"launches": v[0], "avg_us": v[1] * 1e3 / v[0],
                       "share": v[1] / total} for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}
        dom = max(stats, key=lambda k: stats[k][1])
        result["roofline"] = roofline_entry(dom, stats[dom], pr.name)
        if "loss_fwd_bwd" in stats:
            result["roofline_loss"] = roofline_entry("loss_fwd_bwd", stats["loss_fwd_bwd"], pr.name)
        result["kernels"] = kernels
        log(f"[bench] dominant kernel {dom}: {json.dumps(result['roofline'])}")
        for k, v in kernels.items():
            log(f"[bench]   {k:28s} {v['launches']:5d} launches {v['avg_us']:9.2f} us avg "
                f"{100 * v['share']:5.1f}%")

    if rank == 0 and not args.no_cpu_baseline:
        log(f"[bench] timing the FP64 oracle for up to {args.cpu_seconds:.0f}s ...")
        result["cpu_baseline"] = cpu_baseline(pr, g, params, args.cpu_seconds)
        log(f"[bench] cpu baseline: {result['cpu_baseline']}")

    sol.close()
    if rank == 0:
        print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
