#!/usr/bin/env python3
"""Throughput of the CPRA training step on one MI355X.

A step is one full pass of the hot path over the workload: GNN forward,
sigmoid, the fused relaxed loss and its gradient, the hand-written backward
and Adam over every parameter (embedding included).  Steps are replayed
from a captured HIP graph; gamma follows the annealing schedule on the
device, so every timed step is a real training step.

Default workload (the largest single-graph configuration that one GPU
runs): MIS on a seeded random 20-regular graph (N = 100,000, 1,000,000
edges), 3-layer GCN with hidden width 128, S = 64 heads with
lambda_s = logspace(-1, 1, 64), alpha = 2, gamma -2 -> +0.1, Adam lr 1e-3,
FP32, layer recomputation on.  value = S * |E| / seconds per step.  The
10,000-node, 5-regular, GraphSAGE-256, S = 100 configuration is measured
after it with the same contract and reported under the key "C2".

Besides the JSON line's throughput, the run measures per-kernel durations
with HIP events (the library's profiler: an event pair around every kernel
of eager steps queued behind a GPU sleep, so they run back to back, on one
stream so that each kernel has the GPU to itself), reports the dominant
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


def build_workload(name: str, per_graph: bool = False):
    from workloads import get_preset, init_params, init_params_per_graph
    pr = get_preset(name)
    t0 = time.time()
    g = pr.graph()
    log(f"[bench] workload {name}: n={g.n} edges={g.n_edges} graphs={g.n_graphs} "
        f"({time.time() - t0:.1f}s to generate)")
    if per_graph:
        if g.n_graphs < 2:
            raise SystemExit("--per-graph-weights needs a batch of graphs (C3, C3s)")
        params = init_params_per_graph(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S,
                                       g.n_graphs, seed=2024)
    else:
        params = init_params(pr.layer_kind, g.n, pr.n_layers, pr.hidden, pr.S, seed=2024)
    return pr, g, params


FORK_ORDER = "preset"  # --fork-order: "preset", "main" (input gradient first) or "side"


def side_first(pr) -> bool:
    return pr.side_first if FORK_ORDER == "preset" else FORK_ORDER == "side"


def make_solver(pr, g, params, per_graph: bool = False, edge_weight=None):
    from paper_2402_02190_amd import api
    from paper_2402_02190_amd.solver import CPRAConfig, CPRASolver
    # capture order of the backward's forks, chosen per workload by step time (the
    # library reads the switch whenever it records a step)
    if side_first(pr):
        os.environ["CPRA_SIDE_FIRST"] = "1"
    else:
        os.environ.pop("CPRA_SIDE_FIRST", None)
    dg = api.DeviceGraph.from_csr(g)
    cfg = CPRAConfig(problem=pr.problem, layer_kind=pr.layer_kind, n_layers=pr.n_layers,
                     hidden=pr.hidden, S=pr.S, alpha=pr.alpha, nu=pr.nu,
                     gamma_start=pr.gamma_start, gamma_end=pr.gamma_end, T=pr.T, lr=pr.lr,
                     recompute=pr.recompute, per_graph_weights=per_graph)
    sol = CPRASolver(dg, cfg, pr.lam, edge_weight=edge_weight)
    sol.load_params(params)
    return sol


TIMING = "HIP events around each launch of eager steps on one stream, back to back"


def roofline_entry(name, stats, workload):
    """The kernel family's achieved rate from the profiler (algorithmic work per
    launch / average launch time) and, when a counter record for this kernel
    source and workload exists under profiles/, its measured HBM bytes per launch."""
    from paper_2402_02190_amd.traffic import load_traffic
    launches, ms, flops, nbytes, gather = stats
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
                "work_per_launch": flops / launches, "work_unit": "FLOP", "timing": TIMING}
    achieved = nbytes / launches / avg_s / 1e9
    out = {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
           "avg_us": avg_s * 1e6, "launches": launches,
           "work_per_launch": nbytes / launches, "work_unit": "B", "timing": TIMING}
    if gather > 0:
        # the neighbour rows the kernel gathers through the CSR index (4 B per entry and
        # column): what a sparse product over an expander graph streams, from the
        # Infinity Cache or HBM, beside the compulsory bytes above
        g_rate = gather / launches / avg_s / 1e9
        out["gather"] = {"bytes_per_launch": gather / launches, "achieved": g_rate,
                         "unit": "GB/s", "frac_of_hbm_peak": g_rate / PEAK_HBM_GBS}
    return out


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


def cpu_baseline(pr, g, params, seconds: float, per_graph: bool = False, edge_weight=None):
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
                            alpha=pr.alpha, nu=pr.nu, lr=pr.lr, edge_weight=edge_weight)
    opt = otrain.AdamState(p64)
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        gamma = otrain.gamma_at(len(times), pr.T, pr.gamma_start, pr.gamma_end)
        if per_graph:
            _, _, _, grads = otrain.loss_and_grads_per_graph(p64, g, cfg, gamma)
        else:
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


def loss_sweep(sizes, S: int = 64, d: int = 20, reps: int = 10):
    """The fused loss kernel (A P gather + objective + dZ) and the mean-aggregation
    SpMM alone over near-d-regular random graphs of growing N (the 100,000-node,
    20-regular, S = 64 workload and larger), timed by the library profiler: the
    compulsory-byte rate against HBM peak, and the neighbour-gather rate, which
    is what the kernel actually streams (4 nnz S bytes, cache-resident below
    the 256 MB Infinity Cache, from HBM above it)."""
    import torch
    from paper_2402_02190_amd import api
    from workloads import random_permutation_graph
    rows = []
    for n in sizes:
        t0 = time.time()
        g = random_permutation_graph(n, d, seed=1000 + n % 997)
        dg = api.DeviceGraph.from_csr(g, validate=False)
        log(f"[sweep] n={n} nnz={g.nnz} ({time.time() - t0:.1f}s to generate)")
        lam = torch.from_numpy(np.logspace(-1, 1, S).astype(np.float32)).cuda()
        lc = api.make_loss_cfg(api.MIS, S, lam, 2, 0.05, 0.0, 0, None, 0.05, 0.05, 2)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(n)
        Z = torch.randn((n, S), device="cuda", generator=gen) * 2.0
        P = torch.empty_like(Z)
        api.sigmoid(Z, P)
        dZ = torch.empty_like(Z)
        Y = torch.empty_like(Z)
        ws = torch.empty(api.loss_workspace_bytes(dg, lc), dtype=torch.uint8, device="cuda")
        for _ in range(2):  # warm-up
            api.loss_fwd_bwd(dg, lc, Z, dZ, None, ws, P=P)
            api.aggregate_mean(dg, P, Y)
        torch.cuda.synchronize()
        torch.cuda._sleep(int(2.4e9 * 0.002 * reps))
        api.profile_begin()
        for _ in range(reps):
            api.loss_fwd_bwd(dg, lc, Z, dZ, None, ws, P=P)
        for _ in range(reps):
            api.aggregate_mean(dg, P, Y)
        api.profile_stop()
        torch.cuda.synchronize()
        st = api.profile_end()
        row = {"n": n, "nnz": g.nnz, "S": S}
        gather = 4.0 * g.nnz * S
        for name in ("loss_fwd_bwd", "aggregate"):
            la, ms, _, by, _ = st[name]
            t = ms / 1e3 / la
            row[name] = {"avg_us": t * 1e6, "compulsory_bytes": by / la,
                         "compulsory_GBps": by / la / t / 1e9,
                         "frac_hbm_peak": by / la / t / 1e9 / PEAK_HBM_GBS,
                         "gather_bytes": gather, "gather_GBps": gather / t / 1e9}
        log(f"[sweep] n={n}: loss {row['loss_fwd_bwd']['avg_us']:.1f} us "
            f"({row['loss_fwd_bwd']['compulsory_GBps']:.0f} GB/s compulsory, "
            f"{row['loss_fwd_bwd']['gather_GBps']:.0f} GB/s gathered); aggregate "
            f"{row['aggregate']['avg_us']:.1f} us ({row['aggregate']['compulsory_GBps']:.0f} GB/s, "
            f"{row['aggregate']['gather_GBps']:.0f} GB/s gathered)")
        rows.append(row)
        del Z, P, dZ, Y, ws, dg
        torch.cuda.empty_cache()
    return rows


WARM_WEIGHTS = os.path.join(ROOT, "paper_2402_02190_amd", "weights", "warmstart_mis_rrg.npz")


def time_to_target(seeds=(0, 1, 2, 3, 4), n: int = 50_000, d: int = 5):
    """The second half of the metric on the 50,000-node warm-start workload: wall
    time until the best feasible head (decoded every 50 steps) reaches a fraction
    of the plain method's final MIS size, for the plain cold-start run, the
    warm-started run (learned network, committed weights) and the same short
    schedule without the network."""
    from paper_2402_02190_amd.warmstart_train import evaluate
    if not os.path.exists(WARM_WEIGHTS):
        return None
    s = evaluate(WARM_WEIGHTS, n=n, degrees=(d,), seeds=seeds, T=3000, K=50,
                 warm_gamma_start=-0.5, warm_T=1000, decay_steps=500)
    return {"workload": f"C5: random {d}-regular N={n}, MIS, S=32, GCN 2x64, seeds {list(seeds)}",
            "target": "plain (cold-start) CPRA's final best feasible MIS size after 3000 steps",
            "plain": "gamma -2 -> 0.1 over 3000 steps",
            "warm": "z_offset = learned BF16 network output, fading to 0 over 500 steps; "
                    "gamma -0.5 -> 0.1 over 1000 steps (inference time included)",
            "control": "the warm arm's schedule without the network",
            "median_seconds_to_fraction": s["curves"],
            "final_over_target": {"warm": s["mean_warm_final_over_target"],
                                  "control": s["mean_control_final_over_target"]}}


def step_benchmark(workload: str, args, per_graph: bool, instances, instance_drop: float,
                   tuning_file, profile: bool):
    """Build the workload, load (or tune) the GEMM plans, replay the captured step
    args.steps times after args.warmup warm-up steps, and profile eager steps.
    Returns (result dict without the host-side legs, (pr, g, params, W))."""
    import torch
    from paper_2402_02190_amd import api

    label = workload + ("_pergraph" if per_graph else "") + ("_instances" if instances else "")
    pr, g, params = build_workload(workload, per_graph)
    W = None
    if instances:
        from workloads import instance_edge_weights
        W = instance_edge_weights(g, pr.S, 2025, instances, instance_drop)
    sol = make_solver(pr, g, params, per_graph, W)
    torch.cuda.synchronize()
    log(f"[bench] {workload}: params={sol.n_params} workspace={sol.ws.numel() / 2**20:.1f} MiB")

    # GEMM tile shapes: load a saved tuning table, or autotune on this workload's
    # shapes (one real training step) and save the table
    api.autotune_reset()
    if tuning_file and os.path.exists(tuning_file):
        with open(tuning_file) as f:
            for e in json.load(f):
                api.autotune_set(e["key"], e["cfg"], e["splits"])
        log(f"[bench] loaded GEMM tuning table {tuning_file}")
    elif not args.no_autotune:
        table = sol.autotune()
        for key, choice, us, hus in table:
            log(f"[bench] autotune {key:40s} -> {choice:26s} {us:8.2f} us (heuristic {hus:8.2f} us)")
        if tuning_file:
            with open(tuning_file, "w") as f:
                json.dump(api.autotune_table(), f, indent=1)
    if args.pmc_pass:
        pmc_pass(sol, 5)
        sol.close()
        return None, (pr, g, params, W)
    # warm-up: capture once (one step, and args.graph_steps steps in a second graph),
    # replay W steps
    sol.capture(steps_per_graph=args.graph_steps)
    sol.replay(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] {workload}: warmup {args.warmup} steps done")

    # timed region: K replayed steps, synchronised on both sides
    stream = sol._stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # events at the ends of five equal chunks of the K steps (same stream, no sync):
    # the median chunk is reported beside the K-step figure
    # (a chunk ends after the first launch that reaches its share of the steps)
    plan = sol.launch_plan(args.steps)
    n_chunks = 5 if len(plan) >= 5 else 1
    targets = [args.steps * c // n_chunks for c in range(1, n_chunks)]
    chunk_ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_chunks - 1)]
    chunk_steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    done = 0
    for gr, ns in plan:
        api.graph_launch(gr, stream)
        done += ns
        if len(chunk_steps) < n_chunks - 1 and done >= targets[len(chunk_steps)]:
            chunk_ev[len(chunk_steps)].record(stream)
            chunk_steps.append(done)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sol.t += args.steps
    ms_event = ev0.elapsed_time(ev1) / args.steps
    marks = [ev0] + chunk_ev + [ev1]
    ends = [0] + chunk_steps + [args.steps]
    chunk_ms = sorted(marks[c].elapsed_time(marks[c + 1]) / (ends[c + 1] - ends[c])
                      for c in range(n_chunks))
    ms_median_chunk = chunk_ms[n_chunks // 2]
    ms_per_step = wall * 1e3 / args.steps
    value = pr.S * g.n_edges / (ms_per_step / 1e3)
    log(f"[bench] {workload}: {args.steps} steps: {ms_per_step:.4f} ms/step wall "
        f"({ms_event:.4f} ms by events)")
    terms = sol.terms_host()
    if not np.all(np.isfinite(terms)):
        raise RuntimeError("non-finite loss terms")

    result = {
        "metric": METRIC, "value": value, "unit": "head·edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{pr.name}: {pr.description}"
                               + ("; one network per graph" if per_graph else "")
                               + (f"; one instance per head ({instances} edge weights, "
                                  f"{instance_drop:g} left out)" if instances else ""),
                   "n_nodes": g.n,
                   "n_edges": g.n_edges, "n_graphs": g.n_graphs, "S": pr.S,
                   "layer": pr.layer_kind, "layers": pr.n_layers, "hidden": pr.hidden,
                   "problem": pr.problem, "recompute": bool(pr.recompute),
                   "backward_fork_order": "side work first" if side_first(pr) else "input gradient first",
                   "hip_graph_replay": True, "steps_per_graph": args.graph_steps,
                   "per_graph_weights": bool(per_graph),
                   "autotuned_gemm": not args.no_autotune,
                   "ms_per_step_events": ms_event,
                   "ms_per_step_median_of_5_chunks": ms_median_chunk},
    }

    if profile:
        # per-kernel durations: eager steps with an event pair around every kernel,
        # queued behind a GPU sleep so that the host runs ahead of the GPU and the
        # kernels execute back to back as in the replayed graph, all on one stream
        # (the side-stream overlap of the timed steps would have two kernels share
        # the CUs and each event pair time both)
        torch.cuda.synchronize()
        overlap = os.environ.get("CPRA_OVERLAP")
        os.environ["CPRA_OVERLAP"] = "0"
        try:
            with torch.cuda.stream(stream):
                torch.cuda._sleep(int(2.4e9 * 0.004 * args.profile_steps))  # ~4 ms per step
                api.profile_begin()
                for _ in range(args.profile_steps):
                    sol.step(stream)
                api.profile_stop()
            torch.cuda.synchronize()
        finally:
            if overlap is None:
                os.environ.pop("CPRA_OVERLAP", None)
            else:
                os.environ["CPRA_OVERLAP"] = overlap
        stats = api.profile_end()
        total = sum(v[1] for v in stats.values())
        kernels = {k: {"launches": v[0], "avg_us": v[1] * 1e3 / v[0],
                       "share": v[1] / total} for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}
        dom = max(stats, key=lambda k: stats[k][1])
        result["roofline"] = roofline_entry(dom, stats[dom], label)
        if "loss_fwd_bwd" in stats:
            result["roofline_loss"] = roofline_entry("loss_fwd_bwd", stats["loss_fwd_bwd"], label)
        result["kernels"] = kernels
        log(f"[bench] {workload}: dominant kernel {dom}: {json.dumps(result['roofline'])}")
        for k, v in kernels.items():
            log(f"[bench]   {k:28s} {v['launches']:5d} launches {v['avg_us']:9.2f} us avg "
                f"{100 * v['share']:5.1f}%")
    sol.close()
    api.autotune_reset()
    return result, (pr, g, params, W)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the second measurement (the 10,000-node C2 step) after the C4 one")
    ap.add_argument("--per-graph-weights", action="store_true",
                    help="batched workloads: one network per graph instead of one shared network")
    ap.add_argument("--instances", default=None, choices=["uniform", "signed", "integer", "unit"],
                    help="one instance per head: per-head edge weights of this kind on the "
                         "workload's graph (seeded; see workloads.instance_edge_weights)")
    ap.add_argument("--instance-drop", type=float, default=0.0,
                    help="with --instances: fraction of (edge, head) pairs left out")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-time-to-target", action="store_true")
    ap.add_argument("--ttt-seeds", type=int, default=5,
                    help="seeds of the time-to-target comparison (graphs and initialisations)")
    ap.add_argument("--tuning-file", default=None,
                    help="GEMM tuning table: loaded if it exists, else written after autotuning "
                         "(default: the committed MI355X table of the workload, if any)")
    ap.add_argument("--fork-order", choices=("preset", "main", "side"), default="preset",
                    help="capture order at the backward's forks: the workload preset's choice, the "
                         "input gradient first, or the side-stream work first")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="training steps recorded in one HIP graph for the replays (one graph "
                         "launch per that many steps; a one-step graph runs the remainder)")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="run only the short sequence the HBM counter passes profile")
    ap.add_argument("--loss-sweep", type=int, nargs="*", default=None, metavar="N",
                    help="instead of the step benchmark: time the fused loss kernel and the "
                         "aggregation alone on near-20-regular graphs of these sizes, S = 64")
    args = ap.parse_args()
    global FORK_ORDER
    FORK_ORDER = args.fork_order
    if args.loss_sweep is not None:
        sizes = args.loss_sweep or [100_000, 400_000, 1_000_000, 4_000_000]
        rows = loss_sweep(sizes)
        print(json.dumps({"sweep": "loss_fwd_bwd and aggregate, near-20-regular random graphs, S=64",
                          "peak_hbm_GBps": PEAK_HBM_GBS, "rows": rows}), flush=True)
        return
    if args.gpus != 1:
        log("bench.py measures one GPU: the library runs one process on one GPU (a batch of graphs "
            "would shard at graph boundaries, one share per GPU). Run with --gpus 1.")
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    tuning = args.tuning_file
    if tuning is None and not args.no_autotune:
        # the GEMMs do not depend on the instances
        tuning = default_tuning_file(args.workload + ("_pergraph" if args.per_graph_weights else ""))

    result, (pr, g, params, W) = step_benchmark(args.workload, args, args.per_graph_weights,
                                                 args.instances, args.instance_drop, tuning,
                                                 not args.no_profile)
    if result is None:
        return

    if args.workload == "C4" and not (args.no_c2 or args.per_graph_weights or args.instances):
        # the 10,000-node configuration, same contract (its own committed GEMM plans)
        c2, _ = step_benchmark("C2", args, False, None, 0.0,
                               None if args.no_autotune else default_tuning_file("C2"),
                               not args.no_profile)
        result["C2"] = {k: c2[k] for k in ("value", "ms_per_step", "config", "roofline",
                                             "roofline_loss") if k in c2}

    if rank == 0 and not args.no_time_to_target:
        log("[bench] time to target: cold vs warm start on the 50,000-node graph ...")
        ttt = time_to_target(seeds=tuple(range(args.ttt_seeds)))
        if ttt is not None:
            result["time_to_target"] = ttt
            log(f"[bench] time to target: {json.dumps(ttt['median_seconds_to_fraction'])}")

    if rank == 0 and not args.no_cpu_baseline:
        log(f"[bench] timing the FP64 oracle for up to {args.cpu_seconds:.0f}s ...")
        result["cpu_baseline"] = cpu_baseline(pr, g, params, args.cpu_seconds, args.per_graph_weights,
                                              W)
        log(f"[bench] cpu baseline: {result['cpu_baseline']}")

    if rank == 0:
        print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
