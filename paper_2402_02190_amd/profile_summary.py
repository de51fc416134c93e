"""Short markdown summaries of rocprofv3 kernel traces for profiles/.

    python -m paper_2402_02190_amd.profile_summary steps --trace DIR --bench BENCH_JSON \\
        --title "..." --command "..." --out FILE
    python -m paper_2402_02190_amd.profile_summary sweep --trace DIR --bench SWEEP_JSON \\
        --command "..." --out FILE

``steps``: the per-kernel table of ``rocprofv3 --kernel-trace --stats`` over a
``bench.py`` run, the bench line's dominant family and its kernel-trace average
over the eager profiled launches.  ``sweep``: the loss / aggregation size sweep
of ``bench.py --loss-sweep`` with each size's kernel-trace average.
"""

from __future__ import annotations

import argparse
import csv
import glob
import json
import os
from collections import defaultdict

from .traffic import kernel_pattern


def _find(d: str, suffix: str) -> str:
    paths = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not paths:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return paths[0]


def _json_line(path: str) -> dict:
    with open(path) as f:
        return json.loads([line for line in f if line.startswith("{")][-1])


def short(name: str) -> str:
    for a in ("cpra::(anonymous namespace)::", "cpra::gemmk::", "(cpra::gemmk::LaunchArgs)",
              "(cpra::(anonymous namespace)::LaunchArgs)", "(cpra::(anonymous namespace)::AggArgs)",
              "(cpra::(anonymous namespace)::LossArgs)", "(cpra::(anonymous namespace)::AdamArgs)",
              "void "):
        name = name.replace(a, "")
    return name


def steps(trace_dir: str, bench_json: str, title: str, command: str, out: str) -> str:
    with open(_find(trace_dir, "kernel_stats.csv")) as f:
        rows = list(csv.DictReader(f))
    b = _json_line(bench_json)
    keep = [r for r in rows if not ("spin_kernel" in r["Name"] or "at::native" in r["Name"]
                                   or "rocclr" in r["Name"])]
    tot = sum(float(r["TotalDurationNs"]) for r in keep)
    lines = [f"# {title}", "",
             "Command (repository root, one MI355X; `{out}` is a scratch directory):", "",
             f"    {command}", "",
             "`rocprofv3 --stats` kernel summary (all calls of the run: autotune-free warm-up, timed "
             "replayed steps and profiled steps; host-side sleep and torch fill kernels omitted):", "",
             "| kernel | calls | average us | min us | max us | % of library kernel time |",
             "|---|---|---|---|---|---|"]
    for r in keep:
        lines.append(f"| `{short(r['Name'])[:80]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{100.0 * float(r['TotalDurationNs']) / tot:.1f} |")
    rl = b.get("roofline", {})
    lines += ["", f"bench.py of the same build (JSON line): {b['ms_per_step'] * 1e3:.1f} us/step, value "
              f"{b['value']:.4g} head·edges/s; dominant kernel family `{rl.get('kernel')}` at "
              f"{rl.get('avg_us', 0):.1f} us average (HIP events), {rl.get('achieved', 0):.1f} "
              f"{rl.get('unit', '')} = {100 * rl.get('frac', 0):.1f}% of peak."]
    fam = rl.get("kernel", "")
    trace = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if fam and trace:
        rx = kernel_pattern(fam)
        pat = rx.pattern.replace("\\d+", "*").replace("\\", "")
        with open(trace[0]) as f:
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                 for r in csv.DictReader(f) if rx.search(r["Kernel_Name"])]
        n = int(rl.get("launches", 0))
        if n and len(d) >= n:
            lines += ["", f"Dominant family `{fam}` = `{pat}`: rocprofv3 kernel-trace average over the {n} "
                      f"launches of the profiled eager steps (the launches bench.py times with HIP events) = "
                      f"{sum(d[-n:]) / n:.1f} us; over the {len(d) - n} launches of the replayed/warm-up steps "
                      f"= {sum(d[:-n]) / max(1, len(d) - n):.1f} us (the profiled eager steps run on one "
                      f"stream; the replayed steps run the weight-gradient GEMMs on a second stream, beside "
                      f"the input-gradient GEMMs). The HIP-event average ({rl.get('avg_us', 0):.1f} us) "
                      f"also contains the event packets' own latency around each launch, so the reported "
                      f"achieved rate is a lower bound."]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return text


def _sweep_kernel(name: str):
    if "k_loss<" in name:
        return "loss_fwd_bwd"
    if "k_aggregate<" in name and "false>" in name:
        return "aggregate"
    return None


def sweep(trace_dir: str, sweep_json: str, command: str, out: str) -> str:
    rows = _json_line(sweep_json)["rows"]
    with open(_find(trace_dir, "kernel_trace.csv")) as f:
        tr = list(csv.DictReader(f))
    by = defaultdict(lambda: defaultdict(list))  # kernel -> grid -> durations
    order = defaultdict(list)  # grid sizes in order of first appearance (sizes run in order)
    for r in tr:
        k = _sweep_kernel(r["Kernel_Name"])
        if k is None:
            continue
        g = int(r.get("Grid_Size") or r["Grid_Size_X"])
        by[k][g].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        if g not in order[k]:
            order[k].append(g)
    lines = ["# Fused loss kernel and mean-aggregation SpMM vs graph size (near-20-regular random graphs, "
             "S = 64)", "", "Command (repository root, one MI355X; `{out}` is a scratch directory):", "",
             f"    {command}", "",
             "Graphs: `random_permutation_graph(N, 20)` (union of 10 random permutations, duplicates dropped), "
             "N from the 100,000-node workload up to 4,000,000 nodes (Z, P, dZ 1 GB each; well past the 256 MB "
             "Infinity Cache). Z ~ N(0, 2^2), MIS with lambda = logspace(-1, 1, 64), gamma = 0.05, P "
             "precomputed as in the training step.", "",
             "| N | nnz | kernel | event avg us | rocprof avg us | compulsory GB/s | frac of 8 TB/s | "
             "gathered GB/s (4 nnz S B) |", "|---|---|---|---|---|---|---|---|"]
    for i, r in enumerate(rows):
        for k in ("loss_fwd_bwd", "aggregate"):
            e = r[k]
            g = order[k][i] if i < len(order.get(k, [])) else None
            ds = by[k][g] if g is not None else []
            rp = sum(ds) / len(ds) if ds else float("nan")
            lines.append(f"| {r['n']:,} | {r['nnz']:,} | `{k}` | {e['avg_us']:.1f} | {rp:.1f} | "
                         f"{e['compulsory_GBps']:.0f} | {e['frac_hbm_peak']:.3f} | {e['gather_GBps']:.0f} |")
    lines += ["", "rocprof averages are over every dispatch of that kernel at that size (warm-up included), "
              "matched by grid size in order of appearance. The compulsory-byte rate (Z and P read once, dZ "
              "written, CSR) stays near 0.7-1.2 TB/s at every size because the kernel's real traffic is the "
              "neighbour gather, 4 nnz S bytes (512 MB at N = 100,000), served from the Infinity Cache below "
              "~256 MB and from HBM above. Counter passes on the 100,000-node training step give the same "
              "picture: `profiles/aggregate_c4_traffic.md` and `profiles/loss_fwd_bwd_c4_traffic.md`."]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return text


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    a1 = sub.add_parser("steps")
    a2 = sub.add_parser("sweep")
    for a in (a1, a2):
        a.add_argument("--trace", required=True, help="rocprofv3 output directory (-d)")
        a.add_argument("--bench", required=True, help="the bench.py JSON line of the same run")
        a.add_argument("--command", required=True)
        a.add_argument("--out", required=True)
    a1.add_argument("--title", required=True)
    args = ap.parse_args(argv)
    if args.what == "steps":
        steps(args.trace, args.bench, args.title, args.command, args.out)
    else:
        sweep(args.trace, args.bench, args.command, args.out)


if __name__ == "__main__":
    main()
