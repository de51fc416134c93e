"""What bounds a memory-side kernel: occupancy, waiting and L2 hits from
rocprofv3 counter passes.

    rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY \\
        SQ_ACTIVE_INST_ANY SQ_INSTS_VMEM_RD GRBM_GUI_ACTIVE \\
        --output-format csv -d A -o run -- python bench.py --pmc-pass ...
    rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --output-format csv -d B -o run -- python bench.py --pmc-pass ...
    python -m paper_2402_02190_amd.wave_counters --dir A --dir B --kernel k_loss \\
        --workload C2 --out FILE --command "..."

Per kernel (dispatches whose name contains ``--kernel``), averaged over its
dispatches, with each dispatch's own timestamps:

* waves per SIMD resident on average = 4 x SQ_WAVE_CYCLES / (SIMDs x clock x
  duration): the SQ's wave-cycle counters count in units of four cycles (a
  one-wave-per-SIMD GEMM launch of 1.53 blocks per CU on average reads 0.71);
* waves launched per SIMD = SQ_WAVES / SIMDs: below the resident limit, the
  launch is a single generation of waves and its time is one wave's chain of
  dependent memory round trips;
* waiting share = SQ_WAIT_ANY / SQ_WAVE_CYCLES: the part of a wave's life spent
  waiting on a counter or a barrier; issuing share = SQ_ACTIVE_INST_ANY /
  SQ_WAVE_CYCLES;
* vector-memory load instructions per wave = SQ_INSTS_VMEM_RD / SQ_WAVES;
* L2 hit share = TCC_HIT / (TCC_HIT + TCC_MISS), from a pass of its own.

The clock is the MI355X's 2.4 GHz peak engine clock and it has 1,024 SIMDs.
"""

from __future__ import annotations

import argparse
import csv
import glob
import json
import os
from collections import OrderedDict

N_SIMD = 256 * 4
CLOCK_HZ = 2.4e9


def _rows(d: str):
    paths = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not paths:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def kernel_dispatches(rows, kernel: str):
    """Counters per dispatch of the kernels whose name contains `kernel`, in order."""
    out = OrderedDict()
    for r in rows:
        if kernel not in r["Kernel_Name"]:
            continue
        d = out.setdefault(r["Dispatch_Id"], {
            "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    return list(out.values())


def _mean(vals):
    return sum(vals) / len(vals) if vals else float("nan")


def summarise(dirs, kernel: str):
    """Averages over the kernel's dispatches of every pass, and the derived figures."""
    per_counter = {}
    ns = []
    for d in dirs:
        disp = kernel_dispatches(_rows(d), kernel)
        if not disp:
            raise RuntimeError(f"{d}: no dispatch of a kernel named like {kernel!r}")
        for x in disp:
            ns.append(x["ns"])
            for k, v in x.items():
                if k != "ns":
                    per_counter.setdefault(k, []).append(v)
    c = {k: _mean(v) for k, v in per_counter.items()}
    dur_s = _mean(ns) * 1e-9
    rec = {"kernel": kernel, "dispatches": len(per_counter.get("SQ_WAVE_CYCLES", [])),
           "avg_us": dur_s * 1e6, "counters": c}
    if "SQ_WAVE_CYCLES" in c:
        cyc = N_SIMD * CLOCK_HZ * dur_s
        rec["waves_per_simd"] = 4.0 * c["SQ_WAVE_CYCLES"] / cyc
        if "SQ_WAVES" in c:
            rec["waves_launched"] = c["SQ_WAVES"]
            rec["waves_launched_per_simd"] = c["SQ_WAVES"] / N_SIMD
            if c.get("SQ_INSTS_VMEM_RD") is not None and c["SQ_WAVES"]:
                rec["loads_per_wave"] = c["SQ_INSTS_VMEM_RD"] / c["SQ_WAVES"]
        if "SQ_WAIT_ANY" in c:
            rec["wait_share"] = c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"]
        if "SQ_ACTIVE_INST_ANY" in c:
            rec["issue_share"] = c["SQ_ACTIVE_INST_ANY"] / c["SQ_WAVE_CYCLES"]
    if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
        tot = c["TCC_HIT_sum"] + c["TCC_MISS_sum"]
        rec["l2_hit_share"] = c["TCC_HIT_sum"] / tot if tot else float("nan")
    return rec


def write_summary(path: str, recs, workload: str, command: str) -> None:
    def f(r, k, fmt):
        return fmt.format(r[k]) if k in r else "—"
    lines = [f"# What bounds `{recs[0]['kernel']}`: occupancy, waiting and L2 hits ({workload})", "",
             "Counter passes (each its own process), then this summary:", "", "```", command, "```", "",
             "resident waves per SIMD = 4·SQ_WAVE_CYCLES / (1,024 SIMDs × 2.4 GHz × dispatch time); "
             "waves launched per SIMD = SQ_WAVES / 1,024; waiting share = SQ_WAIT_ANY / SQ_WAVE_CYCLES; "
             "issuing share = SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES; loads per wave = SQ_INSTS_VMEM_RD / "
             "SQ_WAVES; L2 hit share = TCC_HIT / (TCC_HIT + TCC_MISS).", "",
             "| workload | dispatches | avg µs | waves launched (per SIMD) | resident waves per SIMD "
             "| waiting share | issuing share | load instructions per wave | L2 hit share |",
             "|---|---|---|---|---|---|---|---|---|"]
    for r in recs:
        lines.append(f"| {r['workload']} | {r['dispatches']} | {r['avg_us']:.1f} | "
                     f"{f(r, 'waves_launched', '{:.0f}')} ({f(r, 'waves_launched_per_simd', '{:.1f}')}) | "
                     f"{f(r, 'waves_per_simd', '{:.2f}')} | "
                     f"{f(r, 'wait_share', '{:.1%}')} | {f(r, 'issue_share', '{:.1%}')} | "
                     f"{f(r, 'loads_per_wave', '{:.1f}')} | {f(r, 'l2_hit_share', '{:.1%}')} |")
    lines += ["", "```json", json.dumps({"workload": workload, "records": recs}), "```", ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--dir", action="append", required=True,
                    help="a counter pass directory; repeat, or give LABEL=DIR to compare workloads")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    groups = OrderedDict()
    for d in a.dir:
        label, _, path = d.rpartition("=")
        groups.setdefault(label or a.workload, []).append(path)
    recs = []
    for label, dirs in groups.items():
        rec = summarise(dirs, a.kernel)
        rec["workload"] = label
        recs.append(rec)
    write_summary(a.out, recs, a.workload, a.command)
    print(json.dumps([{k: v for k, v in r.items() if k != "counters"} for r in recs]))


if __name__ == "__main__":
    main()
