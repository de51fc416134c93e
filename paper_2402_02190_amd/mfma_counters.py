"""MFMA utilisation of the GEMM kernels from one rocprofv3 SQ counter pass.

    rocprofv3 --pmc SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_MFMA \\
        SQ_WAIT_INST_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_LDS SQ_WAIT_INST_ANY \\
        --output-format csv -d D -o run -- python bench.py --pmc-pass ...
    python -m paper_2402_02190_amd.mfma_counters --dir D --workload C2 --out FILE --command "..."

Per kernel instantiation (dispatches of ``k_gemm<...>``): the MFMA instructions
and MFMA-busy cycles per dispatch (summed over all SIMDs by the hardware; a
v_mfma_f32_32x32x2f32 keeps its SIMD's matrix core busy 64 cycles), and the
utilisation busy / (SIMDs x clock x dispatch duration) with the dispatch's
own timestamps, the MI355X's 1,024 SIMDs and its 2.4 GHz peak engine clock
(so a lower clock under load reads as lower utilisation).  LDS figures: bank
conflict cycles per LDS-active cycle and the share of wave time spent
waiting on LDS.
"""

from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
from collections import OrderedDict

N_SIMD = 256 * 4
CLOCK_HZ = 2.4e9
COUNTERS = ("SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_MFMA",
            "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_ANY")


def _rows(d: str):
    paths = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not paths:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def short_name(name: str) -> str:
    m = re.search(r"k_gemm<([^>]*)>", name)
    return f"k_gemm<{m.group(1)}>" if m else name


def dispatches(rows):
    """Counters of every dispatch, keyed by dispatch id, in order of appearance."""
    out = OrderedDict()
    for r in rows:
        d = out.setdefault(r["Dispatch_Id"], {"name": r["Kernel_Name"], "ns":
                                              int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    return out


def summarise(rows):
    """Per k_gemm instantiation: averages over its dispatches."""
    groups = OrderedDict()
    for d in dispatches(rows).values():
        if "k_gemm<" not in d["name"] or d.get("SQ_INSTS_MFMA", 0) <= 0:
            continue
        groups.setdefault(short_name(d["name"]), []).append(d)
    out = []
    for name, ds in groups.items():
        n = len(ds)
        avg = {c: sum(d.get(c, 0.0) for d in ds) / n for c in COUNTERS}
        ns = sum(d["ns"] for d in ds) / n
        util = sum(d["SQ_VALU_MFMA_BUSY_CYCLES"] / (N_SIMD * CLOCK_HZ * d["ns"] * 1e-9) for d in ds) / n
        out.append({
            "kernel": name, "dispatches": n, "avg_us": ns / 1e3,
            "mfma_per_dispatch": avg["SQ_INSTS_MFMA"],
            "busy_cycles_per_mfma": avg["SQ_VALU_MFMA_BUSY_CYCLES"] / avg["SQ_INSTS_MFMA"],
            "mfma_util": util,
            "lds_conflict_per_active": (avg["SQ_LDS_BANK_CONFLICT"] / avg["SQ_ACTIVE_INST_LDS"]
                                        if avg["SQ_ACTIVE_INST_LDS"] > 0 else 0.0),
            "lds_wait_share": (avg["SQ_WAIT_INST_LDS"] / avg["SQ_WAVE_CYCLES"]
                               if avg["SQ_WAVE_CYCLES"] > 0 else 0.0),
            "any_wait_share": (avg["SQ_WAIT_INST_ANY"] / avg["SQ_WAVE_CYCLES"]
                               if avg["SQ_WAVE_CYCLES"] > 0 else 0.0),
        })
    return out


def write_summary(path: str, res, workload: str, command: str) -> None:
    lines = [f"# MFMA utilisation of the GEMM kernels on workload {workload}", "",
             "One rocprofv3 SQ counter pass (its own process; counter collection serialises the "
             "dispatches):", "", "```", command, "```", "",
             f"utilisation = SQ_VALU_MFMA_BUSY_CYCLES / ({N_SIMD} SIMDs x {CLOCK_HZ / 1e9:.1f} GHz x "
             "dispatch duration); busy cycles are summed over all SIMDs by the hardware.", "",
             "| kernel | dispatches | avg us | MFMA instr / dispatch | busy cycles / MFMA | MFMA util "
             "| LDS bank-conflict cycles / LDS-active cycle | wave time waiting on LDS | wave time "
             "waiting (any) |", "|---|---|---|---|---|---|---|---|---|"]
    for r in res:
        lines.append(f"| `{r['kernel']}` | {r['dispatches']} | {r['avg_us']:.1f} | "
                     f"{r['mfma_per_dispatch']:.0f} | {r['busy_cycles_per_mfma']:.1f} | "
                     f"{100 * r['mfma_util']:.1f}% | {r['lds_conflict_per_active']:.3f} | "
                     f"{100 * r['lds_wait_share']:.1f}% | {100 * r['any_wait_share']:.1f}% |")
    lines += ["", "```json", json.dumps({"workload": workload, "kernels": res}), "```", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--dir", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    res = summarise(_rows(a.dir))
    write_summary(a.out, res, a.workload, a.command)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
