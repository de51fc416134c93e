"""Measured HBM traffic of one kernel family from two rocprofv3 counter passes.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d F -o run -- python bench.py --pmc-pass ...
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d W -o run -- python bench.py --pmc-pass ...
    python -m paper_2402_02190_amd.traffic --fetch F --write W --kernel FAMILY \
        --workload C2 --out profiles/<family>_<workload>_traffic.md --command "..."

``bench.py --pmc-pass`` runs a device-to-device copy of a known size (the
calibration) and a few training steps.  Each counter (KiB per dispatch) is
scaled by what it reads for the copy: factor = counter bytes / true bytes of
the copy (reads = writes = its size).  The summary records the traffic per
launch of the kernel family and a hash of the sources the kernel is built
from; ``bench.py`` reports the figure only while the hash still matches.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_02190_amd", "csrc")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
CALIBRATION_BYTES = 1 << 30

# family (as the library's profiler names it) -> source files of its kernel
_SOURCES = {"gemm": ("gemm.hip", "gemm_kernel.hpp", "gemm_grouped.hip", "common.hpp"),
            "aggregate": ("aggregate.hip", "common.hpp"),
            "loss_fwd_bwd": ("loss.hip", "common.hpp"), "adam": ("adam.hip", "common.hpp")}


def source_files(family: str):
    for prefix, files in _SOURCES.items():
        if family.startswith(prefix):
            return [os.path.join(CSRC, f) for f in files]
    raise ValueError(f"no source mapping for kernel family {family}")


def source_hash(family: str) -> str:
    h = hashlib.sha256()
    for p in source_files(family):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_pattern(family: str) -> re.Pattern:
    """Regex on rocprofv3's demangled kernel name for a profiler family."""
    # gemm_<layout>[_byrow|_byk]_<BM>x<BN>x<BK>_w<WM>x<WN>[_p2|_il|_ring] -> k_gemm<BM, BN, BK,
    # WM, WN, A_T, B_T, PF, GM> (PF: 1 one-deep, 2 two-deep (_p2), 3 interleaved (_il), 4 LDS
    # ring (_ring); GM: group mode 0 / 1 by rows / 2 by K)
    m = re.fullmatch(r"gemm_([nt])([nt])(_byrow|_byk)?_(\d+)x(\d+)x(\d+)_w(\d+)x(\d+)(_p2|_il|_ring)?", family)
    if m:
        at, bt, grp, bm, bn, bk, wm, wn, loop = m.groups()
        gm = {None: 0, "_byrow": 1, "_byk": 2}[grp]
        pf = {None: 1, "_p2": 2, "_il": 3, "_ring": 4}[loop]
        args = f"{bm}, {bn}, {bk}, {wm}, {wn}, {'true' if at == 't' else 'false'}, " \
               f"{'true' if bt == 't' else 'false'}, {pf}, {gm}"
        return re.compile(re.escape(f"k_gemm<{args}>"))
    if family == "gemm_splitk_reduce":
        return re.compile(r"k_gemm_splitk_reduce")
    if family == "aggregate":
        return re.compile(r"k_aggregate<\d+, \d+, false>")
    if family == "aggregate_transposed":
        return re.compile(r"k_aggregate<\d+, \d+, true>")
    if family == "loss_fwd_bwd":
        return re.compile(r"k_loss<")
    if family == "adam":
        return re.compile(r"k_adam")
    raise ValueError(f"unknown kernel family {family}")


def _csv(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def per_dispatch(rows, counter: str):
    """{dispatch id: (kernel name, value)} for one counter (summed over its instances)."""
    out = {}
    acc = defaultdict(float)
    names = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = (r.get("Process_Id"), r["Dispatch_Id"])
        acc[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    for k, v in acc.items():
        out[k] = (names[k], v)
    return out


def measure(fetch_dir: str, write_dir: str, family: str, copy_bytes: int = CALIBRATION_BYTES):
    pat = kernel_pattern(family)
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        disp = per_dispatch(_csv(d), counter)
        copies = [v for name, v in disp.values() if COPY_KERNEL in name]
        if not copies:
            raise RuntimeError(f"{counter}: no {COPY_KERNEL} dispatch (calibration copy) found")
        copy_kib = max(copies)  # the calibration copy is the largest copy of the run
        factor = copy_kib * 1024.0 / copy_bytes
        ks = [v for name, v in disp.values() if pat.search(name)]
        if not ks:
            raise RuntimeError(f"{counter}: no dispatch of {family} found")
        res[counter] = {"kib_per_dispatch": sum(ks) / len(ks), "dispatches": len(ks),
                        "calibration_kib": copy_kib, "factor": factor,
                        "bytes_per_dispatch": sum(ks) / len(ks) * 1024.0 / factor}
    traffic = res["FETCH_SIZE"]["bytes_per_dispatch"] + res["WRITE_SIZE"]["bytes_per_dispatch"]
    return {"kernel": family, "traffic_bytes_per_launch": traffic, "counters": res,
            "calibration_bytes": copy_bytes}


def write_summary(path: str, rec: dict, workload: str, command: str) -> None:
    rec = dict(rec, workload=workload, source_sha256=source_hash(rec["kernel"]), command=command)
    c = rec["counters"]
    lines = [f"# HBM traffic of `{rec['kernel']}` on workload {workload}", "",
             "Two rocprofv3 counter passes over the same short run (each its own process):", "",
             "```", command, "```", "",
             "| counter | KiB per dispatch | dispatches | calibration copy KiB | factor (counter / true bytes) "
             "| bytes per dispatch (scaled) |", "|---|---|---|---|---|---|"]
    for k in ("FETCH_SIZE", "WRITE_SIZE"):
        v = c[k]
        lines.append(f"| {k} | {v['kib_per_dispatch']:.1f} | {v['dispatches']} | "
                     f"{v['calibration_kib']:.1f} | {v['factor']:.4f} | {v['bytes_per_dispatch']:.0f} |")
    lines += ["", f"Calibration: one device-to-device copy of {rec['calibration_bytes']} bytes "
              f"(`{COPY_KERNEL}`), which reads and writes that many bytes.",
              f"Traffic per launch: **{rec['traffic_bytes_per_launch']:.0f} bytes**.", "",
              "Record read by bench.py (valid while the kernel sources hash to source_sha256):", "",
              "```json", json.dumps(rec), "```", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def load_traffic(family: str, workload: str, profiles_dir: str = None):
    """Traffic bytes per launch recorded for (family, workload), or None when there
    is no record or the kernel's sources changed since the counters were taken."""
    profiles_dir = profiles_dir or os.path.join(ROOT, "profiles")
    for p in sorted(glob.glob(os.path.join(profiles_dir, "*_traffic.md"))):
        with open(p) as f:
            text = f.read()
        m = re.search(r"```json\n(.*?)\n```", text, re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("kernel") != family or rec.get("workload") != workload:
            continue
        try:
            if rec.get("source_sha256") != source_hash(family):
                return None
        except ValueError:
            return None
        return float(rec["traffic_bytes_per_launch"])
    return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--copy-bytes", type=int, default=CALIBRATION_BYTES)
    a = ap.parse_args(argv)
    rec = measure(a.fetch, a.write, a.kernel, a.copy_bytes)
    write_summary(a.out, rec, a.workload, a.command)
    print(json.dumps({k: v for k, v in rec.items() if k != "counters"}))


if __name__ == "__main__":
    main()
