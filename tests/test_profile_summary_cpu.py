"""Host logic of the profile summariser (paper_2402_02190_amd/profile_summary.py)
on synthetic rocprofv3 CSV files: the kernel table, the dominant family's
kernel-trace average over the eager launches, and the size sweep's matching of
grid sizes in order of appearance."""

import csv
import json
import os

from paper_2402_02190_amd import profile_summary as PS

AGG = "void cpra::(anonymous namespace)::k_aggregate<4, 2, false>(cpra::(anonymous namespace)::AggArgs)"
AGG_T = "void cpra::(anonymous namespace)::k_aggregate<4, 2, true>(cpra::(anonymous namespace)::AggArgs)"
LOSS = "void cpra::(anonymous namespace)::k_loss<1, 4, false>(cpra::(anonymous namespace)::LossArgs)"


def _csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _trace(d, launches):
    """launches: (name, grid, duration ns) in launch order."""
    rows, t = [], 1000
    for name, grid, ns in launches:
        rows.append([name, grid, t, t + ns])
        t += ns + 500
    _csv(os.path.join(d, "host", "run_kernel_trace.csv"),
         ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"], rows)


def test_steps_table_and_dominant_average(tmp_path):
    d = str(tmp_path / "trace")
    _csv(os.path.join(d, "host", "run_kernel_stats.csv"),
         ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"],
         [[AGG, 4, 600000, 150000, 100000, 200000],
          [AGG_T, 2, 200000, 100000, 100000, 100000],
          ["void at::native::fill_kernel(x)", 3, 999000, 333000, 333000, 333000]])
    # two replayed launches (200 us), then the two eager launches bench.py times (100 us)
    _trace(d, [(AGG, 1024, 200000), (AGG_T, 1024, 100000), (AGG, 1024, 200000),
               (AGG, 1024, 100000), (AGG, 1024, 100000)])
    bench = tmp_path / "bench.json"
    bench.write_text("log line\n" + json.dumps({
        "ms_per_step": 0.5, "value": 1.0e10,
        "roofline": {"kernel": "aggregate", "avg_us": 101.0, "achieved": 700.0, "unit": "GB/s",
                     "frac": 0.0875, "launches": 2}}) + "\n")
    out = tmp_path / "s.md"
    text = PS.steps(d, str(bench), "Title", "cmd --x", str(out))
    assert out.read_text() == text
    assert text.startswith("# Title\n")
    assert "    cmd --x" in text
    assert "fill_kernel" not in text
    # percentages over library kernels only: 600 / 800 and 200 / 800
    assert "| `k_aggregate<4, 2, false>(AggArgs)` | 4 | 150.00 | 100.00 | 200.00 | 75.0 |" in text
    assert "| `k_aggregate<4, 2, true>(AggArgs)` | 2 | 100.00 | 100.00 | 100.00 | 25.0 |" in text
    assert "500.0 us/step" in text and "1e+10" in text and "8.8% of peak" in text
    # the two eager launches average 100 us, the two replayed ones 200 us; the transposed
    # aggregation is not in the family
    assert "over the 2 launches of the profiled eager steps" in text
    assert "= 100.0 us; over the 2 launches of the replayed/warm-up steps = 200.0 us" in text
    assert "`k_aggregate<*, *, false>`" in text


def test_sweep_matches_grid_sizes_in_order_of_appearance(tmp_path):
    d = str(tmp_path / "trace")
    # the loss kernel's grid shrinks while the aggregation's grows: sorting sizes would swap
    # the loss rows, order of appearance keeps each with its graph
    _trace(d, [(LOSS, 4096, 10000), (AGG, 512, 20000), (LOSS, 4096, 12000),
               (LOSS, 2048, 50000), (AGG, 2048, 60000), (AGG_T, 2048, 1)])
    rows = []
    for n, ev_l, ev_a in ((100, 11.0, 20.5), (400, 50.5, 60.5)):
        rows.append({"n": n, "nnz": 20 * n,
                     "loss_fwd_bwd": {"avg_us": ev_l, "compulsory_GBps": 900.0, "frac_hbm_peak": 0.11,
                                      "gather_GBps": 6000.0},
                     "aggregate": {"avg_us": ev_a, "compulsory_GBps": 700.0, "frac_hbm_peak": 0.09,
                                   "gather_GBps": 6500.0}})
    sw = tmp_path / "sweep.json"
    sw.write_text(json.dumps({"rows": rows}) + "\n")
    text = PS.sweep(d, str(sw), "cmd", str(tmp_path / "w.md"))
    assert "| 100 | 2,000 | `loss_fwd_bwd` | 11.0 | 11.0 |" in text
    assert "| 100 | 2,000 | `aggregate` | 20.5 | 20.0 |" in text
    assert "| 400 | 8,000 | `loss_fwd_bwd` | 50.5 | 50.0 |" in text
    assert "| 400 | 8,000 | `aggregate` | 60.5 | 60.0 |" in text
