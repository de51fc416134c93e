"""Host logic of the wave-counter summaries (paper_2402_02190_amd/wave_counters.py) on
synthetic counter files: per-kernel averaging over dispatches and passes, and the
derived occupancy, waiting, load and L2 figures."""

import csv
import json
import os

import pytest

from paper_2402_02190_amd import wave_counters as WC


def _write(d, rows):
    """rows: (dispatch id, kernel name, counter, value, duration ns)."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                    "Start_Timestamp", "End_Timestamp"])
        for i, name, counter, value, ns in rows:
            w.writerow([i, name, counter, value, 1000, 1000 + ns])


def test_figures_from_two_passes(tmp_path):
    loss = "void cpra::(anonymous namespace)::k_loss<1, 4, false>(LossArgs)"
    other = "void cpra::gemmk::k_gemm<64, 64, 16, 2, 2, false, true, 2, 0>(x)"
    ns = 10_000  # 10 us: 1,024 SIMDs x 2.4 GHz x 10 us = 24,576,000 SIMD-cycles
    sq = []
    for i in (1, 2):  # two dispatches of the loss with different counts: averaged
        k = 1.0 if i == 1 else 3.0
        sq += [(i, loss, "SQ_WAVE_CYCLES", 2_457_600 * k, ns), (i, loss, "SQ_WAVES", 2048 * k, ns),
               (i, loss, "SQ_WAIT_ANY", 1_228_800 * k, ns), (i, loss, "SQ_ACTIVE_INST_ANY", 245_760 * k, ns),
               (i, loss, "SQ_INSTS_VMEM_RD", 20_480 * k, ns)]
    sq += [(9, other, "SQ_WAVE_CYCLES", 1e12, ns), (9, other, "SQ_WAVES", 1, ns)]
    _write(tmp_path / "a", sq)
    _write(tmp_path / "b", [(1, loss, "TCC_HIT_sum", 300, ns), (1, loss, "TCC_MISS_sum", 100, ns),
                            (2, loss, "TCC_HIT_sum", 500, ns), (2, loss, "TCC_MISS_sum", 100, ns)])
    r = WC.summarise([str(tmp_path / "a"), str(tmp_path / "b")], "k_loss")
    assert r["dispatches"] == 2
    assert r["avg_us"] == pytest.approx(10.0)
    # mean SQ_WAVE_CYCLES 4,915,200 quad-cycles = 19,660,800 cycles over 24,576,000
    assert r["waves_per_simd"] == pytest.approx(0.8)
    assert r["waves_launched"] == pytest.approx(4096)
    assert r["waves_launched_per_simd"] == pytest.approx(4.0)
    assert r["wait_share"] == pytest.approx(0.5)
    assert r["issue_share"] == pytest.approx(0.1)
    assert r["loads_per_wave"] == pytest.approx(10.0)
    assert r["l2_hit_share"] == pytest.approx(800 / 1000)


def test_missing_kernel_is_an_error(tmp_path):
    _write(tmp_path / "a", [(1, "k_other", "SQ_WAVES", 1, 10)])
    with pytest.raises(RuntimeError):
        WC.summarise([str(tmp_path / "a")], "k_loss")


def test_summary_file_holds_the_table_and_the_record(tmp_path):
    ns = 10_000
    _write(tmp_path / "a", [(1, "k_loss<1>", "SQ_WAVE_CYCLES", 2_457_600, ns),
                            (1, "k_loss<1>", "SQ_WAVES", 2048, ns)])
    out = tmp_path / "s.md"
    WC.main(["--dir", f"C2={tmp_path / 'a'}", "--kernel", "k_loss", "--workload", "C2",
             "--out", str(out), "--command", "cmd"])
    text = out.read_text()
    assert "| C2 | 1 | 10.0 | 2048 (2.0) | 0.40 |" in text
    rec = json.loads(text.split("```json\n")[1].split("\n```")[0])
    assert rec["records"][0]["waves_per_simd"] == pytest.approx(0.4)
