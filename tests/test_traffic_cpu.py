"""Host logic of the HBM-traffic records (paper_2402_02190_amd/traffic.py):
kernel-name mapping, counter calibration on a synthetic counter file, and the
rule that a record stops applying once the kernel's sources change."""

import csv
import os

import pytest

from paper_2402_02190_amd import traffic as TR


def test_kernel_pattern_maps_profiler_families_to_trace_names():
    p = TR.kernel_pattern("gemm_tn_64x128x32_w2x2")
    assert p.search("void cpra::gemmk::k_gemm<64, 128, 32, 2, 2, true, false, 1, 0>(x)")
    assert not p.search("void cpra::gemmk::k_gemm<64, 128, 32, 2, 2, false, false, 1, 0>(x)")
    assert not p.search("void cpra::gemmk::k_gemm<64, 128, 32, 2, 2, true, false, 2, 0>(x)")
    assert TR.kernel_pattern("gemm_nt_byrow_64x32x16_w1x1_p2").search(
        "void cpra::gemmk::k_gemm<64, 32, 16, 1, 1, false, true, 2, 1>(x)")
    assert TR.kernel_pattern("gemm_tn_byk_64x64x32_w2x2_p2").search(
        "void cpra::gemmk::k_gemm<64, 64, 32, 2, 2, true, false, 2, 2>(x)")
    assert not TR.kernel_pattern("gemm_tn_64x64x32_w2x2_p2").search(
        "void cpra::gemmk::k_gemm<64, 64, 32, 2, 2, true, false, 2, 2>(x)")
    assert TR.kernel_pattern("aggregate").search("k_aggregate<4, 1, false>(a)")
    assert not TR.kernel_pattern("aggregate").search("k_aggregate<4, 1, true>(a)")
    assert TR.kernel_pattern("loss_fwd_bwd").search("cpra::k_loss<2>(args)")
    with pytest.raises(ValueError):
        TR.kernel_pattern("nonexistent")


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Process_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, v) in enumerate(rows):
            w.writerow([i + 1, 7, name, counter, v])


def test_measure_scales_each_counter_by_the_calibration_copy(tmp_path, monkeypatch):
    copy = 1 << 20
    k = "void cpra::gemmk::k_gemm<64, 64, 16, 2, 2, false, false, 1, 0>(L)"
    # FETCH reads half the true bytes, WRITE exactly them (factors 0.5 and 1.0)
    _write_counters(tmp_path / "F", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", copy / 1024 / 2),
                                                    (k, 100.0), (k, 300.0), ("other", 5.0)])
    _write_counters(tmp_path / "W", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy / 1024),
                                                    (k, 50.0), (k, 50.0)])
    rec = TR.measure(str(tmp_path / "F"), str(tmp_path / "W"), "gemm_nn_64x64x16_w2x2", copy)
    assert rec["counters"]["FETCH_SIZE"]["factor"] == pytest.approx(0.5)
    assert rec["counters"]["WRITE_SIZE"]["factor"] == pytest.approx(1.0)
    assert rec["traffic_bytes_per_launch"] == pytest.approx(200.0 * 1024 / 0.5 + 50.0 * 1024)
    # a written summary is found again, and dropped when the source hash differs
    prof = tmp_path / "profiles"
    prof.mkdir()
    TR.write_summary(str(prof / "x_traffic.md"), rec, "C2", "cmd")
    assert TR.load_traffic("gemm_nn_64x64x16_w2x2", "C2", str(prof)) == pytest.approx(
        rec["traffic_bytes_per_launch"])
    assert TR.load_traffic("gemm_nn_64x64x16_w2x2", "C4", str(prof)) is None
    monkeypatch.setattr(TR, "source_hash", lambda fam: "changed")
    assert TR.load_traffic("gemm_nn_64x64x16_w2x2", "C2", str(prof)) is None
