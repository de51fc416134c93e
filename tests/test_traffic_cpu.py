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
    assert TR.kernel_pattern("gemm_nn_64x64x16_w2x2_il").search(
        "void cpra::gemmk::k_gemm<64, 64, 16, 2, 2, false, false, 3, 0>(x)")
    assert not TR.kernel_pattern("gemm_nn_64x64x16_w2x2_il").search(
        "void cpra::gemmk::k_gemm<64, 64, 16, 2, 2, false, false, 2, 0>(x)")
    assert TR.kernel_pattern("gemm_nt_64x128x16_w2x2_ring").search(
        "void cpra::gemmk::k_gemm<64, 128, 16, 2, 2, false, true, 4, 0>(x)")
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


def test_mfma_counter_summary_on_a_synthetic_pass(tmp_path):
    """MFMA utilisation = busy cycles / (SIMDs x clock x duration), per instantiation."""
    from paper_2402_02190_amd import mfma_counters as mc
    d = tmp_path / "sq"
    d.mkdir()
    name = "void cpra::gemmk::k_gemm<64, 64, 16, 2, 2, false, false, 2, 0>(cpra::gemmk::LaunchArgs)"
    rows = []
    for disp, ns in ((1, 10000), (2, 20000)):  # 10 and 20 us
        busy = 0.5 * mc.N_SIMD * mc.CLOCK_HZ * ns * 1e-9  # half busy
        vals = {"SQ_WAVE_CYCLES": 1000.0, "SQ_BUSY_CYCLES": 10.0, "SQ_VALU_MFMA_BUSY_CYCLES": busy,
                "SQ_INSTS_MFMA": busy / 64, "SQ_WAIT_INST_LDS": 100.0, "SQ_LDS_BANK_CONFLICT": 5.0,
                "SQ_ACTIVE_INST_LDS": 50.0, "SQ_WAIT_INST_ANY": 400.0}
        for c, v in vals.items():
            rows.append({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v,
                         "Start_Timestamp": 1000, "End_Timestamp": 1000 + ns})
    rows.append({"Dispatch_Id": 3, "Kernel_Name": "k_adam<true>", "Counter_Name": "SQ_INSTS_MFMA",
                 "Counter_Value": 0, "Start_Timestamp": 0, "End_Timestamp": 5})
    with open(d / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)
    res = mc.summarise(mc._rows(str(d)))
    assert len(res) == 1
    r = res[0]
    assert r["kernel"] == "k_gemm<64, 64, 16, 2, 2, false, false, 2, 0>" and r["dispatches"] == 2
    assert abs(r["mfma_util"] - 0.5) < 1e-12 and abs(r["busy_cycles_per_mfma"] - 64.0) < 1e-9
    assert abs(r["avg_us"] - 15.0) < 1e-12
    assert abs(r["lds_conflict_per_active"] - 0.1) < 1e-12 and abs(r["lds_wait_share"] - 0.1) < 1e-12
    out = tmp_path / "s.md"
    mc.write_summary(str(out), res, "C2", "cmd")
    assert "50.0%" in out.read_text()
