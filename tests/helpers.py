"""Shared helpers for the GPU parity tests (comparison metrics and tolerances).

Tolerances follow the floating-point contract of the path: FP32 kernels
against the FP64 oracle within 1e-5 relative, where "relative" is
condition-aware:
  * arrays:  ||gpu - oracle||_2 <= tol * ||oracle||_2, and element by element
             |gpu_i - oracle_i| <= ELEM_FACTOR * tol * max(|oracle_i|, rms(oracle)).
             Rounding errors that meet the norm bound have an rms of at most
             tol * rms(oracle) and a maximum of a few times that (about
             sqrt(2 ln n) = 5.7 times for n = 10^7 independent errors); an element
             far above the rms (a hub node's gradient) carries an error relative to
             itself instead.  One wrong element or row (an error of the order of
             the element or of rms(oracle)) fails the gate.  The largest error
             relative to each element itself, floored at 1e-6 * rms(oracle) (the
             statistic FP32 cancellation drives towards 1 on near-zero elements),
             is printed beside both.
  * scalars: |gpu - oracle| <= tol * sum |summands|
Integer results (rounded solutions, counts) must match exactly.
"""

import sys

import numpy as np
import pytest
import torch

TOL = 1e-5


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


ELEM_FACTOR = 10.0  # element gate: |error_i| <= ELEM_FACTOR * tol * max(|oracle_i|, rms(oracle))


def rel_err(gpu, ref) -> float:
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(gpu - ref)
    return float(num / den) if den > 0 else float(num)


def err_stats(gpu, ref):
    """(norm-wise relative error, max_i |error_i| / max(|ref_i|, rms(ref)),
    max_i |error_i| / max(|ref_i|, 1e-6 rms(ref)))."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(gpu - ref)
    if d.size == 0:
        return 0.0, 0.0, 0.0
    rms = float(np.sqrt(np.mean(ref * ref)))
    if rms == 0.0:
        m = float(d.max())
        return m, m, m
    a = np.abs(ref)
    return (rel_err(gpu, ref), float(np.max(d / np.maximum(a, rms))),
            float(np.max(d / np.maximum(a, 1e-6 * rms))))


def assert_close_array(gpu, ref, tol=TOL, what="", elem_factor=ELEM_FACTOR):
    e, emax, erel = err_stats(gpu, ref)
    say(f"  {what}: rel_err={e:.3e} max elem err/max(|ref|,rms)={emax:.3e} "
        f"max elem err/max(|ref|,1e-6 rms)={erel:.3e}")
    assert e <= tol, f"{what}: relative error {e:.3e} > {tol}"
    assert emax <= elem_factor * tol, \
        f"{what}: element error {emax:.3e} of max(|ref|, rms) > {elem_factor * tol:.1e}"
    return e


def check_relu_decisions(active, preacts, what="", band_rel=1e-5):
    """The ReLU derivative is a discrete decision taken on the sign of a
    pre-activation Y.  Where an oracle backward is handed the FP32 forward's
    decisions (``active``, one boolean [N, H] array per hidden layer), every
    decision that differs from the FP64 forward's own (Y > 0) must sit within
    band_rel * rms(Y) of zero, so the oracle takes nothing else from the GPU."""
    assert len(active) == len(preacts)
    for k, (act, Y) in enumerate(zip(active, preacts)):
        Y = np.asarray(Y)
        flips = np.asarray(act) != (Y > 0)
        band = band_rel * float(np.sqrt(np.mean(Y * Y))) if Y.size else 0.0
        worst = float(np.abs(Y[flips]).max()) if flips.any() else 0.0
        say(f"  {what} layer {k}: {int(flips.sum())} of {Y.size} ReLU decisions differ from FP64 "
            f"(max |Y| there {worst:.2e}, band {band:.2e})")
        assert worst <= band, f"{what} layer {k}: a ReLU decision differs at |Y| = {worst:.3e}"


def assert_close_scalar(gpu, ref, scale, tol=TOL, what=""):
    err = abs(float(gpu) - float(ref))
    bound = tol * max(float(scale), 1e-30)
    assert err <= bound, f"{what}: |{gpu} - {ref}| = {err:.3e} > {bound:.3e}"
    return err / max(float(scale), 1e-30)


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def assert_update_close(after, before, ref_after, tol=TOL, what=""):
    """Compare an FP32 parameter update with the FP64 one, allowing the final
    rounding of the stored FP32 value: || max(0, |after - ref| - ulp(ref)) || <=
    tol * || ref - before ||."""
    after = np.asarray(after, dtype=np.float64)
    ref_after = np.asarray(ref_after, dtype=np.float64)
    step = ref_after - np.asarray(before, dtype=np.float64)
    ulp = np.spacing(np.abs(ref_after).astype(np.float32)).astype(np.float64)
    excess = np.maximum(0.0, np.abs(after - ref_after) - ulp)
    den = np.linalg.norm(step)
    e = float(np.linalg.norm(excess) / den) if den > 0 else float(np.linalg.norm(excess))
    say(f"  {what}: update rel_err (beyond one FP32 ulp)={e:.3e}")
    assert e <= tol, f"{what}: update error {e:.3e} > {tol}"
    return e


# tile configurations the library's GEMM tuner chooses from (forced one by one in the
# GEMM tests)
N_GEMM_CFGS = 32
