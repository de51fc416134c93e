"""Shared helpers for the GPU parity tests (comparison metrics and tolerances).

Tolerances follow the floating-point contract of the path: FP32 kernels
against the FP64 oracle within 1e-5 relative, where "relative" is
condition-aware:
  * arrays:  ||gpu - oracle||_2 <= tol * ||oracle||_2
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


def rel_err(gpu, ref) -> float:
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(gpu - ref)
    return float(num / den) if den > 0 else float(num)


def assert_close_array(gpu, ref, tol=TOL, what=""):
    e = rel_err(gpu, ref)
    say(f"  {what}: rel_err={e:.3e}")
    assert e <= tol, f"{what}: relative error {e:.3e} > {tol}"
    return e


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
