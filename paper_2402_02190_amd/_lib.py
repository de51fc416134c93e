"""ctypes declarations of libcpra's C ABI (include/cpra.h).

Loading fails loudly when the shared library has not been built: there is no
fallback implementation of any step of the path.
"""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcpra.so")

STATUS = {
    0: "CPRA_OK", 1: "CPRA_ERR_NULL", 2: "CPRA_ERR_SHAPE", 3: "CPRA_ERR_CSR", 4: "CPRA_ERR_PARAM",
    5: "CPRA_ERR_OVERFLOW", 6: "CPRA_ERR_WORKSPACE", 7: "CPRA_ERR_HIP", 8: "CPRA_ERR_NONFINITE",
}
MIS, MAXCUT = 0, 1
GCN, SAGE = 0, 1


class CpraError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Csr(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_graphs", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("graph_ptr", C.c_void_p),
                ("weight", C.c_void_p), ("inv_deg", C.c_void_p), ("wdeg", C.c_void_p),
                ("col_inv_deg", C.c_void_p)]


class LossCfg(C.Structure):
    _fields_ = [("problem", C.c_int32), ("S", C.c_int32), ("alpha", C.c_int32),
                ("std_ddof", C.c_int32), ("gamma", C.c_float), ("nu", C.c_float),
                ("lambda_", C.c_void_p), ("step_counter", C.c_void_p),
                ("gamma_start", C.c_float), ("gamma_end", C.c_float), ("T", C.c_int32),
                ("node_weight", C.c_void_p), ("ld_node_weight", C.c_int64),
                ("edge_weight", C.c_void_p), ("ld_edge_weight", C.c_int64)]


class ModelCfg(C.Structure):
    _fields_ = [("layer_kind", C.c_int32), ("n_layers", C.c_int32), ("in_dim", C.c_int32),
                ("hidden", C.c_int32), ("S", C.c_int32), ("recompute", C.c_int32),
                ("z_offset", C.c_void_p), ("train_from_layer", C.c_int32),
                ("reuse_frozen_prefix", C.c_int32), ("weight_groups", C.c_int32)]


class AdamCfg(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("weight_decay", C.c_double)]


class EarlyStopState(C.Structure):
    _fields_ = [("prev_head", C.c_double), ("prev_phi", C.c_double), ("stalled", C.c_int32),
                ("stopped", C.c_int32), ("stop_step", C.c_int32), ("seen", C.c_int32)]


class EarlyStopCfg(C.Structure):
    _fields_ = [("tol", C.c_double), ("patience", C.c_int32), ("relative", C.c_int32),
                ("state", C.c_void_p)]


class StepCfg(C.Structure):
    _fields_ = [("model", ModelCfg), ("loss", LossCfg), ("adam", AdamCfg),
                ("early_stop", EarlyStopCfg)]


class MpnnCfg(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("in_dim", C.c_int32), ("hidden", C.c_int32),
                ("S", C.c_int32)]


class MpnnStepCfg(C.Structure):
    _fields_ = [("net", MpnnCfg), ("loss", LossCfg), ("adam", AdamCfg), ("beta", C.c_float)]


P = C.c_void_p
I32, I64, F32, SZ = C.c_int32, C.c_int64, C.c_float, C.c_size_t
PMpnn, PMpnnStep = C.POINTER(MpnnCfg), C.POINTER(MpnnStepCfg)
PCsr, PLoss, PModel, PAdam, PStep = (C.POINTER(Csr), C.POINTER(LossCfg), C.POINTER(ModelCfg),
                                     C.POINTER(AdamCfg), C.POINTER(StepCfg))

# name -> (restype, argtypes); restype None means cpra_status (checked)
LOSS_NOALLOC_SCRATCH_BYTES = 32 << 20  # CPRA_LOSS_NOALLOC_SCRATCH_BYTES

PROTOTYPES = {
    "cpra_abi_version": (I32, []),
    "cpra_status_string": (C.c_char_p, [I32]),
    "cpra_last_error_message": (C.c_char_p, []),
    "cpra_csr_validate_host": (None, [I32, I64, P, P, P]),
    "cpra_csr_prepare": (None, [PCsr, P, P, P]),
    "cpra_csr_prepare_col": (None, [PCsr, P, P]),
    "cpra_aggregate_mean": (None, [PCsr, I32, I32, P, I64, P, I64, P, I64, P, I32, P, I64, P]),
    "cpra_gemm_workspace_bytes": (SZ, [I32, I32, I32, I32, I32]),
    "cpra_gemm": (None, [I32, I32, I32, I32, I32, P, I64, P, I64, F32, P, I64, P, I32, P, SZ, P]),
    "cpra_gemm_grouped_workspace_bytes": (SZ, [PCsr, I32, I32, I32, I32]),
    "cpra_gemm_grouped": (None, [PCsr, I32, I32, I32, I32, I32, P, I64, P, I64, I64, P, I64, I64,
                                 P, I64, P, I64, I32, P, SZ, P]),
    "cpra_loss_workspace_bytes": (SZ, [PCsr, PLoss]),
    "cpra_loss_fwd_bwd": (None, [PCsr, PLoss, P, I64, P, I64, P, I64, P, P, SZ, P]),
    "cpra_loss_fwd_bwd_noalloc": (None, [PCsr, PLoss, P, I64, P, I64, P, I64, P, P]),
    "cpra_loss_total": (None, [I32, I32, P, C.c_double, C.c_double, P, P]),
    "cpra_sigmoid": (None, [I32, I32, P, I64, P, I64, P]),
    "cpra_model_param_count": (I64, [PModel, I32]),
    "cpra_model_param_offsets": (None, [PModel, I32, C.POINTER(I64)]),
    "cpra_model_workspace_bytes": (SZ, [PCsr, PModel]),
    "cpra_model_forward": (None, [PCsr, PModel, P, P, I64, P, SZ, P]),
    "cpra_model_backward": (None, [PCsr, PModel, P, P, I64, P, P, SZ, P]),
    "cpra_model_saved_activation": (None, [PCsr, PModel, P, SZ, I32, C.POINTER(C.c_void_p),
                                           C.POINTER(I64)]),
    "cpra_adam_step": (None, [I64, P, P, P, P, PAdam, I32, P, P]),
    "cpra_early_stop_reset": (None, [P, P]),
    "cpra_train_step_workspace_bytes": (SZ, [PCsr, PStep]),
    "cpra_train_step": (None, [PCsr, PStep, P, P, P, P, P, P, P, I32, P, P, SZ, P]),
    "cpra_round_eval_workspace_bytes": (SZ, [PCsr, I32]),
    "cpra_round_eval": (None, [PCsr, I32, I32, P, I64, P, I64, P, P, P, P, P, I64, P, I64, P, SZ,
                               P]),
    "cpra_pairwise_hamming_workspace_bytes": (SZ, [I32, I32]),
    "cpra_pairwise_hamming": (None, [I32, I32, P, I64, P, I64, P, P, P, SZ, P]),
    "cpra_node_features": (None, [PCsr, I32, I32, P, I64, P, I64, P, P]),
    "cpra_mpnn_param_count": (I64, [PMpnn]),
    "cpra_mpnn_param_offsets": (None, [PMpnn, C.POINTER(I64)]),
    "cpra_mpnn_workspace_bytes": (SZ, [PCsr, PMpnn]),
    "cpra_mpnn_forward": (None, [PCsr, PMpnn, P, P, P, P, SZ, P]),
    "cpra_mpnn_backward": (None, [PCsr, PMpnn, P, P, P, P, SZ, P]),
    "cpra_mpnn_saved": (None, [PCsr, PMpnn, P, SZ, I32, I32, C.POINTER(C.c_void_p),
                               C.POINTER(I64)]),
    "cpra_bce_grad": (None, [I32, I32, P, I64, P, I64, F32, P, I64, P]),
    "cpra_mpnn_train_step_workspace_bytes": (SZ, [PCsr, PMpnnStep]),
    "cpra_mpnn_train_step": (None, [PCsr, PMpnnStep, P, P, P, P, P, P, P, P, P, I32, P, P, SZ,
                                    P]),
    "cpra_capture_begin": (None, [P]),
    "cpra_capture_end": (None, [P, C.POINTER(C.c_void_p)]),
    "cpra_graph_launch": (None, [P, P]),
    "cpra_graph_destroy": (None, [P]),
    "cpra_autotune_begin": (None, []),
    "cpra_autotune_end": (None, [C.POINTER(I32)]),
    "cpra_autotune_reset": (None, []),
    "cpra_autotune_get": (None, [I32, C.c_char_p, SZ, C.POINTER(I32), C.POINTER(I32), C.c_char_p,
                                 SZ, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cpra_autotune_set": (None, [C.c_char_p, I32, I32]),
    "cpra_profile_begin": (None, []),
    "cpra_profile_stop": (None, []),
    "cpra_profile_collect": (None, []),
    "cpra_profile_end": (None, [C.POINTER(I32)]),
    "cpra_profile_get": (None, [I32, C.c_char_p, SZ, C.POINTER(I64), C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]),
}

_lib = None


def lib():
    """The loaded shared library (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -m paper_2402_02190_amd.build); there is no fallback")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(h, name)
            f.restype = I32 if res is None else res
            f.argtypes = args
        _lib = h
    return _lib


def exported_symbols():
    return list(PROTOTYPES)


def check(status: int) -> None:
    if status != 0:
        msg = lib().cpra_last_error_message()
        raise CpraError(status, msg.decode() if msg else "")


def call(name: str, *args):
    """Call a status-returning entry point and raise CpraError on failure."""
    check(getattr(lib(), name)(*args))
