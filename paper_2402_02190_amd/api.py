"""Python binding of the C ABI, one function per entry point, same names.

Each function only marshals arguments: torch tensors (device memory) become
raw pointers, the current torch stream becomes the hipStream_t, and a non-OK
status raises ``CpraError``.  All computation happens in libcpra's kernels.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (GCN, MAXCUT, MIS, SAGE, AdamCfg, CpraError, Csr, EarlyStopCfg,  # noqa: F401
                   EarlyStopState, LossCfg, ModelCfg, MpnnCfg, MpnnStepCfg, StepCfg, call)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_f32(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.float32):
        raise TypeError(f"{name} must be a float32 device tensor")


class DeviceGraph:
    """A CSR graph resident in device memory, with its prepared inv_deg and wdeg.

    ``row_ptr``, ``col_idx`` (int32), optional ``weight`` (float32) and optional
    ``graph_ptr`` (int32 node offsets of a block-diagonal batch) are host arrays.
    """

    def __init__(self, row_ptr, col_idx, weight=None, graph_ptr=None, device="cuda",
                 validate: bool = True):
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        n = row_ptr.size - 1
        if validate:
            csr_validate_host(row_ptr, col_idx, weight)
        self.n = n
        self.nnz = int(row_ptr[-1])
        self.row_ptr = torch.from_numpy(row_ptr).to(device)
        self.col_idx = torch.from_numpy(col_idx).to(device) if self.nnz else \
            torch.zeros(1, dtype=torch.int32, device=device)
        self.weight = None if weight is None else \
            torch.from_numpy(np.ascontiguousarray(weight, dtype=np.float32)).to(device)
        gp = None if graph_ptr is None else np.ascontiguousarray(graph_ptr, dtype=np.int32)
        self.n_graphs = 1 if gp is None else gp.size - 1
        self.graph_ptr = torch.from_numpy(gp).to(device) if (gp is not None and self.n_graphs > 1) else None
        self.inv_deg = torch.empty(max(n, 1), dtype=torch.float32, device=device)
        self.wdeg = torch.empty(max(n, 1), dtype=torch.float32, device=device)
        self.csr = Csr(n, self.n_graphs, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx),
                       _ptr(self.graph_ptr), _ptr(self.weight), None, None)
        csr_prepare(self, self.inv_deg, self.wdeg)
        self.csr.inv_deg = _ptr(self.inv_deg)
        self.csr.wdeg = _ptr(self.wdeg)
        # the column scale of M^T per CSR entry, read in order by the transposed aggregation
        self.col_inv_deg = torch.empty(max(self.nnz, 1), dtype=torch.float32, device=device)
        csr_prepare_col(self, self.col_inv_deg)
        self.csr.col_inv_deg = _ptr(self.col_inv_deg)

    @classmethod
    def from_csr(cls, g, device="cuda", validate=True):
        gp = g.graph_ptr if getattr(g, "graph_ptr", None) is not None and len(g.graph_ptr) > 2 else None
        return cls(g.row_ptr, g.col_idx, g.weight, gp, device, validate)

    @property
    def ref(self):
        return C.byref(self.csr)


def _csr(g) -> C.c_void_p:
    return C.byref(g.csr) if isinstance(g, DeviceGraph) else C.byref(g)


# ---------------------------------------------------------------------------
def abi_version() -> int:
    return int(_lib.lib().cpra_abi_version())


def csr_validate_host(row_ptr, col_idx, weight=None) -> None:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    w = None if weight is None else np.ascontiguousarray(weight, dtype=np.float32)
    call("cpra_csr_validate_host", rp.size - 1, int(rp[-1]), rp.ctypes.data,
         ci.ctypes.data if ci.size else None, None if w is None else w.ctypes.data)


def csr_prepare(g, inv_deg: Optional[torch.Tensor], wdeg: Optional[torch.Tensor], stream=None):
    call("cpra_csr_prepare", _csr(g), _ptr(inv_deg), _ptr(wdeg), _stream(stream))


def csr_prepare_col(g, col_inv_deg: torch.Tensor, stream=None):
    call("cpra_csr_prepare_col", _csr(g), _ptr(col_inv_deg), _stream(stream))


def aggregate_mean(g, X: torch.Tensor, Y: torch.Tensor, transpose: bool = False,
                   add: Optional[torch.Tensor] = None, bias: Optional[torch.Tensor] = None,
                   relu: bool = False, mask: Optional[torch.Tensor] = None, width: int = None,
                   stream=None) -> torch.Tensor:
    width = X.shape[1] if width is None else width
    call("cpra_aggregate_mean", _csr(g), int(transpose), width, _ptr(X), X.stride(0), _ptr(Y),
         Y.stride(0), _ptr(add), 0 if add is None else add.stride(0), _ptr(bias), int(relu),
         _ptr(mask), 0 if mask is None else mask.stride(0), _stream(stream))
    return Y


def gemm_workspace_bytes(trans_a, trans_b, M, N, K) -> int:
    return int(_lib.lib().cpra_gemm_workspace_bytes(int(trans_a), int(trans_b), M, N, K))


def gemm(A: torch.Tensor, B: torch.Tensor, C_out: torch.Tensor, trans_a=False, trans_b=False,
         beta: float = 0.0, bias=None, relu=False, ws: Optional[torch.Tensor] = None, stream=None):
    """C = act(op(A) op(B) + beta C + bias), row-major, op(A) [M,K], op(B) [K,N]."""
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[0] if trans_b else B.shape[1]
    if ws is None:
        nb = gemm_workspace_bytes(trans_a, trans_b, M, N, K)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=C_out.device) if nb else None
    call("cpra_gemm", int(trans_a), int(trans_b), M, N, K, _ptr(A), A.stride(0), _ptr(B),
         B.stride(0), float(beta), _ptr(C_out), C_out.stride(0), _ptr(bias), int(relu), _ptr(ws),
         0 if ws is None else ws.numel(), _stream(stream))
    return C_out


GROUP_ROWS, GROUP_K = 1, 2


def gemm_grouped_workspace_bytes(g, mode: int, M: int, N: int, with_bias_grad=False) -> int:
    return int(_lib.lib().cpra_gemm_grouped_workspace_bytes(_csr(g), int(mode), M, N,
                                                            int(with_bias_grad)))


def gemm_grouped_rows(g, A: torch.Tensor, B: torch.Tensor, C_out: torch.Tensor, trans_b=False,
                      bias: Optional[torch.Tensor] = None, relu=False, ws=None, stream=None):
    """Per graph g of the batch: C[rows of g] = act(A[rows of g] op(B[g]) + bias[g]).
    B [G, N, K] (trans_b) or [G, K, N]; bias [G, N] or None; A [n, K]; C [n, N]."""
    M, K = A.shape
    N = B.shape[1] if trans_b else B.shape[2]
    if ws is None:
        nb = gemm_grouped_workspace_bytes(g, GROUP_ROWS, M, N)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=C_out.device)
    call("cpra_gemm_grouped", _csr(g), GROUP_ROWS, int(trans_b), M, N, K, _ptr(A), A.stride(0),
         _ptr(B), B.stride(1), B.stride(0), _ptr(C_out), C_out.stride(0), 0, _ptr(bias),
         0 if bias is None else bias.stride(0), None, 0, int(relu), _ptr(ws), ws.numel(),
         _stream(stream))
    return C_out


def gemm_grouped_k(g, A: torch.Tensor, B: torch.Tensor, C_out: torch.Tensor,
                   bias_grad: Optional[torch.Tensor] = None, ws=None, stream=None):
    """Per graph g of the batch: C[g] = A[rows of g]^T B[rows of g] and optionally
    bias_grad[g] = the column sums of A over the rows of g.  A [n, M], B [n, N],
    C [G, M, N], bias_grad [G, M]."""
    K, M = A.shape
    N = B.shape[1]
    if ws is None:
        nb = gemm_grouped_workspace_bytes(g, GROUP_K, M, N, bias_grad is not None)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=C_out.device) if nb else None
    call("cpra_gemm_grouped", _csr(g), GROUP_K, 0, M, N, K, _ptr(A), A.stride(0), _ptr(B),
         B.stride(0), 0, _ptr(C_out), C_out.stride(1), C_out.stride(0), None, 0, _ptr(bias_grad),
         0 if bias_grad is None else bias_grad.stride(0), 0, _ptr(ws),
         0 if ws is None else ws.numel(), _stream(stream))
    return C_out


def _node_weight_args(node_weight: Optional[torch.Tensor]):
    """(pointer, leading dimension) of MIS node weights: [N] (ld 0) or [N, S]."""
    if node_weight is None:
        return None, 0
    _dev_f32(node_weight, "node_weight")
    if node_weight.dim() == 1:
        return node_weight.data_ptr(), 0
    return node_weight.data_ptr(), node_weight.stride(0)


def _edge_weight_args(edge_weight: Optional[torch.Tensor]):
    """(pointer, leading dimension) of per-head edge weights [nnz, S]."""
    if edge_weight is None:
        return None, 0
    _dev_f32(edge_weight, "edge_weight")
    if edge_weight.dim() != 2:
        raise ValueError("edge_weight must be [nnz, S]")
    return edge_weight.data_ptr(), edge_weight.stride(0)


def make_loss_cfg(problem: int, S: int, lam: Optional[torch.Tensor], alpha: int = 2,
                  gamma: float = 0.0, nu: float = 0.0, std_ddof: int = 0,
                  step_counter: Optional[torch.Tensor] = None, gamma_start: float = 0.0,
                  gamma_end: float = 0.0, T: int = 1,
                  node_weight: Optional[torch.Tensor] = None,
                  edge_weight: Optional[torch.Tensor] = None) -> LossCfg:
    """node_weight: optional MIS node weights, float32 [N] or [N, S] on the device;
    edge_weight: optional per-head edge weights, float32 [nnz, S] (one instance per
    head; symmetric).  The returned config keeps references to the tensors whose
    addresses it holds; a StepCfg built from it copies the struct, so keep this
    object (or the tensors) while the StepCfg is used."""
    nw, ld = _node_weight_args(node_weight)
    ew, lde = _edge_weight_args(edge_weight)
    cfg = LossCfg(problem, S, alpha, std_ddof, gamma, nu, _ptr(lam), _ptr(step_counter),
                  gamma_start, gamma_end, T, nw, ld, ew, lde)
    # the struct holds raw addresses: keep the tensors alive as long as this object
    cfg._tensors = (lam, step_counter, node_weight, edge_weight)
    return cfg


def loss_workspace_bytes(g, cfg: LossCfg) -> int:
    return int(_lib.lib().cpra_loss_workspace_bytes(_csr(g), C.byref(cfg)))


def loss_fwd_bwd(g, cfg: LossCfg, Z: torch.Tensor, dZ: Optional[torch.Tensor],
                 terms: Optional[torch.Tensor], ws: torch.Tensor, P: Optional[torch.Tensor] = None,
                 stream=None):
    call("cpra_loss_fwd_bwd", _csr(g), C.byref(cfg), _ptr(Z), Z.stride(0), _ptr(P),
         0 if P is None else P.stride(0), _ptr(dZ), 0 if dZ is None else dZ.stride(0),
         _ptr(terms), _ptr(ws), ws.numel(), _stream(stream))


def loss_fwd_bwd_noalloc(g, cfg: LossCfg, Z: torch.Tensor, dZ: Optional[torch.Tensor],
                         terms: Optional[torch.Tensor], P: Optional[torch.Tensor] = None,
                         stream=None):
    """cpra_loss_fwd_bwd with its workspace in the library's static device scratch
    (no allocation; calls that overlap in time on one GPU race)."""
    call("cpra_loss_fwd_bwd_noalloc", _csr(g), C.byref(cfg), _ptr(Z), Z.stride(0), _ptr(P),
         0 if P is None else P.stride(0), _ptr(dZ), 0 if dZ is None else dZ.stride(0),
         _ptr(terms), _stream(stream))


def loss_total(terms: torch.Tensor, gamma: float, nu: float, R: torch.Tensor, stream=None):
    """R (device, one float64) = the total loss from the per-graph terms [n_graphs, S+2]."""
    G, S2 = terms.shape
    call("cpra_loss_total", G, S2 - 2, _ptr(terms), float(gamma), float(nu), _ptr(R),
         _stream(stream))
    return R


def early_stop_reset(state: torch.Tensor, stream=None):
    """Initialise an early-stopping state (a device buffer of at least
    sizeof(cpra_early_stop_state) bytes)."""
    if state.numel() * state.element_size() < C.sizeof(EarlyStopState):
        raise ValueError("early-stopping state buffer too small")
    call("cpra_early_stop_reset", _ptr(state), _stream(stream))


def early_stop_read(state: torch.Tensor) -> dict:
    """The state as a dict (copies 32 bytes to the host; synchronises)."""
    raw = state.detach().cpu().numpy().tobytes()[: C.sizeof(EarlyStopState)]
    st = EarlyStopState.from_buffer_copy(raw)
    return {k: getattr(st, k) for k, _ in EarlyStopState._fields_}


def sigmoid(Z: torch.Tensor, P: torch.Tensor, stream=None):
    call("cpra_sigmoid", Z.shape[0], Z.shape[1], _ptr(Z), Z.stride(0), _ptr(P), P.stride(0),
         _stream(stream))
    return P


def make_model_cfg(layer_kind: int, n_layers: int, in_dim: int, hidden: int, S: int,
                   recompute: bool = False, z_offset: torch.Tensor = None,
                   train_from_layer: int = 0, reuse_frozen_prefix: bool = False,
                   weight_groups: int = 0) -> ModelCfg:
    """z_offset: optional float32 [N, S] contiguous device tensor of fixed logits added to
    the output (the warm start); the caller keeps it alive while the config is used.
    train_from_layer / reuse_frozen_prefix: a frozen encoder (see include/cpra.h).
    weight_groups: G > 1 gives every graph of a G-graph batch its own layer weights."""
    if z_offset is not None:
        if z_offset.dtype != torch.float32 or not z_offset.is_contiguous() or z_offset.dim() != 2 \
                or z_offset.shape[1] != S:
            raise ValueError("z_offset must be a contiguous float32 [N, S] tensor")
    cfg = ModelCfg(layer_kind, n_layers, in_dim, hidden, S, int(recompute),
                   None if z_offset is None else z_offset.data_ptr(), int(train_from_layer),
                   int(reuse_frozen_prefix), int(weight_groups))
    cfg._tensors = (z_offset,)  # kept alive with the struct that holds its address
    return cfg


def model_param_count(cfg: ModelCfg, n_nodes: int) -> int:
    n = int(_lib.lib().cpra_model_param_count(C.byref(cfg), n_nodes))
    if n < 0:
        raise CpraError(4, "invalid model config")
    return n


def model_param_offsets(cfg: ModelCfg, n_nodes: int):
    out = (C.c_int64 * (1 + 3 * cfg.n_layers))()
    call("cpra_model_param_offsets", C.byref(cfg), n_nodes, out)
    return list(out)


def model_workspace_bytes(g, cfg: ModelCfg) -> int:
    return int(_lib.lib().cpra_model_workspace_bytes(_csr(g), C.byref(cfg)))


def model_forward(g, cfg: ModelCfg, params: torch.Tensor, Z: torch.Tensor, ws: torch.Tensor,
                  stream=None):
    call("cpra_model_forward", _csr(g), C.byref(cfg), _ptr(params), _ptr(Z), Z.stride(0),
         _ptr(ws), ws.numel(), _stream(stream))
    return Z


def model_backward(g, cfg: ModelCfg, params: torch.Tensor, dZ: torch.Tensor, grads: torch.Tensor,
                   ws: torch.Tensor, stream=None):
    call("cpra_model_backward", _csr(g), C.byref(cfg), _ptr(params), _ptr(dZ), dZ.stride(0),
         _ptr(grads), _ptr(ws), ws.numel(), _stream(stream))
    return grads


def model_saved_activation(g, cfg: ModelCfg, ws: torch.Tensor, layer: int, n_nodes: int,
                           width: int) -> torch.Tensor:
    """A copy of the saved input of `layer` (the ReLU output of layer - 1)."""
    ptr = C.c_void_p()
    ld = C.c_int64()
    call("cpra_model_saved_activation", _csr(g), C.byref(cfg), _ptr(ws), ws.numel(), layer,
         C.byref(ptr), C.byref(ld))
    off = ptr.value - ws.data_ptr()
    flat = ws[off: off + n_nodes * ld.value * 4].view(torch.float32)
    return flat.view(n_nodes, ld.value)[:, :width].clone()


def adam_step(params, grads, m, v, cfg: AdamCfg, t: int = 1, step_counter=None, stream=None):
    call("cpra_adam_step", params.numel(), _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
         C.byref(cfg), int(t), _ptr(step_counter), _stream(stream))


def train_step_workspace_bytes(g, cfg: StepCfg) -> int:
    return int(_lib.lib().cpra_train_step_workspace_bytes(_csr(g), C.byref(cfg)))


def train_step(g, cfg: StepCfg, params, grads, m, v, Z, dZ, terms, ws, t: int = 1,
               step_counter=None, stream=None):
    call("cpra_train_step", _csr(g), C.byref(cfg), _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
         _ptr(Z), _ptr(dZ), _ptr(terms), int(t), _ptr(step_counter), _ptr(ws), ws.numel(),
         _stream(stream))


def round_eval_workspace_bytes(g, S: int) -> int:
    return int(_lib.lib().cpra_round_eval_workspace_bytes(_csr(g), S))


def round_eval(g, problem: int, Z: torch.Tensor, X=None, value=None, violations=None,
               wvalue=None, pair_hamming=None, ws=None, stream=None, node_weight=None,
               edge_weight=None):
    S = Z.shape[1]
    if ws is None:
        ws = torch.empty(round_eval_workspace_bytes(g, S), dtype=torch.uint8, device=Z.device)
    nw, ld = _node_weight_args(node_weight)
    ew, lde = _edge_weight_args(edge_weight)
    call("cpra_round_eval", _csr(g), problem, S, _ptr(Z), Z.stride(0), _ptr(X),
         0 if X is None else X.stride(0), _ptr(value), _ptr(violations), _ptr(wvalue),
         _ptr(pair_hamming), nw, ld, ew, lde, _ptr(ws), ws.numel(), _stream(stream))


def pairwise_hamming(X: torch.Tensor, D: Optional[torch.Tensor] = None,
                     hist: Optional[torch.Tensor] = None, n_unique: Optional[torch.Tensor] = None,
                     ws: Optional[torch.Tensor] = None, stream=None):
    """Pairwise Hamming distances / histogram / distinct count of the columns of
    a uint8 [N, S] device matrix of rounded solutions."""
    N, S = X.shape
    if ws is None:
        nb = int(_lib.lib().cpra_pairwise_hamming_workspace_bytes(N, S))
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=X.device)
    call("cpra_pairwise_hamming", N, S, _ptr(X), X.stride(0), _ptr(D), 0 if D is None else D.stride(0),
         _ptr(hist), _ptr(n_unique), _ptr(ws), ws.numel(), _stream(stream))


# ---------------------------------------------------------------- warm start
def node_features(g, in_dim: int, rand: Optional[torch.Tensor], feat: torch.Tensor,
                  triangles: Optional[torch.Tensor] = None, stream=None):
    """feat: int16 (bf16 bit patterns) [N, in_dim] device tensor; rand: float32
    [N, n_rand] or None; triangles: int64 [N] or None."""
    n_rand = 0 if rand is None else rand.shape[1]
    call("cpra_node_features", _csr(g), in_dim, n_rand, _ptr(rand),
         0 if rand is None else rand.stride(0), _ptr(feat), feat.stride(0), _ptr(triangles),
         _stream(stream))
    return feat


def make_mpnn_cfg(n_layers: int, in_dim: int, hidden: int, S: int) -> MpnnCfg:
    return MpnnCfg(n_layers, in_dim, hidden, S)


def mpnn_param_count(cfg: MpnnCfg) -> int:
    n = int(_lib.lib().cpra_mpnn_param_count(C.byref(cfg)))
    if n < 0:
        raise CpraError(4, "invalid mpnn config")
    return n


def mpnn_param_offsets(cfg: MpnnCfg):
    out = (C.c_int64 * (3 * cfg.n_layers))()
    call("cpra_mpnn_param_offsets", C.byref(cfg), out)
    return list(out)


def mpnn_workspace_bytes(g, cfg: MpnnCfg) -> int:
    return int(_lib.lib().cpra_mpnn_workspace_bytes(_csr(g), C.byref(cfg)))


def mpnn_forward(g, cfg: MpnnCfg, params, feat, Zw, ws, stream=None):
    call("cpra_mpnn_forward", _csr(g), C.byref(cfg), _ptr(params), _ptr(feat), _ptr(Zw),
         _ptr(ws), ws.numel(), _stream(stream))
    return Zw


def mpnn_backward(g, cfg: MpnnCfg, feat, dZw, grads, ws, stream=None):
    call("cpra_mpnn_backward", _csr(g), C.byref(cfg), _ptr(feat), _ptr(dZw), _ptr(grads),
         _ptr(ws), ws.numel(), _stream(stream))
    return grads


def mpnn_saved(g, cfg: MpnnCfg, ws: torch.Tensor, layer: int, which: int, n_nodes: int):
    """A copy (int16 bf16 patterns) of a tensor saved by the last mpnn_forward:
    which = 0: the input H of `layer` (>= 1); which = 1: its aggregate M H."""
    ptr = C.c_void_p()
    ld = C.c_int64()
    call("cpra_mpnn_saved", _csr(g), C.byref(cfg), _ptr(ws), ws.numel(), layer, which,
         C.byref(ptr), C.byref(ld))
    off = ptr.value - ws.data_ptr()
    flat = ws[off: off + n_nodes * ld.value * 2].view(torch.int16)
    return flat.view(n_nodes, ld.value).clone()


def bce_grad(Z: torch.Tensor, target: torch.Tensor, beta: float, dZ: torch.Tensor, stream=None):
    call("cpra_bce_grad", Z.shape[0], Z.shape[1], _ptr(Z), Z.stride(0), _ptr(target),
         target.stride(0), float(beta), _ptr(dZ), dZ.stride(0), _stream(stream))
    return dZ


def make_mpnn_step_cfg(net: MpnnCfg, loss: LossCfg, adam: AdamCfg, beta: float) -> MpnnStepCfg:
    return MpnnStepCfg(net, loss, adam, float(beta))


def mpnn_train_step_workspace_bytes(g, cfg: MpnnStepCfg) -> int:
    return int(_lib.lib().cpra_mpnn_train_step_workspace_bytes(_csr(g), C.byref(cfg)))


def mpnn_train_step(g, cfg: MpnnStepCfg, params, grads, m, v, feat, target, Zw, dZw, terms, ws,
                    t: int = 1, step_counter=None, stream=None):
    call("cpra_mpnn_train_step", _csr(g), C.byref(cfg), _ptr(params), _ptr(grads), _ptr(m),
         _ptr(v), _ptr(feat), _ptr(target), _ptr(Zw), _ptr(dZw), _ptr(terms), int(t),
         _ptr(step_counter), _ptr(ws), ws.numel(), _stream(stream))


def capture_begin(stream) -> None:
    call("cpra_capture_begin", stream.cuda_stream)


def capture_end(stream) -> C.c_void_p:
    h = C.c_void_p()
    call("cpra_capture_end", stream.cuda_stream, C.byref(h))
    return h


def graph_launch(graph, stream) -> None:
    call("cpra_graph_launch", graph, stream.cuda_stream)


def graph_destroy(graph) -> None:
    call("cpra_graph_destroy", graph)


def profile_begin() -> None:
    call("cpra_profile_begin")


def profile_stop() -> None:
    call("cpra_profile_stop")


def profile_collect() -> None:
    call("cpra_profile_collect")


def profile_end(collect: bool = True):
    """Stop profiling (collecting the recorded events first unless collect=False);
    returns {name: (launches, total_ms, flops, bytes, gathered bytes)}."""
    if collect:
        profile_collect()
    n = C.c_int32()
    call("cpra_profile_end", C.byref(n))
    out = {}
    for i in range(n.value):
        name = C.create_string_buffer(128)
        la, ms, fl, by, ga = C.c_int64(), C.c_double(), C.c_double(), C.c_double(), C.c_double()
        call("cpra_profile_get", i, name, 128, C.byref(la), C.byref(ms), C.byref(fl), C.byref(by),
             C.byref(ga))
        out[name.value.decode()] = (la.value, ms.value, fl.value, by.value, ga.value)
    return out


def autotune_begin() -> None:
    call("cpra_autotune_begin")


def autotune_end():
    """Stop tuning; returns [(shape key, chosen plan, us, heuristic us)] of the table."""
    n = C.c_int32()
    call("cpra_autotune_end", C.byref(n))
    return [(e["key"], e["choice"], e["us"], e["heuristic_us"]) for e in autotune_table(n.value)]


def autotune_table(n: int = None):
    """The tuning table as a list of dicts (key, cfg, splits, choice, us, heuristic_us)."""
    if n is None:
        c = C.c_int32()
        call("cpra_autotune_end", C.byref(c))  # reading the size also stops tuning
        n = c.value
    out = []
    for i in range(n):
        key, choice = C.create_string_buffer(256), C.create_string_buffer(64)
        cfg, splits = C.c_int32(), C.c_int32()
        us, hus = C.c_double(), C.c_double()
        call("cpra_autotune_get", i, key, 256, C.byref(cfg), C.byref(splits), choice, 64,
             C.byref(us), C.byref(hus))
        out.append({"key": key.value.decode(), "cfg": cfg.value, "splits": splits.value,
                    "choice": choice.value.decode(), "us": us.value, "heuristic_us": hus.value})
    return out


def autotune_set(key: str, cfg: int, splits: int) -> None:
    call("cpra_autotune_set", key.encode(), int(cfg), int(splits))


def autotune_reset() -> None:
    call("cpra_autotune_reset")
