"""The learned warm start: node features and the BF16 message-passing network.

Every step runs in libcpra's kernels (cpra_node_features, cpra_mpnn_*); this
module holds the parameters, packs and unpacks them, and keeps the device
buffers.  The network's output Z_w is handed to CPRA as
``CPRAConfig(z_offset=...)``: P = sigmoid(GNN(G) + Z_w).
"""

from __future__ import annotations

from typing import Dict, Optional

import numpy as np
import torch

from . import api


class WarmStartNet:
    """Parameters (float32 masters), Adam state and workspaces of the network."""

    def __init__(self, n_layers: int = 3, in_dim: int = 16, hidden: int = 64, S: int = 32,
                 n_rand: int = 14, device: str = "cuda"):
        if 2 + n_rand > in_dim:
            raise ValueError("in_dim must hold degree, clustering and the random channels")
        self.cfg = api.make_mpnn_cfg(n_layers, in_dim, hidden, S)
        self.n_layers, self.in_dim, self.hidden, self.S, self.n_rand = n_layers, in_dim, hidden, S, n_rand
        self.device = device
        self.n_params = api.mpnn_param_count(self.cfg)
        self.offsets = api.mpnn_param_offsets(self.cfg)
        self.params = torch.zeros(self.n_params, dtype=torch.float32, device=device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_counter = torch.zeros(1, dtype=torch.int32, device=device)

    # ---- parameters
    def dims(self):
        d, out = self.in_dim, []
        for k in range(self.n_layers):
            o = self.S if k == self.n_layers - 1 else self.hidden
            out.append((d, o))
            d = o
        return out

    def pack(self, p: Dict[str, object]) -> np.ndarray:
        flat = np.zeros(self.n_params, dtype=np.float32)
        for k, (d_in, d_out) in enumerate(self.dims()):
            L = p["layers"][k]
            o_ws, o_wn, o_b = self.offsets[3 * k:3 * k + 3]
            flat[o_ws:o_ws + d_out * d_in] = np.asarray(L["Ws"], dtype=np.float32).ravel()
            flat[o_wn:o_wn + d_out * d_in] = np.asarray(L["Wn"], dtype=np.float32).ravel()
            flat[o_b:o_b + d_out] = np.asarray(L["b"], dtype=np.float32).ravel()
        return flat

    def unpack(self, flat) -> Dict[str, object]:
        if isinstance(flat, torch.Tensor):
            flat = flat.detach().cpu().numpy()
        layers = []
        for k, (d_in, d_out) in enumerate(self.dims()):
            o_ws, o_wn, o_b = self.offsets[3 * k:3 * k + 3]
            layers.append({"Ws": flat[o_ws:o_ws + d_out * d_in].reshape(d_out, d_in).copy(),
                           "Wn": flat[o_wn:o_wn + d_out * d_in].reshape(d_out, d_in).copy(),
                           "b": flat[o_b:o_b + d_out].copy()})
        return {"layers": layers}

    def load_params(self, p: Dict[str, object]) -> None:
        self.params.copy_(torch.from_numpy(self.pack(p)).to(self.device))
        self.m.zero_()
        self.v.zero_()
        self.step_counter.zero_()

    def save(self, path: str) -> None:
        np.savez(path, params=self.params.cpu().numpy(),
                 shape=np.array([self.n_layers, self.in_dim, self.hidden, self.S, self.n_rand]))

    @classmethod
    def load(cls, path: str, device: str = "cuda") -> "WarmStartNet":
        z = np.load(path)
        L, in_dim, hidden, S, n_rand = (int(x) for x in z["shape"])
        net = cls(L, in_dim, hidden, S, n_rand, device)
        net.params.copy_(torch.from_numpy(z["params"]).to(device))
        return net

    # ---- device computations
    def features(self, dg, rand: Optional[np.ndarray], triangles: bool = False, stream=None):
        """bf16 feature matrix [N, in_dim] (int16 bit patterns) of a device graph."""
        feat = torch.empty((max(dg.n, 1), self.in_dim), dtype=torch.int16, device=self.device)
        r = None
        if self.n_rand:
            if rand is None or rand.shape != (dg.n, self.n_rand):
                raise ValueError(f"rand must be float32 [{dg.n}, {self.n_rand}]")
            r = torch.from_numpy(np.ascontiguousarray(rand, dtype=np.float32)).to(self.device)
        tri = torch.empty(max(dg.n, 1), dtype=torch.int64, device=self.device) if triangles else None
        api.node_features(dg, self.in_dim, r, feat, tri, stream)
        return (feat, tri) if triangles else feat

    def workspace(self, dg) -> torch.Tensor:
        return torch.empty(max(api.mpnn_workspace_bytes(dg, self.cfg), 256), dtype=torch.uint8,
                           device=self.device)

    def forward(self, dg, feat, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Z_w [N, S] float32."""
        if ws is None:
            ws = self.workspace(dg)
        Zw = torch.empty((max(dg.n, 1), self.S), dtype=torch.float32, device=self.device)
        api.mpnn_forward(dg, self.cfg, self.params, feat, Zw, ws, stream)
        return Zw
