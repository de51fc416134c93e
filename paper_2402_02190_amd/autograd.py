"""``torch.autograd.Function`` around the hand-written CPRA forward/backward.

``CPRALoss.apply(params, solver, gamma)`` returns the relaxed CPRA loss R
(a 0-dim float64 device tensor, summed over the graphs of a batch).  The
forward runs ``cpra_model_forward`` (saving the activations in the solver's
workspace), ``cpra_loss_fwd_bwd`` (which also produces dR/dZ) with the
solver's own objective (node weights, per-head instances) at the given
gamma, and ``cpra_loss_total``, all stream-ordered without a host copy; the
backward runs ``cpra_model_backward`` on that dR/dZ, so torch's autograd
never traces the GNN.  ``params`` must be the solver's flat parameter
tensor (or a tensor of the same layout).
"""

from __future__ import annotations

import torch

from . import api


class CPRALoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, solver, gamma: float):
        s = solver
        api.model_forward(s.graph, s.model_cfg, params, s.Z, s.ws)
        cfg = api.make_loss_cfg(s.problem_id, s.cfg.S, s.lam, s.cfg.alpha, float(gamma), s.cfg.nu,
                                s.cfg.std_ddof, node_weight=s.node_weight,
                                edge_weight=s.edge_weight)
        loss_ws = s.loss_workspace()
        api.loss_fwd_bwd(s.graph, cfg, s.Z, s.dZ, s.terms, loss_ws)
        ctx.solver = s
        ctx.save_for_backward(params)
        R = torch.empty((), dtype=torch.float64, device=params.device)
        api.loss_total(s.terms, float(gamma), s.cfg.nu, R)
        return R

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        s = ctx.solver
        grads = torch.empty_like(params)
        api.model_backward(s.graph, s.model_cfg, params, s.dZ, grads, s.ws)
        grads.mul_(grad_out.to(dtype=grads.dtype))  # stream-ordered, no host read
        return grads, None, None
