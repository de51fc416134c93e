"""``torch.autograd.Function`` around the hand-written CPRA forward/backward.

``CPRALoss.apply(params, solver, gamma)`` returns the relaxed CPRA loss R
(a 0-dim float64 tensor, summed over the graphs of a batch).  The forward
runs ``cpra_model_forward`` (saving the activations in the solver's
workspace) and ``cpra_loss_fwd_bwd`` (which also produces dR/dZ); the
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
                                s.cfg.std_ddof)
        loss_ws = s.loss_workspace()
        api.loss_fwd_bwd(s.graph, cfg, s.Z, s.dZ, s.terms, loss_ws)
        ctx.solver = s
        ctx.save_for_backward(params)
        torch.cuda.synchronize()
        t = s.terms.cpu()
        S = s.cfg.S
        R = t[:, :S].sum() + float(gamma) * t[:, S].sum() + s.cfg.nu * t[:, S + 1].sum()
        return R.to(dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        s = ctx.solver
        grads = torch.empty_like(params)
        api.model_backward(s.graph, s.model_cfg, params, s.dZ, grads, s.ws)
        g = float(grad_out)
        if g != 1.0:
            grads.mul_(g)
        return grads, None, None
