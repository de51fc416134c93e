"""One CPRA training step and the training loop, in float64.  TEST INFRASTRUCTURE ONLY.

The loop (Sec. 3.1 with the settings of Sec. 4.1 Implementation and the
training-setting appendix): at every epoch (one full-graph gradient step)
compute P = sigmoid(GNN_theta(G)), the loss R with the current gamma, its
gradient, and update theta with Adam (Kingma and Ba) or AdamW (decoupled
weight decay).  After the last epoch the relaxed solutions are rounded.

gamma schedule: the paper starts from gamma(0) < 0 and raises gamma by a
fixed rate each epoch (Sec. 4.1 Implementation: gamma(0) = -20 for MIS,
rate 1e-3).  ``gamma_at`` implements the linear schedule between two
endpoints over T epochs, both endpoints included; ``gamma_paper`` the
additive form gamma(0) + rate * t.
"""

from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Dict, List, Optional

import numpy as np

from . import evaluate, gnn, objective


def gamma_at(t: int, T: int, gamma_start: float, gamma_end: float) -> float:
    """Linear schedule, gamma_0 = gamma_start and gamma_{T-1} = gamma_end."""
    if T <= 1:
        return float(gamma_end)
    return float(gamma_start + (gamma_end - gamma_start) * (t / (T - 1)))


def gamma_paper(t: int, gamma0: float, rate: float) -> float:
    return float(gamma0 + rate * t)


def early_stop_step(head, phi, tol: float, patience: int,
                    relative: bool = False) -> Optional[int]:
    """Early stopping (Sec. 4.1 Implementation; training-setting appendix): the
    summed head loss L_t = sum_s l_hat(P_:s) and the annealing term
    Phi_t = gamma_t * S(P_t) are monitored with a tolerance and a patience.

    Reading of the rule: step t >= 1 is stalled when neither monitored value fell
    by more than the tolerance -- absolute (the paper states a plain tolerance),
    or with ``relative`` scaled by the previous value's magnitude:
        L_t - L_{t-1} >= -tol_L  and  Phi_t - Phi_{t-1} >= -tol_Phi;
    training stops at the first step that completes `patience` consecutive
    stalled steps.  Returns that step's index, or None if the sequences end first.
    """
    run = 0
    for t in range(1, len(head)):
        dl = head[t] - head[t - 1]
        dp = phi[t] - phi[t - 1]
        tl = tol * abs(head[t - 1]) if relative else tol
        tp = tol * abs(phi[t - 1]) if relative else tol
        if dl >= -tl and dp >= -tp:
            run += 1
            if run >= patience:
                return t
        else:
            run = 0
    return None


def adam_update(theta: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
                lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                weight_decay: float = 0.0):
    """One Adam step (t >= 1), in place.  weight_decay > 0 gives AdamW's decoupled decay.

    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
    theta <- theta (1 - lr wd) - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
    """
    m *= beta1
    m += (1.0 - beta1) * g
    v *= beta2
    v += (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    if weight_decay:
        theta *= (1.0 - lr * weight_decay)
    theta -= lr * mhat / (np.sqrt(vhat) + eps)


@dataclass
class StepConfig:
    problem: str
    lam: Optional[np.ndarray]
    alpha: int = 2
    nu: float = 0.0
    ddof: int = 0
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    weight_decay: float = 0.0
    node_weight: Optional[np.ndarray] = None  # MIS node weights [N] or [N, S]; None = 1
    edge_weight: Optional[np.ndarray] = None  # one instance per head: [nnz, S]; None = the graph's


def loss_and_grads(params, M, graph, cfg: StepConfig, gamma: float, relu_active=None,
                   return_cache: bool = False, z_offset=None):
    """Forward, loss terms (per graph of a batch) and all parameter gradients.

    ``relu_active``: optional ReLU decisions per hidden layer (see gnn.backward).
    ``z_offset``: optional warm-start logits added to the output (see gnn.forward)."""
    Z, cache = gnn.forward(params, M, z_offset)
    gp = np.asarray(graph.graph_ptr, dtype=np.int64)
    nw, ew = cfg.node_weight, cfg.edge_weight
    if gp.size > 2:
        terms = objective.batched_loss_terms(Z, graph, cfg.problem, cfg.lam, gamma, cfg.alpha,
                                             cfg.nu, cfg.ddof, nw, ew)
        dZ = np.zeros_like(Z)
        for g in range(gp.size - 1):
            lo, hi = int(gp[g]), int(gp[g + 1])
            sub = objective._slice_graph(graph, lo, hi)
            nwg = None if nw is None else np.asarray(nw)[lo:hi]
            a, b = objective.entry_range(graph, lo, hi)
            ewg = None if ew is None else np.asarray(ew)[a:b]
            dZ[lo:hi] = objective.grad_wrt_Z(Z[lo:hi], sub, cfg.problem, cfg.lam, gamma,
                                             cfg.alpha, cfg.nu, cfg.ddof, nwg, ewg)
    else:
        terms = [objective.loss_terms(Z, graph, cfg.problem, cfg.lam, gamma, cfg.alpha,
                                      cfg.nu, cfg.ddof, nw, ew)]
        dZ = objective.grad_wrt_Z(Z, graph, cfg.problem, cfg.lam, gamma, cfg.alpha, cfg.nu,
                                  cfg.ddof, nw, ew)
    grads = gnn.backward(params, M, cache, dZ, relu_active)
    if return_cache:
        return Z, terms, dZ, grads, cache
    return Z, terms, dZ, grads


def graph_params(params, b: int, lo: int, hi: int):
    """The network of graph b of a batch with per-graph weights: rows lo..hi-1 of
    the embedding and entry b (leading index) of every layer's Ws, Wn and b."""
    return {"emb": params["emb"][lo:hi],
            "layers": [{k: v[b] for k, v in L.items()} for L in params["layers"]]}


def loss_and_grads_per_graph(params, graph, cfg: StepConfig, gamma: float, relu_active=None,
                             z_offset=None):
    """Forward, loss terms and gradients of a block-diagonal batch in which every
    graph has its own network (layer weights with a leading graph index).

    Each graph is then an independent CPRA problem (Sec. 3.1 applied per
    instance; the multi-instance use of the heads in Sec. 3.1's last paragraph
    and the DBM experiment, here with one network per instance): it is cut out
    of the batch and handed to ``loss_and_grads`` alone, with its rows of the
    embedding, node weights, z_offset and ReLU decisions, and its results are
    put back in place.  Returns (Z, terms per graph, dZ, grads) in the batch's
    layout, the layer gradients with the same leading graph index."""
    gp = np.asarray(graph.graph_ptr, dtype=np.int64)
    emb = params["emb"]
    S = params["layers"][-1]["Ws"].shape[1]
    N = emb.shape[0]
    Z = np.zeros((N, S))
    dZ = np.zeros((N, S))
    grads = {"emb": np.zeros_like(emb),
             "layers": [{k: np.zeros_like(v) for k, v in L.items()} for L in params["layers"]]}
    terms = []
    nw = None if cfg.node_weight is None else np.asarray(cfg.node_weight)
    ew = None if cfg.edge_weight is None else np.asarray(cfg.edge_weight)
    for b in range(gp.size - 1):
        lo, hi = int(gp[b]), int(gp[b + 1])
        sub = objective._slice_graph(graph, lo, hi)
        M = gnn.mean_aggregation_matrix(sub.row_ptr, sub.col_idx)
        ea, eb = objective.entry_range(graph, lo, hi)
        cfg_b = replace(cfg, node_weight=None if nw is None else nw[lo:hi],
                        edge_weight=None if ew is None else ew[ea:eb])
        ra = None if relu_active is None else [m[lo:hi] for m in relu_active]
        zo = None if z_offset is None else np.asarray(z_offset)[lo:hi]
        Zb, tb, dZb, gb = loss_and_grads(graph_params(params, b, lo, hi), M, sub, cfg_b, gamma,
                                         ra, z_offset=zo)
        Z[lo:hi] = Zb
        dZ[lo:hi] = dZb
        terms.extend(tb)
        grads["emb"][lo:hi] = gb["emb"]
        for Lg, Lb in zip(grads["layers"], gb["layers"]):
            for k in Lg:
                Lg[k][b] = Lb[k]
    return Z, terms, dZ, grads


class AdamState:
    def __init__(self, params):
        self.m = {"emb": np.zeros_like(params["emb"]),
                  "layers": [{k: np.zeros_like(v) for k, v in L.items()} for L in params["layers"]]}
        self.v = {"emb": np.zeros_like(params["emb"]),
                  "layers": [{k: np.zeros_like(v) for k, v in L.items()} for L in params["layers"]]}
        self.t = 0

    def step(self, params, grads, cfg: StepConfig):
        self.t += 1
        adam_update(params["emb"], grads["emb"], self.m["emb"], self.v["emb"], self.t, cfg.lr,
                    cfg.beta1, cfg.beta2, cfg.eps, cfg.weight_decay)
        for L, G, Mm, Vv in zip(params["layers"], grads["layers"], self.m["layers"],
                                self.v["layers"]):
            for k in L:
                adam_update(L[k], G[k], Mm[k], Vv[k], self.t, cfg.lr, cfg.beta1, cfg.beta2,
                            cfg.eps, cfg.weight_decay)


def solve(params_f32, graph, cfg: StepConfig, T: int, gamma_start: float, gamma_end: float,
          record_every: int = 0, z_offset=None) -> Dict[str, object]:
    """Run T training steps from the given initial parameters; round and evaluate."""
    params = gnn.to_f64(params_f32)
    M = gnn.mean_aggregation_matrix(graph.row_ptr, graph.col_idx)
    opt = AdamState(params)
    history: List[Dict[str, object]] = []
    for t in range(T):
        gamma = gamma_at(t, T, gamma_start, gamma_end)
        Z, terms, dZ, grads = loss_and_grads(params, M, graph, cfg, gamma, z_offset=z_offset)
        if record_every and (t % record_every == 0 or t == T - 1):
            history.append({"t": t, "gamma": gamma, "terms": terms})
        opt.step(params, grads, cfg)
    Z, _ = gnn.forward(params, M, z_offset)
    X = evaluate.round_solutions(Z)
    ev = evaluate.evaluate(X, graph, cfg.problem)
    return {"Z": Z, "X": X, "eval": ev, "params": params, "history": history}
