"""CPRA solver: device buffers, the training loop and decoding.

The solver owns the flat parameter vector, its gradient and Adam moments,
the logits Z and dZ, the per-graph loss terms and one workspace, all as
torch device tensors.  Each training step is one ``cpra_train_step`` call
(forward, loss, hand-written backward, Adam) on one stream; with
``use_graph`` the step is captured once into a HIP graph and replayed.  The
annealing weight gamma and Adam's step number come from a device counter
that the step itself advances, so eager and replayed steps are identical.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import torch

from . import api
from .api import DeviceGraph


@dataclass
class CPRAConfig:
    problem: str = "mis"          # "mis" or "maxcut"
    layer_kind: str = "gcn"       # "gcn" or "sage"
    n_layers: int = 2
    hidden: int = 32
    S: int = 10
    in_dim: Optional[int] = None  # embedding width (default: hidden)
    alpha: int = 2
    nu: float = 0.0
    std_ddof: int = 0
    gamma_start: float = -2.0
    gamma_end: float = 0.1
    T: int = 2000
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    weight_decay: float = 0.0
    recompute: bool = False
    train_from_layer: int = 0  # > 0: layers below (and the embedding) are frozen
    per_graph_weights: bool = False  # batches: every graph its own layer weights


def gamma_schedule(t: int, T: int, g0: float, g1: float) -> float:
    """gamma_t = g0 + (g1 - g0) * min(t, T-1) / (T-1): the device formula, on the host."""
    if T <= 1:
        return float(g1)
    return float(np.float32(g0 + (g1 - g0) * (min(t, T - 1) / (T - 1))))


class CPRASolver:
    """z_offset (optional): float32 [N, S] device tensor of fixed logits added to the
    GNN's output (a learned warm start); the solver keeps a reference to it.
    node_weight (optional, MIS): node weights [N] or [N, S].
    edge_weight (optional): per-head edge weights [nnz, S], symmetric -- one instance
    per head on the graph's pattern (a zero leaves the edge out of that head's
    instance); they replace the graph's own weights in the objective and the
    evaluation."""

    def __init__(self, graph: DeviceGraph, cfg: CPRAConfig, lam=None, device="cuda",
                 z_offset: Optional[torch.Tensor] = None,
                 node_weight: Optional[np.ndarray] = None,
                 edge_weight: Optional[np.ndarray] = None):
        if cfg.problem not in ("mis", "maxcut"):
            raise ValueError("problem must be 'mis' or 'maxcut'")
        self.graph = graph
        self.cfg = cfg
        self.device = device
        N, S = graph.n, cfg.S
        self.problem_id = api.MIS if cfg.problem == "mis" else api.MAXCUT
        in_dim = cfg.hidden if cfg.in_dim is None else cfg.in_dim
        if z_offset is not None and tuple(z_offset.shape) != (N, S):
            raise ValueError(f"z_offset must be [{N}, {S}]")
        self.z_offset = z_offset
        # weight sets: one per graph of the batch, or one shared (reported as 0)
        self.G = graph.n_graphs if cfg.per_graph_weights and graph.n_graphs > 1 else 0
        self.model_cfg = api.make_model_cfg(api.SAGE if cfg.layer_kind == "sage" else api.GCN,
                                            cfg.n_layers, in_dim, cfg.hidden, S, cfg.recompute,
                                            z_offset, cfg.train_from_layer,
                                            weight_groups=self.G)
        if cfg.problem == "mis":
            if lam is None:
                raise ValueError("MIS needs a penalty grid lambda [S]")
            lam = np.asarray(lam, dtype=np.float32)
            if lam.shape != (S,):
                raise ValueError("lambda must have S entries")
            self.lam = torch.from_numpy(lam).to(device)
        else:
            self.lam = None
        self.step_counter = torch.zeros(1, dtype=torch.int32, device=device)  # steps done
        self.node_weight = None  # weighted MIS: float32 [N] or [N, S]
        if node_weight is not None:
            nw = np.ascontiguousarray(node_weight, dtype=np.float32)
            if nw.shape not in ((N,), (N, S)):
                raise ValueError(f"node weights must be [{N}] or [{N}, {S}]")
            self.node_weight = torch.from_numpy(nw).to(device)
        self.edge_weight = None  # one instance per head: float32 [nnz, S]
        if edge_weight is not None:
            ew = np.ascontiguousarray(edge_weight, dtype=np.float32)
            if ew.shape != (graph.nnz, S):
                raise ValueError(f"per-head edge weights must be [{graph.nnz}, {S}]")
            self.edge_weight = torch.from_numpy(ew).to(device)
        self.loss_cfg = api.make_loss_cfg(self.problem_id, S, self.lam, cfg.alpha, 0.0, cfg.nu,
                                          cfg.std_ddof, None, cfg.gamma_start, cfg.gamma_end, cfg.T,
                                          self.node_weight, self.edge_weight)
        self.adam_cfg = api.AdamCfg(cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, cfg.weight_decay)
        self.step_cfg = api.StepCfg(self.model_cfg, self.loss_cfg, self.adam_cfg)
        self.n_params = api.model_param_count(self.model_cfg, N)
        self.offsets = api.model_param_offsets(self.model_cfg, N)
        f32 = dict(dtype=torch.float32, device=device)
        self.params = torch.zeros(self.n_params, **f32)
        self.grads = torch.zeros(self.n_params, **f32)
        self.m = torch.zeros(self.n_params, **f32)
        self.v = torch.zeros(self.n_params, **f32)
        self.Z = torch.zeros((max(N, 1), S), **f32)
        self.dZ = torch.zeros((max(N, 1), S), **f32)
        self.terms = torch.zeros((graph.n_graphs, S + 2), dtype=torch.float64, device=device)
        nb = api.train_step_workspace_bytes(graph, self.step_cfg)
        self.ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=device)
        self.t = 0
        self._graph = None
        self._graph_k = None  # (graph of k consecutive steps, k), k > 1
        self._stream = None

    def set_reuse_frozen_prefix(self, on: bool) -> None:
        """Start later forwards at the first trained layer from the activations the
        previous forward saved (valid with a frozen encoder, after one full forward)."""
        if on and self.cfg.train_from_layer < 1:
            raise ValueError("reusing the frozen prefix needs train_from_layer >= 1")
        self.model_cfg.reuse_frozen_prefix = int(on)
        self.step_cfg.model.reuse_frozen_prefix = int(on)
        self.close()  # a captured step would keep the old choice

    # -- parameters ---------------------------------------------------------
    def load_params(self, p: Dict[str, object]) -> None:
        """Copy {"emb", "layers": [{"Ws","Wn"[,"b"]}]} float32 arrays into the flat layout
        (with per-graph weights, Ws / Wn [G, out, in] and b [G, out])."""
        flat = np.zeros(self.n_params, dtype=np.float32)
        emb = np.asarray(p["emb"], dtype=np.float32)
        flat[: emb.size] = emb.ravel()
        in_dim = self.model_cfg.in_dim
        for k, L in enumerate(p["layers"]):
            ows, own, ob = self.offsets[1 + 3 * k: 4 + 3 * k]
            d_out = self.cfg.S if k == self.model_cfg.n_layers - 1 else self.cfg.hidden
            d_in = in_dim if k == 0 else self.cfg.hidden
            want = (self.G, d_out, d_in) if self.G else (d_out, d_in)
            if tuple(np.shape(L["Ws"])) != want or tuple(np.shape(L["Wn"])) != want:
                raise ValueError(f"layer {k}: Ws and Wn must be {want}")
            flat[ows: ows + L["Ws"].size] = np.asarray(L["Ws"], np.float32).ravel()
            flat[own: own + L["Wn"].size] = np.asarray(L["Wn"], np.float32).ravel()
            if ob >= 0:
                flat[ob: ob + L["b"].size] = np.asarray(L["b"], np.float32).ravel()
        self.params.copy_(torch.from_numpy(flat))
        self.m.zero_()
        self.v.zero_()
        self.step_counter.zero_()
        self.t = 0

    def unpack(self, flat: torch.Tensor) -> Dict[str, object]:
        """Inverse of load_params for any flat vector (params or grads), as numpy."""
        a = flat.detach().cpu().numpy()
        N = self.graph.n
        in_dim = self.model_cfg.in_dim
        out = {"emb": a[: N * in_dim].reshape(N, in_dim).copy(), "layers": []}
        d_in = in_dim
        G = max(self.G, 1)
        lead = (self.G,) if self.G else ()
        for k in range(self.model_cfg.n_layers):
            d_out = self.cfg.S if k == self.model_cfg.n_layers - 1 else self.cfg.hidden
            ows, own, ob = self.offsets[1 + 3 * k: 4 + 3 * k]
            n = G * d_out * d_in
            L = {"Ws": a[ows: ows + n].reshape(lead + (d_out, d_in)).copy(),
                 "Wn": a[own: own + n].reshape(lead + (d_out, d_in)).copy()}
            if ob >= 0:
                L["b"] = a[ob: ob + G * d_out].reshape(lead + (d_out,)).copy()
            out["layers"].append(L)
            d_in = d_out
        return out

    def relu_active(self):
        """Per hidden layer, the boolean [N, hidden] ReLU decisions of the last forward."""
        out = []
        for k in range(1, self.model_cfg.n_layers):
            H = api.model_saved_activation(self.graph, self.model_cfg, self.ws, k, self.graph.n,
                                           self.cfg.hidden)
            out.append((H > 0).cpu().numpy())
        return out

    def loss_workspace(self) -> torch.Tensor:
        """A workspace for standalone loss calls (computes P itself), allocated once."""
        if getattr(self, "_loss_ws", None) is None:
            nb = api.loss_workspace_bytes(self.graph, self.loss_cfg)
            self._loss_ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
        return self._loss_ws

    # -- training -----------------------------------------------------------
    def step(self, stream=None) -> None:
        """One eager training step with gamma and t from the device counter."""
        api.train_step(self.graph, self.step_cfg, self.params, self.grads, self.m, self.v, self.Z,
                       self.dZ, self.terms, self.ws, 1, self.step_counter, stream)
        self.t += 1

    def autotune(self):
        """One eager training step with the GEMM autotuner on (tile shapes and split
        counts timed per problem shape); returns the tuning table.  The step is a real
        training step: the device counter advances."""
        api.autotune_begin()
        try:
            self.step()
            torch.cuda.synchronize()
        finally:
            table = api.autotune_end()
        return table

    def capture_step(self, steps: int = 1):
        """Record `steps` consecutive training steps into a new HIP graph on the
        solver's private stream and return its handle (the caller destroys it).
        Adam's step index comes from the device step counter, which every step
        advances, so the recorded steps are the same step repeated."""
        if self._stream is None:
            self._stream = torch.cuda.Stream()
        self._stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self._stream):
            api.capture_begin(self._stream)
            try:
                for _ in range(steps):
                    api.train_step(self.graph, self.step_cfg, self.params, self.grads, self.m,
                                   self.v, self.Z, self.dZ, self.terms, self.ws, 1,
                                   self.step_counter, self._stream)
            finally:
                g = api.capture_end(self._stream)
        return g

    def capture(self, steps_per_graph: int = 1) -> None:
        """Record one training step into the solver's HIP graph (once) and, with
        steps_per_graph = k > 1, also k consecutive steps into a second graph:
        replays then launch one graph per k steps, which saves the idle time
        between two launches of a graph (several microseconds each) inside
        the k steps."""
        if self._graph is None:
            self._graph = self.capture_step()
        if steps_per_graph > 1 and (self._graph_k is None or self._graph_k[1] != steps_per_graph):
            if self._graph_k is not None:
                api.graph_destroy(self._graph_k[0])
                self._graph_k = None
            self._graph_k = (self.capture_step(steps_per_graph), steps_per_graph)

    def launch_plan(self, n: int):
        """The graph launches that replay n steps: [(graph, steps it runs), ...],
        the k-step graph as often as it fits, then the one-step graph."""
        if self._graph is None:
            self.capture()
        plan = []
        if self._graph_k is not None:
            gk, k = self._graph_k
            plan += [(gk, k)] * (n // k)
            n -= (n // k) * k
        return plan + [(self._graph, 1)] * n

    def replay(self, n: int = 1) -> None:
        plan = self.launch_plan(n)
        self._stream.wait_stream(torch.cuda.current_stream())
        for g, _ in plan:
            api.graph_launch(g, self._stream)
        torch.cuda.current_stream().wait_stream(self._stream)
        self.t += n

    def run(self, steps: int, use_graph: bool = True) -> None:
        if use_graph:
            self.replay(steps)
        else:
            for _ in range(steps):
                self.step()

    # -- early stopping ------------------------------------------------------
    def enable_early_stopping(self, tol: float = 1e-5, patience: int = 1000,
                              relative: bool = False) -> None:
        """Turn on the device-side stopping rule of Sec. 4.1 (the summed head loss and the
        annealing term monitored with a tolerance -- absolute, as the paper's, or relative
        to the previous value -- and a patience; see cpra_early_stop_cfg): every later
        step, eager or replayed, updates the rule's state, and a step that fires it
        leaves the parameters as they are."""
        if getattr(self, "_es_state", None) is None:
            self._es_state = torch.zeros(64, dtype=torch.uint8, device=self.device)
        api.early_stop_reset(self._es_state)
        self.step_cfg.early_stop = api.EarlyStopCfg(float(tol), int(patience), int(relative),
                                                    self._es_state.data_ptr())
        self.close()  # a captured step would keep the old configuration

    def disable_early_stopping(self) -> None:
        self.step_cfg.early_stop = api.EarlyStopCfg(0.0, 0, 0, None)
        self.close()

    def early_stop_state(self) -> Dict[str, object]:
        """{prev_head, prev_phi, stalled, stopped, stop_step, seen} (synchronises)."""
        if getattr(self, "_es_state", None) is None:
            raise RuntimeError("early stopping is not enabled")
        return api.early_stop_read(self._es_state)

    def run_with_early_stopping(self, steps: int, check_every: int = 50):
        """Replay up to `steps` steps, reading the device's stop flag (4 bytes) every
        `check_every` steps.  Returns (steps replayed, index of the step that fired the
        rule or None).  Steps replayed after the rule fired change nothing."""
        if self.step_cfg.early_stop.state is None:
            raise RuntimeError("enable_early_stopping() first")
        done = 0
        while done < steps:
            n = min(check_every, steps - done)
            self.replay(n)
            done += n
            st = self.early_stop_state()
            if st["stopped"]:
                return done, int(st["stop_step"])
        return done, None

    def run_until_binary(self, steps: int, eps: float = 1e-4, check_every: int = 50) -> int:
        """Replay up to `steps` steps, stopping early once the annealing term per entry,
        S(P) / (N S), falls below eps (checked every `check_every` steps: the
        stopping rule of the training-setting appendix and the two-stage appendix).
        Returns the number of steps run."""
        done = 0
        N, S = self.graph.n, self.cfg.S
        while done < steps:
            n = min(check_every, steps - done)
            self.replay(n)
            done += n
            if float(self.terms_host()[:, S].sum()) / max(1, N * S) < eps:
                break
        return done

    def forward(self, stream=None) -> torch.Tensor:
        """Z = GNN(params) without a parameter update."""
        api.model_forward(self.graph, self.model_cfg, self.params, self.Z, self.ws, stream)
        return self.Z

    def evaluate(self, Z: Optional[torch.Tensor] = None) -> Dict[str, np.ndarray]:
        """Round at P > 0.5 and evaluate every head of every graph (exact integers)."""
        Z = self.Z if Z is None else Z
        G, S = self.graph.n_graphs, self.cfg.S
        dev = self.device
        X = torch.empty((max(self.graph.n, 1), S), dtype=torch.uint8, device=dev)
        value = torch.empty(G * S, dtype=torch.int64, device=dev)
        viol = torch.empty(G * S, dtype=torch.int64, device=dev)
        ph = torch.empty(G, dtype=torch.int64, device=dev)
        weighted = (self.graph.weight is not None or self.node_weight is not None or
                    self.edge_weight is not None)
        wv = torch.empty(G * S, dtype=torch.float64, device=dev) if weighted else None
        api.round_eval(self.graph, self.problem_id, Z, X, value, viol, wv, ph,
                       node_weight=self.node_weight, edge_weight=self.edge_weight)
        torch.cuda.synchronize()
        out = {"X": X[: self.graph.n].cpu().numpy(), "value": value.cpu().numpy().reshape(G, S),
               "violations": viol.cpu().numpy().reshape(G, S), "pair_hamming": ph.cpu().numpy()}
        if wv is not None:
            out["wvalue"] = wv.cpu().numpy().reshape(G, S)
        return out

    def diversity(self, X: Optional[torch.Tensor] = None, graph_index: int = 0) -> Dict[str, object]:
        """Pairwise Hamming distances, their histogram, the distinct-solution count and
        DScore of the rounded solutions of one graph (all of them for a single graph)."""
        if X is None:
            X = torch.empty((max(self.graph.n, 1), self.cfg.S), dtype=torch.uint8, device=self.device)
            api.round_eval(self.graph, self.problem_id, self.Z, X)
        if self.graph.n_graphs > 1:
            gp = self.graph.graph_ptr.cpu().numpy()
            X = X[int(gp[graph_index]):int(gp[graph_index + 1])]
        N, S = X.shape
        D = torch.empty((S, S), dtype=torch.int32, device=self.device)
        hist = torch.empty(N + 1, dtype=torch.int64, device=self.device)
        nu = torch.empty(1, dtype=torch.int32, device=self.device)
        api.pairwise_hamming(X.contiguous(), D, hist, nu)
        torch.cuda.synchronize()
        h = hist.cpu().numpy()
        total = int(h.dot(np.arange(N + 1)))
        return {"D": D.cpu().numpy(), "hist": h, "unique": int(nu.item()),
                "dscore": 2.0 * total / (N * S * (S - 1)) if S > 1 and N else 0.0}

    def terms_host(self) -> np.ndarray:
        torch.cuda.synchronize()
        return self.terms.cpu().numpy()

    def close(self) -> None:
        if self._graph is not None:
            api.graph_destroy(self._graph)
            self._graph = None
        if self._graph_k is not None:
            api.graph_destroy(self._graph_k[0])
            self._graph_k = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SolveResult:
    """What `solve` returns: the rounded heads of the last step and their scores.
    X [N, S] uint8; value and violations [G, S] int64 (set size or cut per graph and
    head); wvalue [G, S] float64 with node or edge weights (else None); best_head [G]
    the best feasible head of each graph (-1: none feasible) and best_value [G] its
    score (weighted score where there are weights); steps run, the step at which early
    stopping fired (or None) and the wall time of the training loop in seconds."""
    X: np.ndarray
    value: np.ndarray
    violations: np.ndarray
    wvalue: Optional[np.ndarray]
    best_head: np.ndarray
    best_value: np.ndarray
    steps: int
    stop_step: Optional[int]
    seconds: float


def solve(graph, cfg: CPRAConfig, lam=None, params: Optional[Dict[str, object]] = None,
          seed: int = 0, early_stopping: Optional[Dict[str, object]] = None, device="cuda",
          **solver_kw) -> SolveResult:
    """Train CPRA on `graph` (a CSRGraph or a DeviceGraph) for cfg.T steps -- one step
    captured and replayed (Sec. 3.1 loop) -- then round every head at P > 0.5 and score it.
    lam: the MIS penalties [S] (default logspace(-1, 1, S)); params: initial parameters
    (default: seeded `workloads.init_params`, or `init_params_per_graph` with
    per-graph weights); early_stopping: keyword arguments of
    `CPRASolver.enable_early_stopping` (tol, patience, relative), or None to train all
    T steps; solver_kw: z_offset, node_weight, edge_weight of CPRASolver."""
    import time

    dg = graph if isinstance(graph, DeviceGraph) else DeviceGraph.from_csr(graph, device=device)
    if lam is None and cfg.problem == "mis":
        lam = np.logspace(-1.0, 1.0, cfg.S).astype(np.float32)
    sol = CPRASolver(dg, cfg, lam=lam, device=device, **solver_kw)
    try:
        if params is None:
            from workloads import init_params, init_params_per_graph
            if cfg.per_graph_weights:
                params = init_params_per_graph(cfg.layer_kind, dg.n, cfg.n_layers, cfg.hidden,
                                               cfg.S, dg.n_graphs, seed=seed, in_dim=cfg.in_dim)
            else:
                params = init_params(cfg.layer_kind, dg.n, cfg.n_layers, cfg.hidden, cfg.S,
                                     seed=seed, in_dim=cfg.in_dim)
        sol.load_params(params)
        stop_step = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if early_stopping is not None:
            sol.enable_early_stopping(**early_stopping)
            steps, stop_step = sol.run_with_early_stopping(cfg.T)
        else:
            sol.run(cfg.T)
            steps = cfg.T
        sol.forward()  # the logits of the trained parameters
        ev = sol.evaluate()
        seconds = time.perf_counter() - t0
    finally:
        sol.close()
    score = ev.get("wvalue", ev["value"]).astype(np.float64)
    feasible = ev["violations"] == 0
    masked = np.where(feasible, score, -np.inf)
    best_head = np.where(feasible.any(axis=1), masked.argmax(axis=1), -1)
    best_value = np.where(best_head >= 0, masked.max(axis=1), 0.0)
    return SolveResult(X=ev["X"], value=ev["value"], violations=ev["violations"],
                       wvalue=ev.get("wvalue"), best_head=best_head, best_value=best_value,
                       steps=int(steps), stop_step=stop_step, seconds=seconds)
