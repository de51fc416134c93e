"""Training data, training and evaluation of the learned warm start.

    python -m paper_2402_02190_amd.warmstart_train train --out DIR [options]
    python -m paper_2402_02190_amd.warmstart_train eval --weights FILE [options]

train:
  1. draws random d-regular training graphs (d in {3, 5, 10}, N uniform in
     [1000, 20000], seeded);
  2. solves them with CPRA itself -- batched over block-diagonal unions of
     about ``--batch-nodes`` nodes (one shared GCN encoder per union, per-node
     embeddings, the cpra_train_step path replayed from a HIP graph) -- and
     rounds the converged logits to X* [N, S];
  3. trains the BF16 message-passing network with cpra_mpnn_train_step on
     (features, X*) of every union: the CPRA loss of sigmoid(Z_w) at a fixed
     gamma plus beta * BCE(sigmoid(Z_w), X*);
  4. saves the weights (npz) and a JSON summary.
eval: time-to-target on unseen N = 50,000 random d-regular graphs, several
  seeds: the plain (cold-start) CPRA run and the warm-started run
  (P = sigmoid(GNN + scale * Z_w)) with the same kernels, decoding every K
  steps; the target is the cold run's final best feasible MIS size and each
  arm's time is the wall time until its best feasible head first reaches it
  (warm-start inference -- features and network forward -- included).
Every step of both arms runs in libcpra's kernels; this module only drives
them and keeps host-side bookkeeping.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import api
from .solver import CPRAConfig, CPRASolver
from .warmstart import WarmStartNet


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- data
def training_specs(n_graphs: int, seed: int, n_min: int = 1000, n_max: int = 20000,
                   degrees: Sequence[int] = (3, 5, 10)):
    """[(n, d, graph_seed)] with n * d even."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_graphs):
        d = int(rng.choice(degrees))
        n = int(rng.integers(n_min, n_max + 1))
        if (n * d) % 2:
            n = n + 1 if n < n_max else n - 1
        out.append((n, d, int(seed) * 1_000_003 + k))
    return out


def group_specs(specs, max_nodes: int):
    groups, cur, tot = [], [], 0
    for s in specs:
        if cur and tot + s[0] > max_nodes:
            groups.append(cur)
            cur, tot = [], 0
        cur.append(s)
        tot += s[0]
    if cur:
        groups.append(cur)
    return groups


def build_union(group):
    from workloads import disjoint_union, random_regular_graph
    return disjoint_union([random_regular_graph(n, d, s) for n, d, s in group])


def mis_lambda(S: int) -> np.ndarray:
    return np.logspace(-1, 1, S).astype(np.float32)


def cpra_config(S: int, T: int, hidden: int = 64, n_layers: int = 2,
                gamma_start: float = -2.0, gamma_end: float = 0.1) -> CPRAConfig:
    return CPRAConfig(problem="mis", layer_kind="gcn", n_layers=n_layers, hidden=hidden, S=S,
                      gamma_start=gamma_start, gamma_end=gamma_end, T=T)


def converged_solutions(dg, S: int, T: int, seed: int, chunk: int = 250):
    """Run CPRA for T steps on a (batched) device graph; return X* uint8 [N, S]
    (device) and the per-graph best feasible MIS size."""
    from workloads import init_params
    cfg = cpra_config(S, T)
    sol = CPRASolver(dg, cfg, mis_lambda(S))
    sol.load_params(init_params("gcn", dg.n, cfg.n_layers, cfg.hidden, S, seed=seed))
    done = 0
    while done < T:
        n = min(chunk, T - done)
        sol.replay(n)
        done += n
    sol.forward()
    X = torch.empty((dg.n, S), dtype=torch.uint8, device="cuda")
    G = dg.n_graphs
    value = torch.empty(G * S, dtype=torch.int64, device="cuda")
    viol = torch.empty(G * S, dtype=torch.int64, device="cuda")
    api.round_eval(dg, api.MIS, sol.Z, X, value, viol)
    torch.cuda.synchronize()
    v = value.cpu().numpy().reshape(G, S)
    f = viol.cpu().numpy().reshape(G, S) == 0
    best = np.where(f, v, -1).max(axis=1)
    sol.close()
    return X, best


# ---------------------------------------------------------------- training
def generate_data(n_graphs: int = 2000, seed: int = 1, batch_nodes: int = 2_000_000,
                  T_runs: int = 2000, S: int = 32, in_dim: int = 16, n_rand: int = 14,
                  n_min: int = 1000, n_max: int = 20000):
    """Training unions [(device graph, bf16 features, X* uint8 [N, S])] and the
    converged runs' best feasible densities."""
    specs = training_specs(n_graphs, seed, n_min, n_max)
    groups = group_specs(specs, batch_nodes)
    log(f"[warm] {n_graphs} training graphs, {sum(s[0] for s in specs)} nodes, {len(groups)} unions")
    from workloads import random_channels
    featurizer = WarmStartNet(1, in_dim, 32, S, n_rand)  # features only
    data, run_best = [], []
    for b, grp in enumerate(groups):
        t0 = time.time()
        g = build_union(grp)
        dg = api.DeviceGraph.from_csr(g)
        X, best = converged_solutions(dg, S, T_runs, seed=seed * 7919 + b)
        feat = featurizer.features(dg, random_channels(g.n, n_rand, seed=seed * 104729 + b))
        data.append((dg, feat, X))
        nodes = np.array([s_[0] for s_ in grp])
        run_best.extend((best / nodes).tolist())
        log(f"[warm] union {b + 1}/{len(groups)}: {len(grp)} graphs, {g.n} nodes, CPRA {T_runs} steps "
            f"in {time.time() - t0:.1f}s, mean best feasible density {np.mean(best / nodes):.4f}")
    return data, run_best


def train_net(net: WarmStartNet, data, steps: int = 2000, lr: float = 3e-3, beta: float = 1.0,
              gamma: float = 0.1, log_every: int = 250):
    """Adam on the network, one union per step (cycling); returns the history."""
    S = net.S
    lam = torch.from_numpy(mis_lambda(S)).cuda()
    lc = api.make_loss_cfg(api.MIS, S, lam, 2, gamma, 0.0, 0, None, gamma, gamma, 2)
    adam = api.AdamCfg(lr, 0.9, 0.999, 1e-8, 0.0)
    cfg = api.make_mpnn_step_cfg(net.cfg, lc, adam, beta)
    ws = torch.empty(max(api.mpnn_train_step_workspace_bytes(d[0], cfg) for d in data),
                     dtype=torch.uint8, device="cuda")
    Zw = torch.empty((max(d[0].n for d in data), S), dtype=torch.float32, device="cuda")
    dZw = torch.empty_like(Zw)
    terms = torch.zeros((max(d[0].n_graphs for d in data), S + 2), dtype=torch.float64,
                        device="cuda")
    history = []
    t0 = time.time()
    for t in range(1, steps + 1):
        dg, feat, X = data[(t - 1) % len(data)]
        want = t % log_every == 0 or t == steps
        api.mpnn_train_step(dg, cfg, net.params, net.grads, net.m, net.v, feat, X, Zw, dZw,
                            terms if want else None, ws, t=t)
        if want:
            torch.cuda.synchronize()
            head = terms[: dg.n_graphs, :S].sum().item() / dg.n
            history.append({"step": t, "cpra_head_loss_per_node": float(head)})
            log(f"[warm] train step {t}/{steps}: CPRA head loss per node {head:.4f} "
                f"({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    return history


def train(out_dir: str, n_graphs: int = 2000, seed: int = 1, batch_nodes: int = 2_000_000,
          T_runs: int = 2000, S: int = 32, n_layers: int = 3, in_dim: int = 16, hidden: int = 64,
          n_rand: int = 14, steps: int = 2000, lr: float = 3e-3, beta: float = 1.0,
          gamma: float = 0.1, n_min: int = 1000, n_max: int = 20000) -> Dict[str, object]:
    os.makedirs(out_dir, exist_ok=True)
    t_start = time.time()
    data, run_best = generate_data(n_graphs, seed, batch_nodes, T_runs, S, in_dim, n_rand, n_min,
                                   n_max)
    from workloads import init_mpnn_params
    net = WarmStartNet(n_layers, in_dim, hidden, S, n_rand)
    net.load_params(init_mpnn_params(in_dim, hidden, S, n_layers, seed=seed + 17))
    history = train_net(net, data, steps, lr, beta, gamma)
    path = os.path.join(out_dir, "warmstart_net.npz")
    net.save(path)
    summary = {"n_graphs": n_graphs, "unions": len(data), "T_runs": T_runs, "S": S,
               "converged_best_density_mean": float(np.mean(run_best)),
               "train_steps": steps, "lr": lr, "beta": beta, "gamma": gamma,
               "history": history, "seconds": time.time() - t_start, "weights": path}
    with open(os.path.join(out_dir, "train_summary.json"), "w") as f:
        json.dump(summary, f, indent=1)
    return summary


# ---------------------------------------------------------------- evaluation
class Arm:
    """One CPRA run with periodic decoding (best feasible MIS size so far)."""

    def __init__(self, dg, S: int, T: int, seed: int, z_offset: Optional[torch.Tensor] = None,
                 gamma_start: float = -2.0, gamma_end: float = 0.1, decay_steps: int = 0):
        """decay_steps > 0: the offset fades linearly to 0 over that many steps (it is
        rescaled between decoding intervals, i.e. every K steps)."""
        from workloads import init_params
        self.cfg = cpra_config(S, T, gamma_start=gamma_start, gamma_end=gamma_end)
        self.z0 = None if z_offset is None or decay_steps <= 0 else z_offset.clone()
        self.z_offset = z_offset
        self.decay_steps = decay_steps
        self.sol = CPRASolver(dg, self.cfg, mis_lambda(S), z_offset=z_offset)
        p = init_params("gcn", dg.n, self.cfg.n_layers, self.cfg.hidden, S, seed=seed)
        # GEMM plans for this graph's shapes: tuned once per shape (a real step, then
        # the parameters and the step counter are reset), outside every clock
        self.sol.load_params(p)
        self.sol.autotune()
        self.sol.load_params(p)
        self.value = torch.empty(dg.n_graphs * S, dtype=torch.int64, device="cuda")
        self.viol = torch.empty(dg.n_graphs * S, dtype=torch.int64, device="cuda")
        self.ws = torch.empty(max(api.round_eval_workspace_bytes(dg, S), 256), dtype=torch.uint8,
                              device="cuda")
        self.dg = dg

    def best(self):
        """Best feasible MIS size over the heads: an int for one graph, an int64
        array [n_graphs] for a block-diagonal batch (-1 where no head is feasible)."""
        api.round_eval(self.dg, api.MIS, self.sol.Z, None, self.value, self.viol, ws=self.ws)
        G = self.dg.n_graphs
        v = self.value.cpu().numpy().reshape(G, -1)
        f = self.viol.cpu().numpy().reshape(G, -1) == 0
        b = np.where(f, v, -1).max(axis=1)
        return int(b[0]) if G == 1 else b

    def run(self, T: int, K: int, t0: float):
        """[(seconds since t0, steps, best so far)], decoding every K steps; the
        logits decoded after step k are those of step k's forward."""
        self.sol.capture()
        self.sol.forward()
        best = self.best()
        trace = [(time.perf_counter() - t0, 0, best)]
        done = 0
        while done < T:
            n = min(K, T - done)
            if self.z0 is not None:
                f = max(0.0, 1.0 - done / self.decay_steps)
                torch.mul(self.z0, f, out=self.z_offset)
            self.sol.replay(n)
            done += n
            b = self.best()
            best = np.maximum(best, b) if isinstance(b, np.ndarray) else max(best, b)
            trace.append((time.perf_counter() - t0, done, best))
        return trace


def first_time(trace, target):
    for sec, step, best in trace:
        if best >= target:
            return sec, step
    return None, None


def _warm_logits(net, dg, rand, scale):
    feat = net.features(dg, rand)
    Zw = net.forward(dg, feat)
    if scale != 1.0:
        Zw.mul_(scale)
    return Zw


def evaluate(weights: str, n: int = 50_000, degrees: Sequence[int] = (3, 5, 10),
             seeds: Sequence[int] = (0, 1, 2, 3, 4), T: int = 3000, K: int = 50,
             scale: float = 1.0, warm_gamma_start: float = -2.0, warm_T: Optional[int] = None,
             control: bool = True, out: Optional[str] = None, decay_steps: int = 0,
             fractions: Sequence[float] = (0.9, 0.95, 0.98, 0.99, 1.0), extra_steps: int = 0):
    """Arms per graph: cold (plain CPRA, gamma -2 -> 0.1 over T steps); warm
    (z_offset = scale * Z_w, gamma warm_gamma_start -> 0.1 over warm_T steps, then
    extra_steps more at gamma 0.1); control (the warm arm's schedule without the
    network).  Target = the cold arm's final best feasible MIS size."""
    from workloads import random_channels, random_regular_graph
    net = WarmStartNet.load(weights) if isinstance(weights, str) else weights
    S = net.S
    warm_T = T if warm_T is None else warm_T
    rows = []
    for d in degrees:
        for sd in seeds:
            g = random_regular_graph(n, d, seed=900_000 + 1000 * d + sd)
            dg = api.DeviceGraph.from_csr(g)
            rand = random_channels(n, net.n_rand, seed=77_000 + 1000 * d + sd)
            torch.cuda.synchronize()
            cold = Arm(dg, S, T, seed=sd)
            torch.cuda.synchronize()
            trace_c = cold.run(T, K, time.perf_counter())
            cold.sol.close()
            target = trace_c[-1][2]
            # warm arm: inference (features + network forward) is inside the clock
            torch.cuda.synchronize()
            tw = time.perf_counter()
            Zw = _warm_logits(net, dg, rand, scale)
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - tw
            warm = Arm(dg, S, warm_T, seed=sd, z_offset=Zw, gamma_start=warm_gamma_start,
                       decay_steps=decay_steps)
            torch.cuda.synchronize()
            trace_w = [(s_ + t_inf, k, b) for s_, k, b in warm.run(warm_T + extra_steps, K,
                                                                    time.perf_counter())]
            warm.sol.close()
            row = {"d": d, "seed": sd, "n": n, "target": target, "warm_inference_s": t_inf,
                   "warm_best_at_0": trace_w[0][2], "warm_final": trace_w[-1][2]}
            for name, tr in (("cold", trace_c), ("warm", trace_w)):
                t_s, t_k = first_time(tr, target)
                row[f"{name}_time_s"], row[f"{name}_steps"] = t_s, t_k
            trace_x = None
            if control:
                ctl = Arm(dg, S, warm_T, seed=sd, gamma_start=warm_gamma_start)
                torch.cuda.synchronize()
                trace_x = ctl.run(warm_T + extra_steps, K, time.perf_counter())
                ctl.sol.close()
                row["control_time_s"], row["control_steps"] = first_time(trace_x, target)
                row["control_final"] = trace_x[-1][2]
            # time to reach each fraction of the target, per arm
            row["curves"] = {}
            for name, tr in (("cold", trace_c), ("warm", trace_w), ("control", trace_x)):
                if tr is None:
                    continue
                row["curves"][name] = {f"{f:g}": first_time(tr, int(np.ceil(f * target)))[0]
                                       for f in fractions}
            row["speedup"] = (row["cold_time_s"] / row["warm_time_s"]) if row["warm_time_s"] else None
            rows.append(row)
            log(f"[warm-eval] d={d} seed={sd}: target {target} (cold: step {row['cold_steps']}, "
                f"{row['cold_time_s']:.3f}s) | warm: alone {row['warm_best_at_0']}, target at step "
                f"{row['warm_steps']}, final {row['warm_final']} | control: target at step "
                f"{row.get('control_steps')}, final {row.get('control_final')}")
    reached = [r for r in rows if r["warm_time_s"] is not None]

    def med(key, rs):
        v = [r[key] for r in rs if r.get(key) is not None]
        return float(np.median(v)) if v else None

    curves = {}
    for arm in ("cold", "warm", "control"):
        for f in fractions:
            key = f"{f:g}"
            ts = [r["curves"][arm][key] for r in rows if arm in r["curves"]]
            if ts:
                curves.setdefault(arm, {})[key] = {
                    "reached": sum(t is not None for t in ts), "of": len(ts),
                    "median_s": float(np.median([t for t in ts if t is not None]))
                    if any(t is not None for t in ts) else None}
    summ = {"n": n, "degrees": list(degrees), "seeds": list(seeds), "T": T, "K": K, "scale": scale,
            "warm_gamma_start": warm_gamma_start, "warm_T": warm_T, "decay_steps": decay_steps,
            "extra_steps": extra_steps,
            "curves": curves, "rows": rows,
            "warm_reached": len(reached), "total": len(rows),
            "control_reached": sum(1 for r in rows if r.get("control_time_s") is not None),
            "median_speedup": med("speedup", reached),
            "median_cold_time_s": med("cold_time_s", rows),
            "median_warm_time_s": med("warm_time_s", reached),
            "mean_warm_final_over_target": float(np.mean([r["warm_final"] / r["target"] for r in rows])),
            "mean_control_final_over_target": (float(np.mean([r["control_final"] / r["target"]
                                                              for r in rows])) if control else None),
            "mean_warm_alone_over_target": float(np.mean([r["warm_best_at_0"] / r["target"] for r in rows]))}
    if out:
        with open(out, "w") as f:
            json.dump(summ, f, indent=1)
    return summ


def evaluate_batched(weights, n: int = 50_000, degrees: Sequence[int] = (3, 5, 10),
                     seeds: Sequence[int] = (0, 1, 2, 3, 4), T: int = 3000, K: int = 50,
                     warm_gamma_start: float = -0.5, warm_T: int = 1000, decay_steps: int = 500,
                     out: Optional[str] = None):
    """Solving a set of unseen graphs: the plain method graph by graph (each run's
    final best feasible MIS size is that graph's target; the set's time is the
    sum of the runs' times to reach their targets) against one batched CPRA run
    over the block-diagonal union of all graphs -- plain schedule, and warm
    started (inference on the union inside the clock).  A batched arm's time
    is when its last graph reaches its target."""
    from workloads import disjoint_union, random_channels, random_regular_graph
    net = WarmStartNet.load(weights) if isinstance(weights, str) else weights
    S = net.S
    graphs, rands = [], []
    for d in degrees:
        for sd in seeds:
            graphs.append(random_regular_graph(n, d, seed=900_000 + 1000 * d + sd))
            rands.append(random_channels(n, net.n_rand, seed=77_000 + 1000 * d + sd))
    targets, t_seq = [], 0.0
    for i, g in enumerate(graphs):
        dg = api.DeviceGraph.from_csr(g)
        cold = Arm(dg, S, T, seed=i)
        torch.cuda.synchronize()
        tr = cold.run(T, K, time.perf_counter())
        cold.sol.close()
        targets.append(tr[-1][2])
        t_seq += first_time(tr, tr[-1][2])[0]
        log(f"[batched] plain run {i + 1}/{len(graphs)}: target {tr[-1][2]}")
    targets = np.array(targets)
    u = disjoint_union(graphs)
    du = api.DeviceGraph.from_csr(u)
    res = {"graphs": len(graphs), "n": n, "targets": targets.tolist(),
           "plain_sequential_s": t_seq}

    def reach(trace):
        """(seconds when every graph reached its target or None, fraction of graphs
        reaching it by the end, final best / target per graph)."""
        t_all = None
        for sec, step, b in trace:
            if np.all(np.asarray(b) >= targets):
                t_all = sec
                break
        fin = np.asarray(trace[-1][2], dtype=np.float64) / targets
        return t_all, float(np.mean(fin >= 1.0)), fin

    torch.cuda.synchronize()
    bc = Arm(du, S, T, seed=12345)
    torch.cuda.synchronize()
    tr_c = bc.run(T, K, time.perf_counter())
    bc.sol.close()
    t, frac, fin = reach(tr_c)
    res["batched_plain"] = {"T": T, "time_all_s": t, "wall_s": tr_c[-1][0],
                            "fraction_reached": frac, "mean_final_over_target": float(fin.mean())}
    log(f"[batched] plain schedule on the union: {res['batched_plain']}")
    torch.cuda.synchronize()
    tw = time.perf_counter()
    r_all = np.concatenate(rands, axis=0)
    Zw = _warm_logits(net, du, r_all, 1.0)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - tw
    bw = Arm(du, S, warm_T, seed=12345, z_offset=Zw, gamma_start=warm_gamma_start,
             decay_steps=decay_steps)
    torch.cuda.synchronize()
    tr_w = [(s_ + t_inf, k, b) for s_, k, b in bw.run(warm_T, K, time.perf_counter())]
    bw.sol.close()
    t, frac, fin = reach(tr_w)
    res["batched_warm"] = {"T": warm_T, "gamma_start": warm_gamma_start, "decay_steps": decay_steps,
                           "inference_s": t_inf, "time_all_s": t, "wall_s": tr_w[-1][0],
                           "fraction_reached": frac, "mean_final_over_target": float(fin.mean())}
    log(f"[batched] warm start on the union: {res['batched_warm']}")
    if out:
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned warm start: train / evaluate")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("train")
    a.add_argument("--out", required=True)
    a.add_argument("--graphs", type=int, default=2000)
    a.add_argument("--seed", type=int, default=1)
    a.add_argument("--batch-nodes", type=int, default=2_000_000)
    a.add_argument("--runs-T", type=int, default=2000)
    a.add_argument("--steps", type=int, default=1500)
    a.add_argument("--lr", type=float, default=3e-3)
    a.add_argument("--beta", type=float, default=1.0)
    a.add_argument("--gamma", type=float, default=0.1)
    a.add_argument("--n-max", type=int, default=20000)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--n", type=int, default=50_000)
    e.add_argument("--degrees", type=int, nargs="+", default=[3, 5, 10])
    e.add_argument("--seeds", type=int, nargs="+", default=[0, 1, 2, 3, 4])
    e.add_argument("--T", type=int, default=3000)
    e.add_argument("--K", type=int, default=50)
    e.add_argument("--scale", type=float, default=1.0)
    e.add_argument("--warm-gamma-start", type=float, default=-2.0)
    e.add_argument("--warm-T", type=int, default=None)
    e.add_argument("--no-control", action="store_true")
    e.add_argument("--decay-steps", type=int, default=0)
    e.add_argument("--out", default=None)
    b = sub.add_parser("eval-batched")
    b.add_argument("--weights", required=True)
    b.add_argument("--n", type=int, default=50_000)
    b.add_argument("--degrees", type=int, nargs="+", default=[3, 5, 10])
    b.add_argument("--seeds", type=int, nargs="+", default=[0, 1, 2, 3, 4])
    b.add_argument("--T", type=int, default=3000)
    b.add_argument("--warm-T", type=int, default=1000)
    b.add_argument("--warm-gamma-start", type=float, default=-0.5)
    b.add_argument("--decay-steps", type=int, default=500)
    b.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "eval-batched":
        s = evaluate_batched(args.weights, args.n, args.degrees, args.seeds, args.T, 50,
                             args.warm_gamma_start, args.warm_T, args.decay_steps, args.out)
        print(json.dumps({k: v for k, v in s.items() if k != "targets"}))
        return
    if args.cmd == "train":
        s = train(args.out, args.graphs, args.seed, args.batch_nodes, args.runs_T, steps=args.steps,
                  lr=args.lr, beta=args.beta, gamma=args.gamma, n_max=args.n_max)
        print(json.dumps({k: v for k, v in s.items() if k != "history"}))
    else:
        s = evaluate(args.weights, args.n, args.degrees, args.seeds, args.T, args.K, args.scale,
                     args.warm_gamma_start, args.warm_T, not args.no_control, args.out,
                     args.decay_steps)
        print(json.dumps({k: v for k, v in s.items() if k != "rows"}))


if __name__ == "__main__":
    main()
