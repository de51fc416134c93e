"""Kernel-level parity of the HIP path against the FP64 oracle, through the C ABI.

Covers graph preparation, mean aggregation (forward and transposed, with the
epilogue options), the MFMA GEMM in all operand layouts (ragged tiles,
split-K), the fused relaxed loss (both problems, several S, alpha, nu, ddof,
weights, saturated logits, block-diagonal batches), Adam and the integer
rounding/evaluation.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from helpers import (N_GEMM_CFGS, assert_close_array, assert_close_scalar, assert_update_close, need_gpu,
                     rel_err, say, to_dev)
from oracle import evaluate as oev
from oracle import gnn as ognn
from oracle import objective as oobj
from oracle import train as otrain
from workloads import (csr_from_edges, disjoint_union, erdos_renyi_graph, random_regular_graph)
from workloads.params import random_logits

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def api():
    from paper_2402_02190_amd import api as a
    return a


def weighted_er(n, p, seed):
    g = erdos_renyi_graph(n, p, seed)
    u, v, _ = g.edge_list()
    w = np.random.default_rng(seed).uniform(0.25, 3.0, size=u.size).astype(np.float32)
    return csr_from_edges(n, u, v, w)


def batch_graph(seed, sizes=(37, 1, 250, 90, 3, 600)):
    rng = np.random.default_rng(seed)
    gs = [erdos_renyi_graph(n, min(1.0, rng.uniform(2, 8) / max(n - 1, 1)), seed + i)
          for i, n in enumerate(sizes)]
    return disjoint_union(gs)


GRAPHS = {
    "rrg3_100": lambda: random_regular_graph(100, 3, 1),
    "er_sparse_300": lambda: erdos_renyi_graph(300, 1.5 / 299, 2),  # isolated nodes
    "rrg20_500": lambda: random_regular_graph(500, 20, 3),
    "weighted_er_400": lambda: weighted_er(400, 0.02, 4),
    "batch": lambda: batch_graph(5),
}


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("gname", list(GRAPHS))
def test_csr_prepare(gname):
    a = api()
    g = GRAPHS[gname]()
    say(f"csr_prepare {gname} n={g.n} nnz={g.nnz}")
    dg = a.DeviceGraph.from_csr(g)
    torch.cuda.synchronize()
    deg = np.diff(g.row_ptr).astype(np.float32)
    inv = np.where(deg > 0, np.float32(1) / np.maximum(deg, 1), 0).astype(np.float32)
    assert np.array_equal(dg.inv_deg.cpu().numpy()[: g.n], inv)
    if g.weight is None:
        assert np.array_equal(dg.wdeg.cpu().numpy()[: g.n], deg)
    else:
        ref = np.add.reduceat(g.weight.astype(np.float64), g.row_ptr[:-1]) if g.nnz else 0
        ref = np.where(deg > 0, ref, 0.0)
        assert rel_err(dg.wdeg.cpu().numpy()[: g.n], ref) < 1e-6


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("width", [1, 3, 10, 32, 100, 256, 520])
@pytest.mark.parametrize("transpose", [False, True])
def test_aggregate_mean(gname, width, transpose):
    a = api()
    g = GRAPHS[gname]()
    say(f"aggregate {gname} width={width} transpose={transpose}")
    dg = a.DeviceGraph.from_csr(g)
    rng = np.random.default_rng(width)
    X = rng.standard_normal((g.n, width)).astype(np.float32)
    M = ognn.mean_aggregation_matrix(g.row_ptr, g.col_idx)
    ref = (M.T if transpose else M) @ X.astype(np.float64)
    Y = torch.empty((g.n, width), dtype=torch.float32, device="cuda")
    a.aggregate_mean(dg, to_dev(X), Y, transpose=transpose)
    torch.cuda.synchronize()
    assert_close_array(Y.cpu().numpy(), ref, 1e-6, "MX")
    # epilogue: add + bias, relu, mask (strided views)
    add = rng.standard_normal((g.n, width + 3)).astype(np.float32)
    bias = rng.standard_normal(width).astype(np.float32)
    mask = (rng.random((g.n, width)) < 0.5).astype(np.float32)
    add_d = to_dev(add)[:, :width]
    Y2 = torch.empty((g.n, width), dtype=torch.float32, device="cuda")
    a.aggregate_mean(dg, to_dev(X), Y2, transpose=transpose, add=add_d, bias=to_dev(bias),
                     relu=True, mask=to_dev(mask))
    torch.cuda.synchronize()
    ref2 = np.maximum(ref + add[:, :width] + bias, 0) * (mask > 0)
    assert_close_array(Y2.cpu().numpy(), ref2, 1e-6, "epilogue")


# ---------------------------------------------------------------------------
GEMM_SHAPES = [(1, 1, 1), (37, 19, 5), (100, 10, 32), (1037, 100, 256), (10000, 256, 512),
               (777, 130, 77), (200, 256, 10000), (64, 64, 64), (129, 65, 33)]


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("shape", GEMM_SHAPES)
def test_gemm(ta, tb, shape):
    a = api()
    M, N, K = shape
    say(f"gemm ta={ta} tb={tb} M={M} N={N} K={K}")
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    bias = rng.standard_normal(N).astype(np.float32)
    opA = A.T if ta else A
    opB = B.T if tb else B
    ref = opA.astype(np.float64) @ opB.astype(np.float64)
    Cd = torch.zeros((M, N), dtype=torch.float32, device="cuda")
    a.gemm(to_dev(A), to_dev(B), Cd, ta, tb)
    torch.cuda.synchronize()
    assert_close_array(Cd.cpu().numpy(), ref, 2e-6, "C")
    Cd = to_dev(C0)
    a.gemm(to_dev(A), to_dev(B), Cd, ta, tb, beta=0.5, bias=to_dev(bias), relu=True)
    torch.cuda.synchronize()
    assert_close_array(Cd.cpu().numpy(), np.maximum(ref + 0.5 * C0 + bias, 0), 2e-6, "epilogue")


def test_gemm_autotuned_plans_keep_parity():
    a = api()
    rng = np.random.default_rng(3)
    shapes = [(False, True, 3000, 256, 512), (True, False, 256, 256, 5000), (False, False, 999, 100, 200)]
    a.autotune_reset()
    a.autotune_begin()
    try:
        for ta, tb, M, N, K in shapes:
            A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
            B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
            C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
            a.gemm(to_dev(A), to_dev(B), C, ta, tb)
            torch.cuda.synchronize()
            ref = (A.T if ta else A).astype(np.float64) @ (B.T if tb else B).astype(np.float64)
            assert_close_array(C.cpu().numpy(), ref, 2e-6, f"tuning run {ta}{tb}")
    finally:
        table = a.autotune_end()
    assert len(table) == len(shapes)
    for key, choice, us, hus in table:
        say(f"  tuned {key} -> {choice} {us:.1f} us (heuristic {hus:.1f} us)")
        assert us > 0 and (hus < 0 or us <= hus * 1.0001)
    for ta, tb, M, N, K in shapes:  # tuned plans in use, tuning off
        A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
        B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
        C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
        a.gemm(to_dev(A), to_dev(B), C, ta, tb)
        torch.cuda.synchronize()
        ref = (A.T if ta else A).astype(np.float64) @ (B.T if tb else B).astype(np.float64)
        assert_close_array(C.cpu().numpy(), ref, 2e-6, f"tuned plan {ta}{tb}")
    a.autotune_reset()


def test_gemm_strided_and_unaligned_views():
    a = api()
    rng = np.random.default_rng(0)
    big = to_dev(rng.standard_normal((300, 203)).astype(np.float32))
    A = big[:, 1:101]  # unaligned start, ld 203
    Bm = to_dev(rng.standard_normal((100, 70)).astype(np.float32))
    C = torch.zeros((300, 70), dtype=torch.float32, device="cuda")
    a.gemm(A, Bm, C)
    torch.cuda.synchronize()
    ref = A.cpu().double().numpy() @ Bm.cpu().double().numpy()
    assert_close_array(C.cpu().numpy(), ref, 2e-6, "strided")


# ---------------------------------------------------------------------------
def _head_scale(Z, g, problem, lam):
    ei, ej, w = oobj.edges_of(g.row_ptr, g.col_idx, g.weight)
    P, _ = oobj.sigmoid_pair(Z)
    pair = np.sum(np.abs(w)[:, None] * P[ei] * P[ej], axis=0)
    if problem == "mis":
        return P.sum(0) + np.abs(lam) * pair
    return 2 * pair + np.sum(np.abs(w)[:, None] * (P[ei] + P[ej]), axis=0)


LOSS_CASES = [
    # name, graph, S, problem, alpha, nu, ddof, near_binary
    ("c1_like", "rrg3_100", 10, "mis", 2, 0.0, 0, False),
    ("s1_isolated", "er_sparse_300", 1, "mis", 2, 0.0, 0, False),
    ("s100_saturated", "rrg3_100", 100, "mis", 2, 0.0, 0, True),
    ("s130_alpha6_nu", "rrg20_500", 130, "mis", 6, 0.2, 0, False),
    ("maxcut_s32_nu", "er_sparse_300", 32, "maxcut", 2, 0.1, 0, False),
    ("maxcut_w_s64_a4_ddof1", "weighted_er_400", 64, "maxcut", 4, 0.3, 1, False),
    ("batch_maxcut_s32", "batch", 32, "maxcut", 2, 0.1, 0, False),
    ("batch_mis_s7", "batch", 7, "mis", 2, 0.05, 0, False),
    ("s1000", "rrg3_100", 1000, "mis", 2, 0.1, 0, False),
]


@pytest.mark.parametrize("case", LOSS_CASES, ids=[c[0] for c in LOSS_CASES])
def test_loss_fwd_bwd(case):
    a = api()
    name, gname, S, problem, alpha, nu, ddof, nb = case
    g = GRAPHS[gname]()
    say(f"loss {name} n={g.n} S={S}")
    dg = a.DeviceGraph.from_csr(g)
    Z = random_logits(g.n, S, seed=S + alpha, near_binary=nb)
    lam = np.logspace(-1, 1, S).astype(np.float32)
    gamma = -0.8
    pid = a.MIS if problem == "mis" else a.MAXCUT
    lam_d = to_dev(lam) if problem == "mis" else None
    cfg = a.make_loss_cfg(pid, S, lam_d, alpha, gamma, nu, ddof)
    ws = torch.empty(a.loss_workspace_bytes(dg, cfg), dtype=torch.uint8, device="cuda")
    Zd = to_dev(Z)
    dZ = torch.empty_like(Zd)
    terms = torch.empty((dg.n_graphs, S + 2), dtype=torch.float64, device="cuda")
    a.loss_fwd_bwd(dg, cfg, Zd, dZ, terms, ws)
    torch.cuda.synchronize()
    T = terms.cpu().numpy()
    dZh = dZ.cpu().numpy()
    Z64 = Z.astype(np.float64)
    gp = g.graph_ptr
    cfg_o = otrain.StepConfig(problem=problem, lam=lam.astype(np.float64), alpha=alpha, nu=nu,
                              ddof=ddof)
    worst = 0.0
    for gi in range(len(gp) - 1):
        lo, hi = int(gp[gi]), int(gp[gi + 1])
        sub = oobj._slice_graph(g, lo, hi) if len(gp) > 2 else g
        ref = oobj.loss_terms(Z64[lo:hi], sub, problem, cfg_o.lam, gamma, alpha, nu, ddof)
        scale = _head_scale(Z64[lo:hi], sub, problem, cfg_o.lam) if hi > lo else np.zeros(S)
        for s in range(S):
            worst = max(worst, assert_close_scalar(T[gi, s], ref["head"][s], scale[s], what=f"l_{s}"))
        worst = max(worst, assert_close_scalar(T[gi, S], ref["entropy"], abs(ref["entropy"]) + 1e-30,
                                               what="S(P)"))
        worst = max(worst, assert_close_scalar(T[gi, S + 1], ref["psi"], abs(ref["psi"]) + 1e-30,
                                               what="Psi"))
        if hi > lo:
            gref = oobj.grad_wrt_Z(Z64[lo:hi], sub, problem, cfg_o.lam, gamma, alpha, nu, ddof)
            worst = max(worst, assert_close_array(dZh[lo:hi], gref, what=f"dZ graph {gi}"))
    say(f"  worst relative error {worst:.3e}")
    # deterministic: a second call gives identical bits; a precomputed P gives the same result
    dZ2 = torch.empty_like(Zd)
    terms2 = torch.empty_like(terms)
    P = torch.empty_like(Zd)
    a.sigmoid(Zd, P)
    a.loss_fwd_bwd(dg, cfg, Zd, dZ2, terms2, ws, P=P)
    torch.cuda.synchronize()
    assert torch.equal(dZ2, dZ) and torch.equal(terms2, terms)


IDENTICAL_CASES = [("rrg3_100", 7, "mis", 0), ("rrg20_500", 32, "maxcut", 0),
                   ("batch", 100, "mis", 1), ("weighted_er_400", 64, "maxcut", 1)]


@pytest.mark.parametrize("gname,S,problem,ddof", IDENTICAL_CASES)
def test_loss_identical_heads_have_zero_psi_gradient(gname, S, problem, ddof):
    """Nodes whose heads all coincide (a fifth of the rows, non-dyadic values) with
    nu > 0: sigma_i = 0 there, so the diversity term adds nothing to their gradient --
    dZ on those rows equals, bit for bit, the nu = 0 result -- and the rest matches
    the oracle."""
    a = api()
    g = GRAPHS[gname]()
    say(f"identical heads {gname} S={S} {problem} ddof={ddof}")
    dg = a.DeviceGraph.from_csr(g)
    Z = random_logits(g.n, S, seed=S + 17)
    same = np.zeros(g.n, dtype=bool)
    same[::5] = True
    Z[same] = Z[same, :1]  # all heads equal on these rows
    lam = np.logspace(-1, 1, S).astype(np.float32)
    lam_d = to_dev(lam) if problem == "mis" else None
    pid = a.MIS if problem == "mis" else a.MAXCUT
    gamma, nu = -0.6, 0.4
    Zd = to_dev(Z)
    out = {}
    for v in (nu, 0.0):
        cfg = a.make_loss_cfg(pid, S, lam_d, 2, gamma, v, ddof)
        ws = torch.empty(a.loss_workspace_bytes(dg, cfg), dtype=torch.uint8, device="cuda")
        dZ = torch.empty_like(Zd)
        terms = torch.empty((dg.n_graphs, S + 2), dtype=torch.float64, device="cuda")
        a.loss_fwd_bwd(dg, cfg, Zd, dZ, terms, ws)
        torch.cuda.synchronize()
        out[v] = (dZ.cpu().numpy(), terms.cpu().numpy())
    dZn, Tn = out[nu]
    dZ0, _ = out[0.0]
    assert np.array_equal(dZn[same], dZ0[same]), "diversity gradient on rows with identical heads"
    assert not np.array_equal(dZn[~same], dZ0[~same])
    Z64 = Z.astype(np.float64)
    gp = g.graph_ptr
    lam64 = lam.astype(np.float64)
    for gi in range(len(gp) - 1):
        lo, hi = int(gp[gi]), int(gp[gi + 1])
        if hi == lo:
            continue
        sub = oobj._slice_graph(g, lo, hi) if len(gp) > 2 else g
        ref = oobj.loss_terms(Z64[lo:hi], sub, problem, lam64, gamma, 2, nu, ddof)
        assert_close_scalar(Tn[gi, S + 1], ref["psi"], abs(ref["psi"]) + 1e-30, what="Psi")
        gref = oobj.grad_wrt_Z(Z64[lo:hi], sub, problem, lam64, gamma, 2, nu, ddof)
        assert_close_array(dZn[lo:hi], gref, what=f"dZ graph {gi}")


def test_loss_device_schedule_matches_host_gamma():
    a = api()
    g = GRAPHS["rrg3_100"]()
    dg = a.DeviceGraph.from_csr(g)
    S = 16
    Z = to_dev(random_logits(g.n, S, 3))
    lam = to_dev(np.linspace(0.5, 5, S).astype(np.float32))
    counter = torch.tensor([37], dtype=torch.int32, device="cuda")
    from paper_2402_02190_amd.solver import gamma_schedule
    gam = gamma_schedule(37, 100, -2.0, 0.1)
    c_dev = a.make_loss_cfg(a.MIS, S, lam, 2, 0.0, 0.0, 0, counter, -2.0, 0.1, 100)
    c_host = a.make_loss_cfg(a.MIS, S, lam, 2, gam, 0.0, 0)
    ws = torch.empty(a.loss_workspace_bytes(dg, c_dev), dtype=torch.uint8, device="cuda")
    d1, d2 = torch.empty_like(Z), torch.empty_like(Z)
    a.loss_fwd_bwd(dg, c_dev, Z, d1, None, ws)
    a.loss_fwd_bwd(dg, c_host, Z, d2, None, ws)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [7, 100003, 5000003])  # one vector; partial pairs; grid-stride passes
@pytest.mark.parametrize("wd", [0.0, 1e-2])
def test_adam_step(wd, n):
    a = api()
    rng = np.random.default_rng(1)
    p = rng.standard_normal(n).astype(np.float32)
    gr = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = (0.01 * rng.random(n)).astype(np.float32)
    pd, gd, md, vd = to_dev(p), to_dev(gr), to_dev(m), to_dev(v)
    cfg = a.AdamCfg(1e-3, 0.9, 0.999, 1e-8, wd)
    a.adam_step(pd, gd, md, vd, cfg, t=7)
    torch.cuda.synchronize()
    p64, m64, v64 = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    otrain.adam_update(p64, gr.astype(np.float64), m64, v64, 7, 1e-3, weight_decay=wd)
    assert_close_array(md.cpu().numpy(), m64, 1e-6, "m")
    assert_close_array(vd.cpu().numpy(), v64, 1e-6, "v")
    assert_update_close(pd.cpu().numpy(), p, p64, 1e-5, "update")


# ---------------------------------------------------------------------------
EVAL_CASES = [("rrg3_100", 10, "mis"), ("er_sparse_300", 1, "mis"), ("rrg20_500", 130, "mis"),
              ("weighted_er_400", 64, "maxcut"), ("batch", 32, "maxcut"), ("batch", 5, "mis")]


@pytest.mark.parametrize("gname,S,problem", EVAL_CASES)
def test_round_eval_bit_exact(gname, S, problem):
    a = api()
    g = GRAPHS[gname]()
    say(f"round_eval {gname} S={S} {problem}")
    dg = a.DeviceGraph.from_csr(g)
    rng = np.random.default_rng(S)
    Z = (rng.standard_normal((g.n, S)) + rng.uniform(-1, 1, size=(1, S))).astype(np.float32)
    Z[0, 0] = 0.0  # the tie P = 0.5 rounds to 0
    Zd = to_dev(Z)
    G = dg.n_graphs
    X = torch.empty((g.n, S), dtype=torch.uint8, device="cuda")
    val = torch.empty(G * S, dtype=torch.int64, device="cuda")
    vio = torch.empty(G * S, dtype=torch.int64, device="cuda")
    ph = torch.empty(G, dtype=torch.int64, device="cuda")
    wv = torch.empty(G * S, dtype=torch.float64, device="cuda")
    a.round_eval(dg, a.MIS if problem == "mis" else a.MAXCUT, Zd, X, val, vio, wv, ph)
    torch.cuda.synchronize()
    Xo = oev.round_solutions(Z.astype(np.float64))
    assert np.array_equal(X.cpu().numpy(), Xo)
    ev = oev.evaluate(Xo, g, problem)
    val, vio, ph, wv = (t.cpu().numpy() for t in (val, vio, ph, wv))
    for gi, e in enumerate(ev):
        assert ph[gi] == e["pair_hamming"]
        if problem == "mis":
            assert np.array_equal(val[gi * S:(gi + 1) * S], e["size"])
            assert np.array_equal(vio[gi * S:(gi + 1) * S], e["violations"])
            assert np.array_equal(wv[gi * S:(gi + 1) * S], e["weight"])  # unit weights: the size
        else:
            assert np.array_equal(val[gi * S:(gi + 1) * S], e["cut_edges"])
            np.testing.assert_allclose(wv[gi * S:(gi + 1) * S], e["cut"], rtol=1e-12)


def test_round_eval_tiny_and_subnormal_logits():
    """Rounding at P > 1/2 is Z > 0 exactly: tiny positive and subnormal logits round to
    1, zeros of either sign and negative values to 0, as the oracle rounds them."""
    a = api()
    g = GRAPHS["rrg3_100"]()
    dg = a.DeviceGraph.from_csr(g)
    S = 12
    vals = np.array([0.0, -0.0, 1e-45, -1e-45, 1e-40, 1e-38, 1e-20, 1e-17, 1e-16, 2e-16, -1e-16,
                     3.0], dtype=np.float32)
    rng = np.random.default_rng(4)
    Z = vals[rng.integers(0, vals.size, size=(g.n, S))]
    Zd = to_dev(Z)
    X = torch.empty((g.n, S), dtype=torch.uint8, device="cuda")
    val = torch.empty(S, dtype=torch.int64, device="cuda")
    vio = torch.empty(S, dtype=torch.int64, device="cuda")
    a.round_eval(dg, a.MIS, Zd, X, val, vio)
    torch.cuda.synchronize()
    Xo = oev.round_solutions(Z.astype(np.float64))
    assert np.array_equal(X.cpu().numpy(), Xo)
    assert Xo[Z > 0].all() and not Xo[Z <= 0].any()
    e = oev.evaluate_one(Xo, g, "mis")
    assert np.array_equal(val.cpu().numpy(), e["size"])
    assert np.array_equal(vio.cpu().numpy(), e["violations"])




@pytest.mark.parametrize("cfg", range(N_GEMM_CFGS))
def test_gemm_every_tile_config_and_layout_matches_oracle(cfg):
    """Each tile configuration, forced through the tuning table, in every operand
    layout, with and without split-K, on ragged shapes (M, N, K not multiples
    of any tile) with bias and ReLU: one with sizes off every multiple of 4
    (the two-deep prefetch configurations run their one-deep twins there) and
    one with sizes that are multiples of 4 (they run their branch-free loads,
    with a K tail inside the last tile)."""
    a = api()
    rng = np.random.default_rng(cfg)
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    cases = [(M, N, K, ta, tb, splits) for M, N, K in ((333, 130, 77), (332, 132, 76))
             for ta in (False, True) for tb in (False, True) for splits in (1, 3, 40)]
    try:
        for M, N, K, ta, tb, splits in cases:
            key = f"{'T' if ta else 'N'}{'T' if tb else 'N'}|{M}x{N}x{K}"
            a.autotune_reset()
            a.autotune_set(key, cfg, splits)
            A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
            B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
            bias = rng.standard_normal(N).astype(np.float32)
            C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
            a.gemm(to_dev(A), to_dev(B), C, ta, tb, bias=to_dev(bias), relu=True, ws=ws)
            torch.cuda.synchronize()
            ref = (A.T if ta else A).astype(np.float64) @ (B.T if tb else B).astype(np.float64)
            ref = np.maximum(ref + bias, 0.0)
            assert_close_array(C.cpu().numpy(), ref, 2e-6, f"cfg {cfg} {key} splits {splits}")
    finally:
        a.autotune_reset()


@pytest.mark.parametrize("M,ring", [(4_000_000, True), (8_400_000, False)])
def test_gemm_ring_offsets_and_fallback_past_2gib(M, ring):
    """The LDS-ring loop addresses its operands with 32-bit byte offsets: an A of
    1.0 GB runs the ring configuration forced through the table, one of 2.15 GB
    (past 2^31 bytes) its interleaved twin; the profiler names which one ran, and
    sampled rows (the first, the last, and random ones in between) match FP64."""
    a = api()
    N = K = 64
    torch.manual_seed(M)
    A = torch.randn((M, K), dtype=torch.float32, device="cuda")
    B = torch.randn((N, K), dtype=torch.float32, device="cuda")
    C = torch.empty((M, N), dtype=torch.float32, device="cuda")
    try:
        a.autotune_reset()
        a.autotune_set(f"NT|{M}x{N}x{K}", 27, 1)
        a.profile_begin()
        a.gemm(A, B, C, False, True)
        torch.cuda.synchronize()
        prof = a.profile_end()
        fam = "gemm_nt_64x64x16_w2x2_ring" if ring else "gemm_nt_64x64x16_w2x2_il"
        assert fam in prof, sorted(prof)
        rows = np.unique(np.concatenate([[0, 1, M - 2, M - 1],
                                         np.random.default_rng(M).integers(0, M, 2000)]))
        idx = torch.as_tensor(rows, device="cuda")
        As = A[idx].cpu().numpy().astype(np.float64)
        ref = As @ B.cpu().numpy().astype(np.float64).T
        assert_close_array(C[idx].cpu().numpy(), ref, 2e-6, f"M={M} sampled rows")
    finally:
        a.autotune_reset()
        del A, C
        torch.cuda.empty_cache()


@pytest.mark.parametrize("M,cfg,splits", [(32, 27, 1024), (64, 27, 512), (32, 16, 1024), (64, 11, 512)])
def test_gemm_committed_large_split_plans(M, cfg, splits):
    """The split-K plans of the committed 256-graph tuning table at their real shape
    (and the two-deep plans the LDS ring replaced): weight gradients A^T B over
    K = 710,241 rows in 1,024 and 512 splits, summed in a fixed order."""
    a = api()
    N, K = 64, 710241
    rng = np.random.default_rng(M)
    A = rng.standard_normal((K, M)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    key = f"TN|{M}x{N}x{K}"
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    try:
        a.autotune_reset()
        a.autotune_set(key, cfg, splits)
        C = torch.zeros((M, N), dtype=torch.float32, device="cuda")
        a.gemm(to_dev(A), to_dev(B), C, True, False, ws=ws)
        torch.cuda.synchronize()
        ref = A.astype(np.float64).T @ B.astype(np.float64)
        assert_close_array(C.cpu().numpy(), ref, 2e-6, f"{key} cfg {cfg} splits {splits}")
    finally:
        a.autotune_reset()


# ---------------------------------------------------------------------------
# Weighted MIS: node weights per node ([N], ld 0) or per head ([N, S])
@pytest.mark.parametrize("per_head", [False, True])
@pytest.mark.parametrize("gname,S", [("rrg3_100", 10), ("batch", 7), ("rrg20_500", 130)])
def test_weighted_mis_loss_and_eval(gname, S, per_head):
    a = api()
    g = GRAPHS[gname]()
    say(f"weighted MIS {gname} S={S} per_head={per_head}")
    dg = a.DeviceGraph.from_csr(g)
    rng = np.random.default_rng(S)
    W = rng.uniform(0, 1, (g.n, S) if per_head else g.n).astype(np.float32)
    Wd = to_dev(W)
    Z = random_logits(g.n, S, seed=S + 5)
    lam = np.logspace(-1, 1, S).astype(np.float32)
    lam_d = to_dev(lam)
    gamma, nu = -0.4, 0.1
    cfg = a.make_loss_cfg(a.MIS, S, lam_d, 2, gamma, nu, 0, node_weight=Wd)
    ws = torch.empty(a.loss_workspace_bytes(dg, cfg), dtype=torch.uint8, device="cuda")
    Zd = to_dev(Z)
    dZ = torch.empty_like(Zd)
    terms = torch.empty((dg.n_graphs, S + 2), dtype=torch.float64, device="cuda")
    a.loss_fwd_bwd(dg, cfg, Zd, dZ, terms, ws)
    G = dg.n_graphs
    val = torch.empty(G * S, dtype=torch.int64, device="cuda")
    vio = torch.empty(G * S, dtype=torch.int64, device="cuda")
    wv = torch.empty(G * S, dtype=torch.float64, device="cuda")
    a.round_eval(dg, a.MIS, Zd, None, val, vio, wv, node_weight=Wd)
    torch.cuda.synchronize()
    T, dZh, wv = terms.cpu().numpy(), dZ.cpu().numpy(), wv.cpu().numpy()
    Z64, W64 = Z.astype(np.float64), W.astype(np.float64)
    gp = g.graph_ptr
    Xo = oev.round_solutions(Z64)
    for gi in range(len(gp) - 1):
        lo, hi = int(gp[gi]), int(gp[gi + 1])
        sub = oobj._slice_graph(g, lo, hi) if len(gp) > 2 else g
        ref = oobj.loss_terms(Z64[lo:hi], sub, "mis", lam.astype(np.float64), gamma, 2, nu, 0,
                              W64[lo:hi])
        for s in range(S):
            scale = abs(ref["head"][s]) + np.sum(np.abs(oobj.sigmoid_pair(Z64[lo:hi, s])[0])) + 1.0
            assert_close_scalar(T[gi, s], ref["head"][s], scale, what=f"weighted l_{s}")
        gref = oobj.grad_wrt_Z(Z64[lo:hi], sub, "mis", lam.astype(np.float64), gamma, 2, nu, 0,
                               W64[lo:hi])
        assert_close_array(dZh[lo:hi], gref, what=f"weighted dZ graph {gi}")
        ev = oev.evaluate_one(Xo[lo:hi], sub, "mis", W64[lo:hi])
        np.testing.assert_allclose(wv[gi * S:(gi + 1) * S], ev["weight"], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,S", [(1, 1), (63, 5), (64, 33), (1000, 100), (3000, 500), (0, 4)])
def test_pairwise_hamming_bit_exact(N, S):
    a = api()
    rng = np.random.default_rng(N + S)
    X = (rng.random((N, S)) < 0.3).astype(np.uint8)
    if S > 3 and N > 0:
        X[:, 3] = X[:, 1]  # a duplicated solution
    Xd = torch.from_numpy(X).cuda() if N else torch.zeros((0, S), dtype=torch.uint8, device="cuda")
    D = torch.empty((S, S), dtype=torch.int32, device="cuda")
    hist = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    nu = torch.empty(1, dtype=torch.int32, device="cuda")
    a.pairwise_hamming(Xd, D, hist, nu)
    torch.cuda.synchronize()
    ref = oev.diversity_stats(X)
    assert np.array_equal(D.cpu().numpy(), ref["D"])
    assert np.array_equal(hist.cpu().numpy(), ref["hist"])
    assert int(nu.item()) == ref["unique"]
    # without the matrix: histogram and count alone (the workspace holds D)
    hist2 = torch.empty_like(hist)
    nu2 = torch.empty_like(nu)
    a.pairwise_hamming(Xd, None, hist2, nu2)
    torch.cuda.synchronize()
    assert torch.equal(hist2, hist) and torch.equal(nu2, nu)


@pytest.mark.parametrize("gname", ["er_sparse_300", "rrg20_500", "batch"])
@pytest.mark.parametrize("width", [1, 6, 64, 300])
def test_transposed_aggregation_with_per_entry_scale_is_bit_identical(gname, width):
    """cpra_csr_prepare_col gives inv_deg[col_idx[e]] per entry, and the transposed
    aggregation reading it in CSR order equals the one gathering inv_deg per
    neighbour, bit for bit (the same products in the same order)."""
    a = api()
    g = GRAPHS[gname]()
    dg = a.DeviceGraph.from_csr(g)
    inv = dg.inv_deg[: g.n].cpu().numpy()
    col = dg.col_inv_deg[: g.nnz].cpu().numpy()
    assert np.array_equal(col, inv[g.col_idx])
    X = to_dev(np.random.default_rng(width).standard_normal((g.n, width)).astype(np.float32))
    Y1 = torch.empty_like(X)
    Y2 = torch.empty_like(X)
    a.aggregate_mean(dg, X, Y1, transpose=True)
    saved = dg.csr.col_inv_deg
    dg.csr.col_inv_deg = None  # the gathering form
    try:
        a.aggregate_mean(dg, X, Y2, transpose=True)
    finally:
        dg.csr.col_inv_deg = saved
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    ref = A @ (inv[:, None].astype(np.float64) * X.cpu().double().numpy())
    assert_close_array(Y1.cpu().numpy(), ref, 1e-6, "M^T X")
