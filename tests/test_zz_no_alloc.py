"""cpra_loss_fwd_bwd_noalloc (the fused loss with its workspace in the library's
static device scratch) against cpra_loss_fwd_bwd with a caller workspace, through
the C ABI: two calls in a row on the same stream, the second on a smaller input,
must give the same dZ and loss terms bit for bit (the same kernels on the same
inputs; only the workspace's place differs); a workspace larger than the static
array is refused before any launch."""

import numpy as np
import pytest
import torch

from helpers import need_gpu, say, to_dev
from workloads import get_preset, random_regular_graph
from workloads.params import random_logits

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _run_both(a, dg, problem, S, nu, seed, with_p):
    Z = to_dev(random_logits(dg.n, S, seed=seed))
    lam = to_dev(np.logspace(-1, 1, S).astype(np.float32)) if problem == a.MIS else None
    cfg = a.make_loss_cfg(problem, S, lam, 2, -0.7, nu, 0)
    P = None
    if with_p:
        P = torch.empty_like(Z)
        a.sigmoid(Z, P)
    ws = torch.empty(a.loss_workspace_bytes(dg, cfg), dtype=torch.uint8, device="cuda")
    d_ref, d_na = torch.empty_like(Z), torch.empty_like(Z)
    t_ref = torch.empty((dg.n_graphs, S + 2), dtype=torch.float64, device="cuda")
    t_na = torch.empty_like(t_ref)
    a.loss_fwd_bwd(dg, cfg, Z, d_ref, t_ref, ws, P=P)
    a.loss_fwd_bwd_noalloc(dg, cfg, Z, d_na, t_na, P=P)
    torch.cuda.synchronize()
    return d_ref, d_na, t_ref, t_na


def test_noalloc_loss_matches_the_workspace_entry_point_on_two_calls():
    from paper_2402_02190_amd import api as a
    big = get_preset("C2").graph()  # 10,000 nodes, S = 100: P (4 MB) staged in the scratch
    small = random_regular_graph(777, 4, 3)
    cases = [(big, a.MIS, 100, 0.1, 1, False), (small, a.MAXCUT, 32, 0.2, 2, False),
             (big, a.MIS, 64, 0.0, 3, True)]
    for g, problem, S, nu, seed, with_p in cases:
        say(f"noalloc: n={g.n} S={S} problem={problem} nu={nu} P given={with_p}")
        dg = a.DeviceGraph.from_csr(g)
        d_ref, d_na, t_ref, t_na = _run_both(a, dg, problem, S, nu, seed, with_p)
        assert torch.equal(d_ref, d_na), "dZ differs"
        assert torch.equal(t_ref, t_na), "loss terms differ"


def test_noalloc_loss_refuses_more_than_the_static_scratch():
    from paper_2402_02190_amd import _lib
    from paper_2402_02190_amd import api as a
    g = random_regular_graph(70_000, 3, 4)  # P alone: 70,000 x 128 x 4 B = 35.8 MB > 32 MiB
    dg = a.DeviceGraph.from_csr(g)
    S = 128
    cfg = a.make_loss_cfg(a.MAXCUT, S, None, 2, 0.0, 0.0, 0)
    assert a.loss_workspace_bytes(dg, cfg) > _lib.LOSS_NOALLOC_SCRATCH_BYTES
    Z = torch.zeros((g.n, S), dtype=torch.float32, device="cuda")
    dZ = torch.empty_like(Z)
    with pytest.raises(a.CpraError) as e:
        a.loss_fwd_bwd_noalloc(dg, cfg, Z, dZ, None)
    assert "static array" in str(e.value)
    # with P given the P area is not needed, and the call runs
    P = torch.empty_like(Z)
    a.sigmoid(Z, P)
    a.loss_fwd_bwd_noalloc(dg, cfg, Z, dZ, None, P=P)
    torch.cuda.synchronize()
    ref = torch.empty_like(Z)
    ws = torch.empty(a.loss_workspace_bytes(dg, cfg), dtype=torch.uint8, device="cuda")
    a.loss_fwd_bwd(dg, cfg, Z, ref, None, ws, P=P)
    torch.cuda.synchronize()
    assert torch.equal(ref, dZ)
