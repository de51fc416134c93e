"""The C-ABI library on the CPU: it loads, exports every declared symbol, its
struct layouts match the header as compiled by gcc, and the host-only entry
points (validation, parameter layout, workspace queries, argument checks)
behave as documented.  No GPU work is launched here."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2402_02190_amd import _lib
from paper_2402_02190_amd._lib import CpraError
from workloads import csr_from_edges, erdos_renyi_graph, random_regular_graph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpra.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpra_[a-z0-9_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.exported_symbols())
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (cpra_\w+)", out))
    assert set(names) <= exported


def test_abi_version_and_status_strings():
    lib = _lib.lib()
    assert lib.cpra_abi_version() == 8
    for code, name in _lib.STATUS.items():
        assert lib.cpra_status_string(code).decode() == name


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "cpra.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(cpra_csr), sizeof(cpra_loss_cfg), sizeof(cpra_model_cfg),
         sizeof(cpra_adam_cfg), sizeof(cpra_step_cfg));
  printf("%zu %zu %zu %zu %zu %zu\\n", offsetof(cpra_csr, inv_deg), offsetof(cpra_loss_cfg, lambda),
         offsetof(cpra_loss_cfg, step_counter), offsetof(cpra_loss_cfg, T),
         offsetof(cpra_step_cfg, adam), offsetof(cpra_loss_cfg, edge_weight));
  printf("%zu\\n", offsetof(cpra_csr, col_inv_deg));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(cpra_early_stop_state), sizeof(cpra_early_stop_cfg),
         offsetof(cpra_step_cfg, early_stop), offsetof(cpra_early_stop_cfg, state),
         offsetof(cpra_early_stop_state, stop_step));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in lines[0].split()]
    offs = [int(x) for x in lines[1].split()]
    assert sizes == [C.sizeof(_lib.Csr), C.sizeof(_lib.LossCfg), C.sizeof(_lib.ModelCfg),
                     C.sizeof(_lib.AdamCfg), C.sizeof(_lib.StepCfg)]
    assert offs == [_lib.Csr.inv_deg.offset, _lib.LossCfg.lambda_.offset,
                    _lib.LossCfg.step_counter.offset, _lib.LossCfg.T.offset, _lib.StepCfg.adam.offset,
                    _lib.LossCfg.edge_weight.offset]
    assert int(lines[2]) == _lib.Csr.col_inv_deg.offset
    assert [int(x) for x in lines[3].split()] == [
        C.sizeof(_lib.EarlyStopState), C.sizeof(_lib.EarlyStopCfg), _lib.StepCfg.early_stop.offset,
        _lib.EarlyStopCfg.state.offset, _lib.EarlyStopState.stop_step.offset]


def _validate(rp, ci, w=None):
    from paper_2402_02190_amd import api
    api.csr_validate_host(rp, ci, w)


def test_validate_accepts_generated_graphs():
    for g in (random_regular_graph(50, 3, 0), erdos_renyi_graph(80, 0.05, 1)):
        _validate(g.row_ptr, g.col_idx)
    g = erdos_renyi_graph(30, 0.2, 2)
    u, v, _ = g.edge_list()
    gw = csr_from_edges(30, u, v, np.linspace(0.5, 2, u.size))
    _validate(gw.row_ptr, gw.col_idx, gw.weight)


@pytest.mark.parametrize("mutation,code", [
    ("row_ptr0", "CPRA_ERR_CSR"), ("nonmonotone", "CPRA_ERR_CSR"), ("range", "CPRA_ERR_CSR"),
    ("unsorted", "CPRA_ERR_CSR"), ("selfloop", "CPRA_ERR_CSR"), ("asym", "CPRA_ERR_CSR"),
    ("nanweight", "CPRA_ERR_NONFINITE"), ("asymweight", "CPRA_ERR_CSR")])
def test_validate_rejects_malformed_csr(mutation, code):
    g = random_regular_graph(12, 3, 5)
    rp = g.row_ptr.copy()
    ci = g.col_idx.copy()
    w = None
    if mutation == "row_ptr0":
        rp = rp + 1
    elif mutation == "nonmonotone":
        rp[3], rp[4] = rp[4], rp[3]
    elif mutation == "range":
        ci[0] = 12
    elif mutation == "unsorted":
        ci[0], ci[1] = ci[1], ci[0]
    elif mutation == "selfloop":
        ci[rp[2]] = 2
        ci[rp[2]: rp[3]] = np.sort(ci[rp[2]: rp[3]])
    elif mutation == "asym":
        u, v, _ = g.edge_list()
        g2 = csr_from_edges(12, u[1:], v[1:])
        rp, ci = g2.row_ptr.copy(), g2.col_idx.copy()
        # re-add only one direction of the removed edge
        a, b = int(u[0]), int(v[0])
        row = list(ci[rp[a]: rp[a + 1]]) + [b]
        ci = np.concatenate([ci[: rp[a]], np.sort(row), ci[rp[a + 1]:]]).astype(np.int32)
        rp[a + 1:] += 1
    elif mutation == "nanweight":
        w = np.ones(ci.size, dtype=np.float32)
        w[5] = np.nan
    elif mutation == "asymweight":
        w = np.ones(ci.size, dtype=np.float32)
        w[0] = 2.0
    with pytest.raises(CpraError) as ei:
        _validate(rp, ci, w)
    assert ei.value.name == code


def test_model_param_count_and_offsets_host_only():
    from paper_2402_02190_amd import api
    cfg = api.make_model_cfg(api.SAGE, 2, 1584, 1584, 20)
    n_nodes = 0  # embedding excluded: the paper's tables count only layer weights
    assert api.model_param_count(cfg, n_nodes) == 5_083_076
    cfg = api.make_model_cfg(api.SAGE, 2, 2500, 2500, 121)
    assert api.model_param_count(cfg, 0) == 13_107_621
    cfg = api.make_model_cfg(api.GCN, 3, 128, 128, 64)
    offs = api.model_param_offsets(cfg, 10)
    assert offs[0] == 0 and offs[1] == 10 * 128 and offs[2] == offs[1] + 128 * 128
    assert offs[3] == -1 and offs[4] == offs[2] + 128 * 128
    assert api.model_param_count(cfg, 10) == 10 * 128 + 2 * (128 * 128 * 2 + 128 * 64)
    # one network per graph: every layer block repeated G times (Ws, then Wn, then b)
    G = 7
    cfg = api.make_model_cfg(api.SAGE, 2, 16, 16, 8, weight_groups=G)
    offs = api.model_param_offsets(cfg, 50)
    assert offs[1] == 50 * 16 and offs[2] == offs[1] + G * 16 * 16 and offs[3] == offs[2] + G * 16 * 16
    assert offs[4] == offs[3] + G * 16 and offs[5] == offs[4] + G * 8 * 16
    assert api.model_param_count(cfg, 50) == 50 * 16 + G * (2 * 16 * 16 + 16 + 2 * 8 * 16 + 8)


def test_host_argument_errors_need_no_gpu():
    from paper_2402_02190_amd import api
    lib = _lib.lib()
    csr = _lib.Csr(10, 1, 20, 8, 8, None, None, 8, 8)  # pointers never dereferenced on failure
    bad_alpha = api.make_loss_cfg(api.MIS, 4, None, alpha=3)
    assert lib.cpra_loss_fwd_bwd(C.byref(csr), C.byref(bad_alpha), 8, 4, None, 0, None, 0, None,
                                 None, 0, None) == 4
    assert "alpha" in lib.cpra_last_error_message().decode()
    nan_cfg = api.make_loss_cfg(api.MAXCUT, 4, None, gamma=float("nan"))
    assert lib.cpra_loss_fwd_bwd(C.byref(csr), C.byref(nan_cfg), 8, 4, None, 0, None, 0, None,
                                 None, 0, None) == 8
    ok_cfg = api.make_loss_cfg(api.MAXCUT, 4, None)
    # workspace too small is detected before any launch
    assert lib.cpra_loss_fwd_bwd(C.byref(csr), C.byref(ok_cfg), 8, 4, None, 0, None, 0, None,
                                 None, 0, None) == 6
    big = _lib.Csr(10, 1, 2 ** 31, 8, 8, None, None, 8, 8)
    assert lib.cpra_loss_fwd_bwd(C.byref(big), C.byref(ok_cfg), 8, 4, None, 0, None, 0, None,
                                 None, 0, None) == 5
    assert lib.cpra_gemm(0, 0, -1, 4, 4, 8, 4, 8, 4, 0.0, 8, 4, None, 0, None, 0, None) == 2
    ew_cfg = api.make_loss_cfg(api.MAXCUT, 4, None)
    ew_cfg.edge_weight, ew_cfg.ld_edge_weight = 8, 3  # leading dimension below S
    assert lib.cpra_loss_fwd_bwd(C.byref(csr), C.byref(ew_cfg), 8, 4, None, 0, None, 0, None,
                                 None, 0, None) == 2
    ddof_cfg = api.make_loss_cfg(api.MAXCUT, 1, None, nu=0.5, std_ddof=1)
    assert lib.cpra_loss_fwd_bwd(C.byref(csr), C.byref(ddof_cfg), 8, 1, None, 0, None, 0, None,
                                 None, 0, None) == 4
    mis_cfg = api.make_loss_cfg(api.MIS, 4, None)
    assert lib.cpra_loss_fwd_bwd(C.byref(csr), C.byref(mis_cfg), 8, 4, None, 0, None, 0, None,
                                 None, 0, None) == 1
    adam = _lib.AdamCfg(1e-3, 0.9, 1.5, 1e-8, 0.0)
    assert lib.cpra_adam_step(4, 8, 8, 8, 8, C.byref(adam), 1, None, None) == 4
    assert lib.cpra_capture_begin(None) == 4


def test_workspace_queries_are_host_only():
    from paper_2402_02190_amd import api
    csr = _lib.Csr(10000, 1, 50000, 8, 8, None, None, 8, 8)
    cfg = api.make_loss_cfg(api.MIS, 100, None)
    assert api.loss_workspace_bytes(csr, cfg) >= 10000 * 100 * 4
    mcfg = api.make_model_cfg(api.SAGE, 2, 256, 256, 100)
    assert api.model_workspace_bytes(csr, mcfg) > 0
    assert api.gemm_workspace_bytes(1, 0, 200, 256, 10000) > 0  # weight-gradient shape splits K
    assert api.gemm_workspace_bytes(0, 1, 64, 64, 8) == 0       # one short K step: never split


def test_configs_keep_the_tensors_whose_addresses_they_hold():
    """A tensor passed straight into a config builder lives as long as the config."""
    import gc
    import weakref
    import torch
    from paper_2402_02190_amd import api
    lam = torch.linspace(0.5, 2.0, 4)
    ref = weakref.ref(lam)
    cfg = api.make_loss_cfg(api.MIS, 4, lam)
    del lam
    gc.collect()
    assert ref() is not None and cfg.lambda_ == ref().data_ptr()
    del cfg
    gc.collect()
    assert ref() is None
