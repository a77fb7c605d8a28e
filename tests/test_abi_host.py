"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, validates arguments before touching a GPU, and its graph preparation
is bit-exact against the oracle's closure."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.graph import jacobian_pattern
from paper_2602_17601_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gnmpc.h")

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gnmpc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = gn.lib()
    names = _declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_version_and_status_strings():
    assert "gfx950" in gn.version()
    assert gn.status_string(gn.BAD_GRAPH) == "malformed graph"
    assert gn.status_string(gn.BAD_CONSTRAINT) == "bad constraint row"


@pytest.mark.parametrize("M,hops,L", [(10, 1, 1), (100, 2, 2), (1000, 2, 3), (1000, 2, 1), (37, 3, 2)])
def test_closure_bit_exact_against_oracle(M, hops, L):
    rp, col = wl.chain_csr(M, hops)
    prow, pcol = gn.graph_closure(rp, col, L)
    orow, ocol = jacobian_pattern(rp, col, M, L)
    assert np.array_equal(prow, orow) and np.array_equal(pcol, ocol)


def test_closure_on_irregular_directed_graph():
    rng = np.random.default_rng(0)
    M = 60
    rows = []
    for i in range(M):
        k = int(rng.integers(0, 5))
        rows.append(sorted(set(int(j) for j in rng.integers(0, M, size=k)) - {i}))
    rp = np.zeros(M + 1, np.int32)
    for i in range(M):
        rp[i + 1] = rp[i] + len(rows[i])
    col = np.asarray([j for r in rows for j in r], np.int32)
    for L in (1, 2, 4):
        prow, pcol = gn.graph_closure(rp, col, L)
        orow, ocol = jacobian_pattern(rp, col, M, L)
        assert np.array_equal(prow, orow) and np.array_equal(pcol, ocol)


def test_graph_check_rejects_malformed_csr():
    rp, col = wl.chain_csr(6, 1)
    assert gn.graph_check(rp, col) == gn.OK
    bad = col.copy(); bad[0], bad[1] = bad[1], bad[0]           # row 1 unsorted
    assert gn.graph_check(rp, bad) == gn.BAD_GRAPH
    bad = col.copy(); bad[1] = bad[2] = 0                         # duplicate
    assert gn.graph_check(rp, bad) == gn.BAD_GRAPH
    bad = col.copy(); bad[0] = 0                                  # self loop (row 0 holds 1)
    assert gn.graph_check(rp, bad) == gn.BAD_GRAPH
    bad = col.copy(); bad[-1] = 6                                 # out of range
    assert gn.graph_check(rp, bad) == gn.BAD_GRAPH
    rbad = rp.copy(); rbad[-1] += 1                               # row_ptr[M] != E
    assert gn.graph_check(rbad, col) == gn.BAD_GRAPH
    rbad = rp.copy(); rbad[2], rbad[3] = rbad[3], rbad[2]          # decreasing row_ptr
    assert gn.graph_check(rbad, col) == gn.BAD_GRAPH


def test_plan_create_validates_before_touching_the_gpu():
    L = gn.lib()
    h = C.c_void_p()
    for d in [gn.Dims(0, 6, 10, 0, gn.F64), gn.Dims(10, 0, 10, 0, gn.F64), gn.Dims(10, 6, 0, 0, gn.F64),
              gn.Dims(10, 6, 10, -1, gn.F64), gn.Dims(10, 6, 10, 0, 7), gn.Dims(10, 6, 10, 0, gn.BF16)]:
        assert L.gnmpc_plan_create(C.byref(h), C.byref(d), 0) == gn.INVALID_ARG
    assert L.gnmpc_plan_create(C.byref(h), None, 0) == gn.INVALID_ARG


def test_plan_create_without_a_gpu_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = gn.lib()
    h = C.c_void_p()
    d = gn.Dims(10, 6, 10, 0, gn.F64)
    assert L.gnmpc_plan_create(C.byref(h), C.byref(d), 0) == gn.NO_DEVICE


def test_null_plan_calls_are_rejected():
    L = gn.lib()
    assert L.gnmpc_graph_set(None, None, None, 0, 0, 1) == gn.INVALID_ARG
    assert L.gnmpc_linearize(None, None, None, None, None, None, None, None, None) == gn.INVALID_ARG
    assert L.gnmpc_rollout_linear(None, None, None, None, None, None, None, None) == gn.INVALID_ARG
    assert L.gnmpc_rows_set(None, 0, None, None) == gn.INVALID_ARG
    s = gn.AdmmSettings()
    assert L.gnmpc_solve_box_qp(None, 1, None, None, None, None, 0, None, None, None, C.byref(s), None, None,
                                None) == gn.INVALID_ARG


def test_linearization_report_layout_matches_the_header():
    """gnmpc_lin_info: four int32 then six int64 counts (48 bytes, no padding)."""
    assert gn.LIN_INFO_BYTES == 4 * 4 + 6 * 8
    assert gn.LinInfo.nonfinite.offset == 16


def test_noalloc_qp_validates_before_touching_the_gpu():
    """gnmpc_solve_box_qp_noalloc checks dtype, arrays, sizes and settings on
    the host (no GPU is needed to be told no)."""
    L = gn.lib()
    s = gn.AdmmSettings()
    L.gnmpc_admm_default_settings(C.byref(s))
    fake = C.c_void_p(256)   # never dereferenced: every call below fails validation first
    f = L.gnmpc_solve_box_qp_noalloc
    assert f(gn.BF16, 8, fake, fake, fake, fake, 0, None, None, None, C.byref(s), fake, None, None) == gn.INVALID_ARG
    assert f(gn.F32, 8, None, fake, fake, fake, 0, None, None, None, C.byref(s), fake, None, None) == gn.INVALID_ARG
    assert f(gn.F32, 8, fake, fake, fake, fake, 3, None, None, None, C.byref(s), fake, None, None) == gn.INVALID_ARG
    assert f(gn.F32, 465, fake, fake, fake, fake, 0, None, None, None, C.byref(s), fake, None, None) == gn.SHAPE
    assert f(gn.F64, 0, fake, fake, fake, fake, 0, None, None, None, C.byref(s), fake, None, None) == gn.SHAPE
    assert f(gn.F32, 64, fake, fake, fake, fake, 100000, fake, None, None, C.byref(s), fake, None,
             None) == gn.UNSUPPORTED
    bad = gn.AdmmSettings()
    L.gnmpc_admm_default_settings(C.byref(bad))
    bad.alpha = 2.5
    assert f(gn.F32, 8, fake, fake, fake, fake, 0, None, None, None, C.byref(bad), fake, None, None) == gn.INVALID_ARG
