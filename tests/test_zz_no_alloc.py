"""The allocation-free QP entry (gnmpc_solve_box_qp_noalloc) against the
plan-based gnmpc_solve_box_qp: the same kernels on the same inputs, so the
results must agree bit for bit; both are also checked against the
interior-point oracle within 1e-4.  Two calls in a row, the second with a
smaller problem, so the second runs on the scratch the first one left."""
import numpy as np
import pytest
import torch

from oracle.qp import qp_ipm

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _problem(rng, n, nc, dtype):
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    H = Qm @ np.diag(np.geomspace(0.1, 10.0, n)) @ Qm.T
    g = rng.normal(0, 3.0, size=n)
    Ct = rng.normal(size=(nc, n)) / np.sqrt(n)
    uc = rng.uniform(-0.3, 0.3, size=nc)
    npd = np.float64 if dtype == torch.float64 else np.float32
    H, g, Ct, uc = (np.asarray(v, npd).astype(np.float64) for v in (H, g, Ct, uc))
    H = 0.5 * (H + H.T)
    return H, g, -np.ones(n), np.ones(n), Ct, np.full(nc, -np.inf), uc


def _solve_both(P, dtype):
    H, g, lb, ub, Ct, lc, uc = P
    n, nc = len(g), Ct.shape[0]
    args = [_t(v, dtype) for v in (H, g, lb, ub, Ct, lc, uc)]
    u_plan = torch.empty(n, dtype=dtype, device="cuda")
    u_free = torch.full((n,), float("nan"), dtype=dtype, device="cuda")
    i_plan = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    i_free = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan = gn.Plan(1, n, 1, max(nc, 1), gn.F64 if dtype == torch.float64 else gn.F32)
    plan.solve_box_qp(*args, u_plan, i_plan)
    gn.solve_box_qp_noalloc(*args, u_free, i_free)
    torch.cuda.synchronize()
    return u_plan, i_plan, u_free, i_free


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_qp_matches_the_plan_entry_on_two_calls(dtype):
    rng = np.random.default_rng(21)
    # first call: n = 360 (the largest serving QP; the FP32 factor lives in the
    # scratch array, not in LDS), then a smaller one (factor in LDS)
    for n, nc in ((360, 60), (120, 40)):
        P = _problem(rng, n, nc, dtype)
        u_plan, i_plan, u_free, i_free = _solve_both(P, dtype)
        print(n, nc, dtype, gn.qp_info(i_free).status, gn.qp_info(i_free).iters)
        assert torch.equal(u_free, u_plan), (n, nc, "u differs from the plan entry")
        assert torch.equal(i_free, i_plan), (n, nc, "info differs from the plan entry")
        info = gn.qp_info(i_free)
        assert info.status == gn.QP_SOLVED
        H, g, lb, ub, Ct, lc, uc = P
        ref, *_ = qp_ipm(H, g, lb, ub, Ct, lc, uc)
        u = u_free.double().cpu().numpy()
        assert np.linalg.norm(u - ref) / max(np.linalg.norm(ref), 1e-12) < 1e-4


def test_noalloc_qp_fp64_handover_and_size_limits():
    """An ill-conditioned FP32 QP hands over to the FP64 pass through the
    scratch flags; sizes past the scratch are rejected on the host."""
    rng = np.random.default_rng(22)
    n = 40
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    H = Qm @ np.diag(np.geomspace(1e-3, 1e6, n)) @ Qm.T
    H = np.asarray(0.5 * (H + H.T), np.float32).astype(np.float64)
    H = 0.5 * (H + H.T)
    g = np.asarray(rng.normal(size=n), np.float32).astype(np.float64)
    P = (H, g, -10 * np.ones(n), 10 * np.ones(n), np.zeros((0, n)), np.zeros(0), np.zeros(0))
    st = gn.default_admm_settings(eps_abs=1e-9, eps_rel=1e-9, max_iter=20000)
    args = [_t(v, torch.float32) for v in P[:4]]
    u_plan = torch.empty(n, device="cuda")
    u_free = torch.empty(n, device="cuda")
    i_plan = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    i_free = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan = gn.Plan(1, n, 1, 1, gn.F32)
    plan.solve_box_qp(*args, None, None, None, u_plan, i_plan, settings=st)
    gn.solve_box_qp_noalloc(*args, None, None, None, u_free, i_free, settings=st)
    torch.cuda.synchronize()
    assert gn.qp_info(i_free).used_fp64 == 1
    assert torch.equal(u_free, u_plan) and torch.equal(i_free, i_plan)
    big = 465
    z = torch.zeros(big, big, device="cuda")
    v = torch.zeros(big, device="cuda")
    with pytest.raises(gn.GnmpcError) as e:
        gn.solve_box_qp_noalloc(z, v, v, v, None, None, None, v)
    assert e.value.status == gn.SHAPE
