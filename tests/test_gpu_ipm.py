"""The interior-point QP solver (gnmpc_solve_qp_ipm) against the oracle's
interior-point method (refined on its active set, so exact for nondegenerate
problems), on random QPs with one- and two-sided rows, the condensed QP of the
1000-node chain with 200 obstacle rows (against the ADMM too), an
ill-conditioned H, and an infeasible one."""
import numpy as np
import pytest
import torch

from oracle.qp import qp_ipm
from paper_2602_17601_amd import workloads as wl

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _cast(a, dtype):
    return np.asarray(a, dtype=np.float64 if dtype == torch.float64 else np.float32).astype(np.float64)


def _ipm(plan, H, g, lb, ub, Ct, lc, uc, dtype, tol=1e-12):
    n = g.shape[0]
    u = torch.full((n,), float("nan"), dtype=dtype, device="cuda")
    info = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan.solve_qp_ipm(_t(H, dtype), _t(g, dtype), _t(lb, dtype), _t(ub, dtype),
                      None if Ct is None else _t(Ct, dtype), None if lc is None else _t(lc, dtype),
                      None if uc is None else _t(uc, dtype), u, info, tol=tol)
    torch.cuda.synchronize()
    return u.double().cpu().numpy(), gn.qp_info(info)


def _random_qp(n, nc, seed, cond=100.0):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    H = Qm @ np.diag(np.geomspace(10.0 / cond, 10.0, n)) @ Qm.T
    g = rng.normal(0, 3.0, size=n)
    lb, ub = -np.ones(n), np.ones(n)
    lb[::7] = -np.inf                         # some one-sided box entries
    Ct = rng.normal(size=(nc, n)) / np.sqrt(n)
    uc = rng.uniform(-0.3, 0.3, size=nc)
    lc = uc - rng.uniform(0.1, 1.0, size=nc)  # two-sided rows
    lc[::3] = -np.inf
    return 0.5 * (H + H.T), g, lb, ub, Ct, lc, uc


@pytest.mark.parametrize("n,nc,seed,dtype,tol", [(60, 0, 1, torch.float64, 1e-12), (120, 40, 2, torch.float64, 1e-12),
                                                 (240, 200, 3, torch.float64, 1e-10), (96, 30, 4, torch.float32, 1e-12)])
def test_ipm_matches_the_oracle_on_random_qps(n, nc, seed, dtype, tol):
    H, g, lb, ub, Ct, lc, uc = _random_qp(n, nc, seed)
    H, g, lb, ub, Ct, lc, uc = (_cast(v, dtype) for v in (H, g, lb, ub, Ct, lc, uc))
    H = 0.5 * (H + H.T)
    ref, *_ = qp_ipm(H, g, lb, ub, Ct if nc else None, lc if nc else None, uc if nc else None)
    plan = gn.Plan(1, n, 1, max(nc, 1), gn.F64 if dtype == torch.float64 else gn.F32)
    u, info = _ipm(plan, H, g, lb, ub, Ct if nc else None, lc if nc else None, uc if nc else None, dtype, tol)
    print((n, nc), "iters", info.iters, "mu", info.kappa_est, "rel", _rel(u, ref))
    assert info.status == gn.QP_SOLVED, (info.status, info.iters)
    # an interior-point stop leaves the iterate O(sqrt(mu)) from the exact minimizer
    # (the oracle refines to the vertex) where constraints are nearly degenerate
    assert _rel(u, ref) < max(1e-5, 10 * np.sqrt(info.kappa_est))
    assert np.all(u <= ub + 1e-9) and np.all(u >= lb - 1e-9)


def test_ipm_on_the_condensed_paper_scale_qp_agrees_with_admm_and_the_oracle():
    """1000-node chain (spring-damper form, FP32), N = 20, n_u = 12, 200 obstacle rows."""
    P = wl.gnn1000_bf16(model="msd")
    n = P.N * P.nu
    plan = gn.Plan(P.M, P.nu, P.N, P.rows.n, gn.F32)
    plan.graph_set(P.row_ptr, P.col, 1)
    plan.model_set_msd(P.msd, P.act)
    plan.rows_set(P.rows.node, P.rows.stage)
    f = torch.float32
    e = lambda *s: torch.empty(*s, device="cuda")
    A, B, c = e(P.N, plan.nnz, 6, 6), e(P.N, P.M, 6, P.nu), e(P.N, P.M, 6)
    plan.linearize(_t(P.xhat, f), _t(P.uhat, f), A, B, c)
    H, g, Ct, dt = e(n, n), e(n), e(P.rows.n, n), e(P.rows.n)
    plan.condense(A, B, c, _t(P.x0, f), _t(P.costs.Q, f), _t(P.costs.q, f), _t(P.costs.R, f), _t(P.costs.r, f),
                  _t(P.rows.C, f), _t(P.rows.d, f), H, g, Ct, dt)
    u_ipm = torch.empty(n, device="cuda")
    info = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan.solve_qp_ipm(H, g, _t(P.lb, f), _t(P.ub, f), Ct, None, dt, u_ipm, info, tol=1e-12)
    u_admm = torch.empty(n, device="cuda")
    plan.solve_box_qp(H, g, _t(P.lb, f), _t(P.ub, f), Ct, None, dt, u_admm)
    torch.cuda.synchronize()
    inf = gn.qp_info(info)
    assert inf.status == gn.QP_SOLVED, (inf.status, inf.iters)
    Hn, gn_, Ctn, dtn = (v.double().cpu().numpy() for v in (H, g, Ct, dt))
    Hn = 0.5 * (Hn + Hn.T)
    ref, *_ = qp_ipm(Hn, gn_, P.lb, P.ub, Ctn, np.full(P.rows.n, -np.inf), dtn)  # one-sided rows
    ui = u_ipm.double().cpu().numpy()
    print("iters", inf.iters, "ipm vs oracle", _rel(ui, ref), "admm vs oracle", _rel(u_admm.double().cpu().numpy(), ref))
    assert _rel(ui, ref) < 1e-5
    assert _rel(u_admm.double().cpu().numpy(), ref) < 1e-4


def test_ipm_handles_an_ill_conditioned_hessian():
    H, g, lb, ub, Ct, lc, uc = _random_qp(80, 20, 5, cond=1e8)
    ref, *_ = qp_ipm(H, g, lb, ub, Ct, lc, uc)
    plan = gn.Plan(1, 80, 1, 20, gn.F64)
    u, info = _ipm(plan, H, g, lb, ub, Ct, lc, uc, torch.float64)
    assert info.status == gn.QP_SOLVED
    assert _rel(u, ref) < 1e-5


def test_ipm_reports_an_infeasible_problem_and_rejects_bad_calls():
    n = 10
    H, g = np.eye(n), np.zeros(n)
    lb, ub = -np.ones(n), np.ones(n)
    Ct = np.zeros((1, n))
    Ct[0, 0] = 1.0
    lc, uc = np.array([2.0]), np.array([3.0])  # u_0 >= 2 contradicts u_0 <= 1
    plan = gn.Plan(1, n, 1, 1, gn.F64)
    u, info = _ipm(plan, H, g, lb, ub, Ct, lc, uc, torch.float64)
    assert info.status != gn.QP_SOLVED
    with pytest.raises(gn.GnmpcError) as e:
        plan.solve_qp_ipm(_t(H, torch.float64), _t(g, torch.float64), _t(lb, torch.float64), _t(ub, torch.float64),
                          None, None, None, torch.empty(n, dtype=torch.float64, device="cuda"), tol=0.0)
    assert e.value.status == gn.INVALID_ARG
