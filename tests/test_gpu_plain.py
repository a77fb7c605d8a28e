"""GPU parity of the plain (analytic-Jacobian) path and of condensing and the
QP, through the C-ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle.condense import condense_local
from oracle.graph import jacobian_pattern
from oracle.msd import msd_linearize
from oracle.qp import qp_ipm
from paper_2602_17601_amd import workloads as wl
from tests.tolerance import U32, U64, h_err

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _plan_msd(P, dtype, L=1, n_c_max=None):
    plan = gn.Plan(P.M, P.nu, P.N, n_c_max if n_c_max is not None else max(P.rows.n, 1), dtype)
    plan.graph_set(P.row_ptr, P.col, L)
    plan.model_set_msd(P.msd, P.act)
    plan.rows_set(P.rows.node, P.rows.stage)
    return plan


def _cast(a, dtype):
    """Round to the device precision and back, so both sides see the same values."""
    return np.asarray(a, dtype=np.float64 if dtype == torch.float64 else np.float32).astype(np.float64)


def _condense_both(plan, tdt, A, B, c, x0, cost, rows, prow, pcol):
    """Run GPU condense and the oracle's local recursion on identical (rounded) inputs."""
    A, B, c, x0 = (_cast(v, tdt) for v in (A, B, c, x0))
    Q, q, R, r = (_cast(v, tdt) for v in (cost.Q, cost.q, cost.R, cost.r))
    rC, rd = _cast(rows.C, tdt), _cast(rows.d, tdt)
    n = plan.N * plan.nu
    H = torch.empty(n, n, dtype=tdt, device="cuda")
    g = torch.empty(n, dtype=tdt, device="cuda")
    Ct = torch.empty(rows.n, n, dtype=tdt, device="cuda")
    dt = torch.empty(rows.n, dtype=tdt, device="cuda")
    Gx = torch.empty(plan.N + 1, plan.M, 6, dtype=tdt, device="cuda")
    plan.condense(_t(A, tdt), _t(B, tdt), _t(c, tdt), _t(x0, tdt), _t(Q, tdt), _t(q, tdt), _t(R, tdt),
                  _t(r, tdt), _t(rC, tdt) if rows.n else None, _t(rd, tdt) if rows.n else None, H, g,
                  Ct if rows.n else None, dt if rows.n else None, Gx)
    torch.cuda.synchronize()
    ref = condense_local(A, B, c, prow, pcol, x0, Q, q, R, r,
                         wl.StateRows(rows.node, rows.stage, rC, rd))
    Rb = np.zeros((n, n))
    for k in range(plan.N):
        Rb[k * plan.nu:(k + 1) * plan.nu, k * plan.nu:(k + 1) * plan.nu] = R[k]
    return dict(H=_np(H), g=_np(g), Ct=_np(Ct), dt=_np(dt), Gx=_np(Gx)), ref, Rb


# ----------------------------------------------------------------------------- linearize (plain form)

def test_msd_linearize_fp64_matches_oracle_exactly():
    P = wl.msd10_fp64()
    plan = _plan_msd(P, gn.F64)
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    gp, gc = plan.graph_pattern()
    assert np.array_equal(gp, prow) and np.array_equal(gc, pcol)
    tA = torch.empty(P.N, plan.nnz, 6, 6, dtype=torch.float64, device="cuda")
    tB = torch.empty(P.N, P.M, 6, P.nu, dtype=torch.float64, device="cuda")
    tc = torch.empty(P.N, P.M, 6, dtype=torch.float64, device="cuda")
    plan.linearize(_t(P.xhat, torch.float64), _t(P.uhat, torch.float64), tA, tB, tc)
    torch.cuda.synchronize()
    np.testing.assert_allclose(_np(tA), A, rtol=0, atol=1e-15)
    np.testing.assert_allclose(_np(tB), B, rtol=0, atol=1e-16)
    np.testing.assert_allclose(_np(tc), c, rtol=0, atol=1e-15)


@pytest.mark.parametrize("M,hops,dtype", [(100, 2, torch.float32), (37, 3, torch.float64)])
def test_msd_linearize_nonlinear_matches_oracle(M, hops, dtype):
    P = wl.make_problem("msd_nl", M=M, hops=hops, N=5, n_act=3, model="msd", seed=21, x0_sigma=0.2, walk=0.05,
                        msd=wl.MSDParams(k3=50.0, gravity=9.81))
    gdt = gn.F64 if dtype == torch.float64 else gn.F32
    plan = _plan_msd(P, gdt)
    xh, uh = _cast(P.xhat, dtype), _cast(P.uhat, dtype)
    prow, pcol, A, B, c = msd_linearize(xh, uh, P.row_ptr, P.col, P.act, P.msd)
    tA = torch.empty(P.N, plan.nnz, 6, 6, dtype=dtype, device="cuda")
    tB = torch.empty(P.N, P.M, 6, P.nu, dtype=dtype, device="cuda")
    tc = torch.empty(P.N, P.M, 6, dtype=dtype, device="cuda")
    tf = torch.empty(P.N, P.M, 6, dtype=dtype, device="cuda")
    plan.linearize(_t(xh, dtype), _t(uh, dtype), tA, tB, tc, tf)
    torch.cuda.synchronize()
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert _rel(_np(tA), A) < tol
    assert _rel(_np(tB), B) < tol
    # c carries cancellation between f and the linear part: bound it by the state scale
    assert np.abs(_np(tc) - c).max() < tol * 10 * (1 + np.abs(xh).max())


# ----------------------------------------------------------------------------- condense

def test_condense_fp64_chain10_matches_oracle():
    P = wl.msd10_fp64()
    plan = _plan_msd(P, gn.F64)
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    out, ref, Rb = _condense_both(plan, torch.float64, A, B, c, P.x0, P.costs, P.rows, prow, pcol)
    assert h_err(out["H"], ref["H"], Rb, U64) < 1e-12
    assert _rel(out["g"], ref["g"]) < 1e-12
    assert _rel(out["Gx"], ref["Gx"]) < 1e-13
    assert np.array_equal(out["H"], out["H"].T)


def _random_blocks(rng, M, hops, L, N, nu, spread=0.6):
    rp, col = wl.chain_csr(M, hops)
    prow, pcol = jacobian_pattern(rp, col, M, L)
    nnz = len(pcol)
    A = rng.normal(0, spread / np.sqrt(6 * (prow[1:] - prow[:-1]).max()), size=(N, nnz, 6, 6))
    for i in range(M):                      # near-identity diagonal keeps the products bounded
        e = prow[i] + list(pcol[prow[i]:prow[i + 1]]).index(i)
        A[:, e] += np.eye(6) * 0.7
    B = rng.normal(size=(N, M, 6, nu))
    c = rng.normal(size=(N, M, 6))
    return rp, col, prow, pcol, A, B, c


@pytest.mark.parametrize("M,hops,L,N,nu,n_c,full_Q,dtype", [
    (37, 2, 2, 7, 9, 11, True, torch.float64),
    (37, 2, 2, 7, 9, 11, False, torch.float32),
    (130, 1, 3, 5, 6, 0, False, torch.float32),     # more than one node chunk, ragged tiles
    (50, 1, 1, 9, 4, 5, True, torch.float64),       # two-stage recursion launches, odd N (last stage alone)
    (1, 1, 1, 4, 3, 2, True, torch.float64),        # a single node (textbook dense condensing)
    (20, 2, 1, 1, 6, 3, False, torch.float64),      # horizon one
    (60, 2, 3, 12, 12, 9, False, torch.float32),    # 13-wide pattern: one-stage launches, up to 3 column slices
])
def test_condense_random_instances_match_oracle(M, hops, L, N, nu, n_c, full_Q, dtype):
    rng = np.random.default_rng(M * 100 + N)
    rp, col, prow, pcol, A, B, c = _random_blocks(rng, M, hops, L, N, nu)
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu, full_Q=full_Q)
    rows = wl.random_rows(rng, M, N, n_c)
    gdt = gn.F64 if dtype == torch.float64 else gn.F32
    plan = gn.Plan(M, nu, N, max(n_c, 1), gdt)
    plan.graph_set(rp, col, L)
    plan.rows_set(rows.node, rows.stage)
    out, ref, Rb = _condense_both(plan, dtype, A, B, c, x0, cost, rows, prow, pcol)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert h_err(out["H"], ref["H"], Rb, U64 if dtype == torch.float64 else U32) < tol
    assert _rel(out["g"], ref["g"]) < tol
    if n_c:
        assert _rel(out["Ct"], ref["Ct"]) < tol
        assert _rel(out["dt"], ref["dt"]) < tol
    assert _rel(out["Gx"], ref["Gx"]) < tol


def test_condense_paper_scale_plain_fp32_and_bitwise_repeatable():
    """1000-node 1-2-hop chain, N=20, nu=12, 200 obstacle rows, analytic Jacobians."""
    P = wl.gnn1000_bf16(model="msd")
    plan = _plan_msd(P, gn.F32)
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    cost = wl.random_costs(np.random.default_rng(99), P.M, P.N, P.nu)
    out, ref, Rb = _condense_both(plan, torch.float32, A, B, c, P.x0, cost, P.rows, prow, pcol)
    assert h_err(out["H"], ref["H"], Rb, U32) < 1e-5
    assert _rel(out["g"], ref["g"]) < 1e-5
    assert _rel(out["Ct"], ref["Ct"]) < 1e-5
    assert _rel(out["dt"], ref["dt"]) < 1e-5
    # determinism: identical bits over repeated calls
    tA, tB, tc = (_t(_cast(v, torch.float32), torch.float32) for v in (A, B, c))
    args = [_t(_cast(v, torch.float32), torch.float32) for v in (P.x0, cost.Q, cost.q, cost.R, cost.r,
                                                                  P.rows.C, P.rows.d)]
    n = P.N * P.nu
    Hs = []
    for _ in range(4):
        H = torch.empty(n, n, device="cuda")
        g = torch.empty(n, device="cuda")
        Ct = torch.empty(P.rows.n, n, device="cuda")
        dt = torch.empty(P.rows.n, device="cuda")
        plan.condense(tA, tB, tc, *args, H, g, Ct, dt)
        torch.cuda.synchronize()
        Hs.append((H.cpu().numpy().tobytes(), g.cpu().numpy().tobytes(), Ct.cpu().numpy().tobytes()))
    assert all(h == Hs[0] for h in Hs)


# ----------------------------------------------------------------------------- QP

def _solve_gpu(plan, H, g, lb, ub, Ct, lc, uc, dtype, **kw):
    n = len(g)
    u = torch.empty(n, dtype=dtype, device="cuda")
    info = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    nc = 0 if Ct is None else Ct.shape[0]
    plan.solve_box_qp(_t(H, dtype), _t(g, dtype), _t(lb, dtype), _t(ub, dtype),
                      _t(Ct, dtype) if nc else None, _t(lc, dtype) if nc else None,
                      _t(uc, dtype) if nc else None, u, info, settings=gn.default_admm_settings(**kw))
    torch.cuda.synchronize()
    return _np(u), gn.qp_info(info)


def _qp_rel(u, ref):
    return np.linalg.norm(u - ref) / max(np.linalg.norm(ref), 1e-12)


def test_qp_chain10_fp64_matches_ipm():
    P = wl.msd10_fp64()
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    cst = P.costs
    rng = np.random.default_rng(5)
    q = rng.normal(0, 30.0, size=cst.q.shape)       # drive some inputs onto their bounds
    l = condense_local(A, B, c, prow, pcol, P.x0, cst.Q, q, cst.R, cst.r, wl.no_rows())
    ref, *_ = qp_ipm(l["H"], l["g"], P.lb, P.ub)
    assert np.any(np.isclose(np.abs(ref), 1.0))
    plan = gn.Plan(P.M, P.nu, P.N, 1, gn.F64)
    u, info = _solve_gpu(plan, l["H"], l["g"], P.lb, P.ub, None, None, None, torch.float64)
    assert info.status == gn.QP_SOLVED, info.status
    assert _qp_rel(u, ref) < 1e-4


@pytest.mark.parametrize("n,nc,seed,dtype", [(60, 0, 1, torch.float32), (120, 40, 2, torch.float32),
                                             (240, 200, 3, torch.float32), (45, 17, 4, torch.float64)])
def test_qp_random_with_active_rows_matches_ipm(n, nc, seed, dtype):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    H = Qm @ np.diag(np.geomspace(0.1, 10.0, n)) @ Qm.T
    g = rng.normal(0, 3.0, size=n)
    lb, ub = -np.ones(n), np.ones(n)
    Ct = rng.normal(size=(nc, n)) / np.sqrt(n)
    lc = np.full(nc, -np.inf)
    uc = rng.uniform(-0.3, 0.3, size=nc)
    H, g, lb, ub, Ct, uc = (_cast(v, dtype) for v in (H, g, lb, ub, Ct, uc))
    H = 0.5 * (H + H.T)
    ref, *_ = qp_ipm(H, g, lb, ub, Ct, lc, uc)
    gdt = gn.F64 if dtype == torch.float64 else gn.F32
    plan = gn.Plan(1, n, 1, max(nc, 1), gdt)
    u, info = _solve_gpu(plan, H, g, lb, ub, Ct if nc else None, lc, uc, dtype)
    assert info.status == gn.QP_SOLVED, (info.status, info.iters)
    assert info.used_fp64 == 0
    assert _qp_rel(u, ref) < 1e-4


def test_qp_ill_conditioned_takes_the_fp64_path():
    rng = np.random.default_rng(7)
    n = 40
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    H = Qm @ np.diag(np.geomspace(1e-3, 1e6, n)) @ Qm.T
    H = 0.5 * (H + H.T)
    g = rng.normal(size=n)
    lb, ub = -10 * np.ones(n), 10 * np.ones(n)
    H32, g32 = _cast(H, torch.float32), _cast(g, torch.float32)
    H32 = 0.5 * (H32 + H32.T)
    ref, *_ = qp_ipm(H32, g32, lb, ub)
    plan = gn.Plan(1, n, 1, 1, gn.F32)
    u, info = _solve_gpu(plan, H32, g32, lb, ub, None, None, None, torch.float32, eps_abs=1e-9, eps_rel=1e-9,
                         max_iter=20000)
    assert info.used_fp64 == 1
    assert info.kappa_est > 1e7
    assert _qp_rel(u, ref) < 1e-4


def test_qp_condition_report_is_an_upper_bound_when_it_decides():
    """A well-conditioned QP keeps the FP32 factor on the bound ||K||_1 ||W||_1 ||W||_inf
    (W = L^{-1}), which the info reports: it must lie between kappa_1(K) and n kappa_1(K)
    (||W||_1 ||W||_inf <= n ||W||_2^2 = n ||K^{-1}||_2 <= n ||K^{-1}||_1), with K = H +
    sigma I + rho (I + Ct' Ct) formed here in FP64 (default rho 0.1, sigma 1e-6; box and
    one-sided rows have relative weight 1)."""
    rng = np.random.default_rng(11)
    n, nc = 60, 20
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    H = _cast(Qm @ np.diag(np.geomspace(0.1, 10.0, n)) @ Qm.T, torch.float32)
    H = 0.5 * (H + H.T)
    g = _cast(rng.normal(size=n), torch.float32)
    Ct = _cast(rng.normal(size=(nc, n)) / np.sqrt(n), torch.float32)
    lb, ub = -np.ones(n), np.ones(n)
    lc, uc = np.full(nc, -np.inf), np.full(nc, 0.5)
    plan = gn.Plan(1, n, 1, nc, gn.F32)
    u, info = _solve_gpu(plan, H, g, lb, ub, Ct, lc, uc, torch.float32)
    K = H + 1e-6 * np.eye(n) + 0.1 * (np.eye(n) + Ct.T @ Ct)
    kappa1 = np.linalg.norm(K, 1) * np.linalg.norm(np.linalg.inv(K), 1)
    assert info.status == gn.QP_SOLVED and info.used_fp64 == 0
    assert kappa1 * (1 - 1e-3) <= info.kappa_est <= 1.01 * n * kappa1, (info.kappa_est, kappa1)


def test_qp_reports_infeasible_rows():
    n = 6
    H = np.eye(n)
    g = np.zeros(n)
    lb, ub = -np.ones(n), np.ones(n)
    Ct = np.ones((1, n))
    lc, uc = np.array([10.0]), np.array([np.inf])     # sum(u) >= 10 with |u| <= 1: infeasible
    plan = gn.Plan(1, n, 1, 1, gn.F64)
    u, info = _solve_gpu(plan, H, g, lb, ub, Ct, lc, uc, torch.float64)
    assert info.status == gn.QP_PRIMAL_INFEASIBLE


def test_qp_maxiter_is_soft():
    rng = np.random.default_rng(3)
    n = 30
    H = np.diag(rng.uniform(0.1, 1.0, n))
    g = rng.normal(0, 5, n)
    plan = gn.Plan(1, n, 1, 1, gn.F32)
    u, info = _solve_gpu(plan, H, g, -np.ones(n), np.ones(n), None, None, None, torch.float32, max_iter=1,
                         check_every=1)
    assert info.status == gn.QP_MAXITER
    assert np.all(np.isfinite(u))


def test_qp_fp64_pass_with_the_factor_in_global_memory():
    """n = 240 with 200 rows and kappa(K) above 1e7: the FP64 pass takes over,
    and its packed factor (about 245 KB) does not fit one workgroup's LDS, so it
    lives in global memory.  Against the interior-point oracle within 1e-4.

    H has eigenvalues 1e-2 .. 1e8, mixed only inside 4x4 diagonal blocks (then
    symmetrically permuted): each entry is then of the size of its block's
    eigenvalues, so rounding H to FP32 keeps it positive definite (a dense
    rotation would not: the FP32 rounding of entries of size 1e8 / n moves
    the smallest eigenvalues by more than 1e-2)."""
    rng = np.random.default_rng(11)
    n, nc = 240, 200
    lam = np.geomspace(1e-2, 1e8, n)
    H = np.zeros((n, n))
    for b in range(0, n, 4):
        Qb, _ = np.linalg.qr(rng.normal(size=(4, 4)))
        H[b:b + 4, b:b + 4] = Qb @ np.diag(lam[b:b + 4]) @ Qb.T
    perm = rng.permutation(n)
    H = H[np.ix_(perm, perm)]
    g = rng.normal(0, 3.0, size=n) * np.sqrt(lam[np.argsort(perm)])
    lb, ub = -np.ones(n), np.ones(n)
    Ct = rng.normal(size=(nc, n)) / np.sqrt(n)
    uc = rng.uniform(-0.3, 0.3, size=nc)
    lc = np.full(nc, -np.inf)
    H, g, Ct, uc = (_cast(v, torch.float32) for v in (H, g, Ct, uc))
    H = 0.5 * (H + H.T)
    assert np.linalg.eigvalsh(H).min() > 0.9e-2      # the FP32-rounded H is still positive definite
    ref, *_ = qp_ipm(H, g, lb, ub, Ct, lc, uc)
    plan = gn.Plan(1, n, 1, nc, gn.F32)
    u, info = _solve_gpu(plan, H, g, lb, ub, Ct, lc, uc, torch.float32, eps_abs=1e-9, eps_rel=1e-9,
                         max_iter=40000)
    print("kappa", info.kappa_est, "iters", info.iters, "status", info.status, "rel", _qp_rel(u, ref))
    assert info.used_fp64 == 1 and info.kappa_est > 1e7
    assert info.status == gn.QP_SOLVED, (info.status, info.iters)
    assert _qp_rel(u, ref) < 1e-4


def test_qp_fp32_n360_factor_in_global_memory():
    """n = 360 (the largest condensed QP of the serving workload, N = 30 and
    n_u = 12): the FP32 packed factor (about 282 KB) lives in global memory.
    Against the interior-point oracle within 1e-4."""
    rng = np.random.default_rng(12)
    n, nc = 360, 60
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    H = Qm @ np.diag(np.geomspace(0.1, 10.0, n)) @ Qm.T
    g = rng.normal(0, 3.0, size=n)
    lb, ub = -np.ones(n), np.ones(n)
    Ct = rng.normal(size=(nc, n)) / np.sqrt(n)
    lc = np.full(nc, -np.inf)
    uc = rng.uniform(-0.3, 0.3, size=nc)
    H, g, Ct, uc = (_cast(v, torch.float32) for v in (H, g, Ct, uc))
    H = 0.5 * (H + H.T)
    ref, *_ = qp_ipm(H, g, lb, ub, Ct, lc, uc)
    plan = gn.Plan(1, n, 1, nc, gn.F32)
    u, info = _solve_gpu(plan, H, g, lb, ub, Ct, lc, uc, torch.float32)
    print("iters", info.iters, "status", info.status, "rel", _qp_rel(u, ref))
    assert info.status == gn.QP_SOLVED and info.used_fp64 == 0
    assert _qp_rel(u, ref) < 1e-4
