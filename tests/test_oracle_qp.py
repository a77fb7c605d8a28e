"""Pins of the oracle's QP solver: closed form, brute-force enumeration, KKT
conditions, and agreement with the uncondensed OCP under the active set."""
import numpy as np
import pytest

from oracle.condense import condense_local, state_row_matrix
from oracle.kkt import solve_uncondensed
from oracle.msd import msd_linearize
from oracle.qp import kkt_residuals, qp_enumerate, qp_ipm
from paper_2602_17601_amd import workloads as wl


def _spd(rng, n, cond=10.0):
    Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.geomspace(1.0, cond, n)
    return Qm @ np.diag(ev) @ Qm.T


def test_unconstrained_is_newton_step():
    rng = np.random.default_rng(0)
    H = _spd(rng, 8)
    g = rng.normal(size=8)
    inf = np.full(8, np.inf)
    u, lam, G, h = qp_ipm(H, g, -inf, inf)
    np.testing.assert_allclose(u, np.linalg.solve(H, -g), atol=1e-12)
    # bounds far away are inactive
    u2, *_ = qp_ipm(H, g, -1e3 * np.ones(8), 1e3 * np.ones(8))
    np.testing.assert_allclose(u2, u, atol=1e-9)


@pytest.mark.parametrize("seed", range(6))
def test_ipm_matches_enumeration_box_and_rows(seed):
    rng = np.random.default_rng(seed)
    n, m = 4, 2
    H = _spd(rng, n, cond=30.0)
    g = 3 * rng.normal(size=n)
    lb, ub = -0.5 * np.ones(n), 0.5 * np.ones(n)
    Ct = rng.normal(size=(m, n))
    lc, uc = -0.3 * np.ones(m), 0.2 * np.ones(m)
    lc[1] = -np.inf
    u, lam, G, h = qp_ipm(H, g, lb, ub, Ct, lc, uc)
    ref = qp_enumerate(H, g, lb, ub, Ct, lc, uc)
    np.testing.assert_allclose(u, ref, atol=1e-8)
    st, pinf, comp, dinf = kkt_residuals(H, g, u, lam, G, h)
    assert max(st, pinf, comp, dinf) < 1e-9


def test_box_only_enumeration_with_many_active():
    rng = np.random.default_rng(42)
    n = 7
    H = _spd(rng, n, cond=5.0)
    g = 10 * rng.normal(size=n)       # pushes most variables onto their bounds
    lb, ub = -np.ones(n), np.ones(n)
    u, *_ = qp_ipm(H, g, lb, ub)
    ref = qp_enumerate(H, g, lb, ub)
    np.testing.assert_allclose(u, ref, atol=1e-8)
    assert np.sum(np.isclose(np.abs(ref), 1.0)) >= 2


def test_condensed_qp_equals_uncondensed_ocp_with_active_set():
    """Solve the condensed QP of the 10-node chain with input bounds and state rows,
    then re-solve the *uncondensed* OCP with the active constraints as equalities:
    the input trajectories must agree and the inequality multipliers be >= 0."""
    P = wl.msd10_fp64()
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    cst = P.costs
    rng = np.random.default_rng(8)
    g_push = wl.Costs(cst.Q, rng.normal(0, 50.0, size=cst.q.shape), cst.R, rng.normal(0, 0.2, size=cst.r.shape))
    # rows on the actuated nodes (where the inputs move the state), stages >= 2
    node = np.repeat(P.act, 2).astype(np.int32)
    stage = rng.integers(2, P.N + 1, size=node.size).astype(np.int32)
    Crow = np.hstack([rng.normal(size=(node.size, 3)), np.zeros((node.size, 3))])
    rows = wl.StateRows(node, stage, Crow, np.zeros(node.size))
    l = condense_local(A, B, c, prow, pcol, P.x0, g_push.Q, g_push.q, g_push.R, g_push.r, rows)
    lb, ub = -5.0 * np.ones(P.N * P.nu), 5.0 * np.ones(P.N * P.nu)
    u_box, *_ = qp_ipm(l["H"], l["g"], lb, ub)
    # make the state rows bind: put their upper bound just inside the box-only optimum
    lc = np.full(rows.n, -np.inf)
    uc = l["Ct"] @ u_box - 0.2 * np.abs(l["Ct"]).sum(axis=1)
    u, lam, G, h = qp_ipm(l["H"], l["g"], lb, ub, l["Ct"], lc, uc)
    st, pinf, comp, dinf = kkt_residuals(l["H"], l["g"], u, lam, G, h)
    assert max(st, pinf, comp, dinf) < 1e-8
    act_u = np.isclose(u, ub, atol=1e-9) | np.isclose(u, lb, atol=1e-9)
    act_r = np.isclose(l["Ct"] @ u, uc, atol=1e-9)
    assert act_u.any() and act_r.any()
    Eu = np.eye(P.N * P.nu)[act_u]
    eu = u[act_u]
    Cx, _ = state_row_matrix(rows, P.M, P.N)
    # row t: C x^i_k = uc_t + (d_t - dt_t)  (Ct u - dt = C x - d)
    ex = (uc + rows.d - l["dt"])[act_r]
    x, u_unc, _ = solve_uncondensed(A, B, c, prow, pcol, P.x0, g_push.Q, g_push.q, g_push.R, g_push.r,
                                    Eu=Eu, eu=eu, Ex=Cx[act_r], ex=ex)
    np.testing.assert_allclose(u_unc.reshape(-1), u, atol=1e-8)
