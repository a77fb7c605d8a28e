"""Pins of the oracle's GNN-MPC loop iteration (Algorithm 1): on a linear
spring-damper chain with inactive bounds it must reproduce the finite-horizon
LQ optimum of the backward Riccati recursion (a textbook computation that shares
nothing with condensing or the QP solver), and the shift must hand the next
iteration the optimal trajectory advanced by one stage; in closed loop on the
nonlinear chain it must respect the input bounds and beat zero input."""
import numpy as np

from oracle.mpc import initial_trajectory, rti_step
from oracle.msd import msd_linearize, msd_step
from paper_2602_17601_amd import workloads as wl


def _lin(P, prm):
    return lambda xh, uh: msd_linearize(xh, uh, P.row_ptr, P.col, P.act, prm)


def _dense(prow, pcol, A0, B0, M):
    Ad = np.zeros((6 * M, 6 * M))
    for i in range(M):
        for e in range(prow[i], prow[i + 1]):
            j = int(pcol[e])
            Ad[6 * i:6 * i + 6, 6 * j:6 * j + 6] = A0[e]
    return Ad, B0.reshape(6 * M, -1)


def test_rti_step_on_a_linear_chain_is_the_riccati_lq_optimum_and_shifts_it():
    prm = wl.MSDParams(k=10.0, c=0.1, m=1.0, dt=0.05)
    P = wl.make_problem("lq", M=6, hops=1, N=8, n_act=2, model="msd", seed=21, msd=prm, x0_sigma=0.3, umax=1e3)
    N, M, nu = P.N, P.M, P.nu
    xh, uh = initial_trajectory(P.x0, N, nu)
    out = rti_step(P.x0, xh, uh, _lin(P, prm), P.costs, wl.no_rows(), P.lb, P.ub)
    prow, pcol, A, B, c = msd_linearize(xh, uh, P.row_ptr, P.col, P.act, prm)
    assert np.abs(c).max() < 1e-12  # a linear model has no offset
    Ad, Bd = _dense(prow, pcol, A[0], B[0], M)
    Qk = [np.diag(P.costs.Q[k].reshape(-1)) for k in range(N + 1)]
    Pm = Qk[N]
    K = [None] * N
    for k in range(N - 1, -1, -1):
        K[k] = np.linalg.solve(P.costs.R[k] + Bd.T @ Pm @ Bd, Bd.T @ Pm @ Ad)
        Pm = Qk[k] + Ad.T @ Pm @ (Ad - Bd @ K[k])
    x = P.x0.reshape(-1).copy()
    xs, us = [x], []
    for k in range(N):
        u = -K[k] @ x
        x = Ad @ x + Bd @ u
        us.append(u)
        xs.append(x)
    us, xs = np.concatenate(us), np.stack(xs).reshape(N + 1, M, 6)
    assert np.linalg.norm(out["u"] - us) <= 1e-8 * np.linalg.norm(us)
    assert np.linalg.norm(out["x"] - xs) <= 1e-8 * np.linalg.norm(xs)
    # the shift: stage k of the next trajectory is stage k + 1 of the optimum
    U = us.reshape(N, nu)
    assert np.allclose(out["xhat"][:N], xs[1:], rtol=0, atol=1e-10)
    assert np.allclose(out["xhat"][N], xs[N], rtol=0, atol=1e-10)
    assert np.allclose(out["uhat"][:N - 1], U[1:], rtol=0, atol=1e-10)
    assert np.allclose(out["uhat"][N - 1], U[N - 1], rtol=0, atol=1e-10)


def test_closed_loop_on_the_nonlinear_chain_respects_bounds_and_beats_zero_input():
    prm = wl.MSDParams(k=10.0, c=0.1, m=1.0, dt=0.05, k3=50.0)
    P = wl.make_problem("cl", M=8, hops=2, N=15, n_act=2, model="msd", seed=22, msd=prm, x0_sigma=0.05, umax=0.5,
                        qdiag=(100, 100, 100, 1, 1, 1), rho_r=1e-3)
    N, nu = P.N, P.nu
    Q = P.costs.Q[0].reshape(-1)

    def cost(x, u):
        return 0.5 * float(np.sum(Q * x.reshape(-1) ** 2)) + 0.5 * float(u @ P.costs.R[0] @ u)

    x, x_free = P.x0.copy(), P.x0.copy()
    xh, uh = initial_trajectory(x, N, nu)
    J, J_free, at_bound = 0.0, 0.0, 0
    for t in range(30):
        out = rti_step(x, xh, uh, _lin(P, prm), P.costs, wl.no_rows(), P.lb, P.ub)
        u0 = out["u"][:nu]
        assert np.all(np.abs(u0) <= 0.5 + 1e-9)
        at_bound += int(np.any(np.abs(u0) > 0.5 - 1e-6))
        J += cost(x, u0)
        J_free += cost(x_free, np.zeros(nu))
        x = msd_step(x, u0, P.row_ptr, P.col, P.act, prm)
        x_free = msd_step(x_free, np.zeros(nu), P.row_ptr, P.col, P.act, prm)
        xh, uh = out["xhat"], out["uhat"]
    assert at_bound > 0  # the bounds were active at some step
    assert J < 0.9 * J_free
