"""Pins of the oracle's tangent maps (jvp / vjp of the linearized dynamics):
central differences of the mass-spring-damper step (nonlinear springs, so the
blocks are neither symmetric nor stage-independent), the adjoint identity, and
a hand-built two-node system."""
import numpy as np

from oracle.msd import msd_linearize, msd_step
from oracle.tangent import jvp_blocks, vjp_blocks
from paper_2602_17601_amd import workloads as wl


def _problem():
    return wl.make_problem("tangent", M=7, hops=2, N=3, n_act=2, model="msd", seed=5, x0_sigma=0.3,
                           walk=0.1, msd=wl.MSDParams(k3=40.0, gravity=9.81))


def test_jvp_matches_central_differences_of_the_step():
    P = _problem()
    prow, pcol, A, B, _ = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    rng = np.random.default_rng(1)
    N, M, nu = P.N, P.M, P.nu
    dx = rng.normal(size=(N, M, 6))
    du = rng.normal(size=(N, nu))
    t = jvp_blocks(A, B, prow, pcol, dx, du)
    h = 1e-5
    for k in range(N):
        fp = msd_step(P.xhat[k] + h * dx[k], P.uhat[k] + h * du[k], P.row_ptr, P.col, P.act, P.msd)
        fm = msd_step(P.xhat[k] - h * dx[k], P.uhat[k] - h * du[k], P.row_ptr, P.col, P.act, P.msd)
        fd = (fp - fm) / (2 * h)
        assert np.abs(fd - t[k]).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_vjp_is_the_adjoint_of_jvp():
    P = _problem()
    prow, pcol, A, B, _ = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    rng = np.random.default_rng(2)
    dx = rng.normal(size=(P.N, P.M, 6))
    du = rng.normal(size=(P.N, P.nu))
    g = rng.normal(size=(P.N, P.M, 6))
    t = jvp_blocks(A, B, prow, pcol, dx, du)
    gx, gu = vjp_blocks(A, B, prow, pcol, g)
    for k in range(P.N):
        lhs = float(np.sum(g[k] * t[k]))
        rhs = float(np.sum(gx[k] * dx[k]) + np.sum(gu[k] * du[k]))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_two_nodes_by_hand():
    # pattern: node 0 reads {0, 1}, node 1 reads {1}; one stage, nu = 1
    prow = np.array([0, 2, 3])
    pcol = np.array([0, 1, 1])
    A = np.zeros((1, 3, 6, 6))
    A[0, 0] = np.eye(6) * 2.0          # A^{00}
    A[0, 1, 0, 5] = 3.0                # A^{01}: row 0 reads state 5 of node 1
    A[0, 2] = np.eye(6)                # A^{11}
    B = np.zeros((1, 2, 6, 1))
    B[0, 1, 2, 0] = 4.0                # node 1, row 2 reads the input
    dx = np.zeros((1, 2, 6))
    dx[0, 0, 1] = 1.0
    dx[0, 1, 5] = 1.0
    du = np.array([[0.5]])
    t = jvp_blocks(A, B, prow, pcol, dx, du)
    expect = np.zeros((1, 2, 6))
    expect[0, 0, 1] = 2.0              # 2 * dx^0_1
    expect[0, 0, 0] = 3.0              # 3 * dx^1_5
    expect[0, 1, 5] = 1.0              # dx^1_5
    expect[0, 1, 2] = 2.0              # 4 * du
    assert np.array_equal(t, expect)
    g = np.zeros((1, 2, 6))
    g[0, 0, 0] = 1.0
    gx, gu = vjp_blocks(A, B, prow, pcol, g)
    ex = np.zeros((1, 2, 6))
    ex[0, 0, 0] = 2.0                  # A^{00}' e_0
    ex[0, 1, 5] = 3.0                  # A^{01}' e_0 lands on state 5 of node 1
    assert np.array_equal(gx, ex) and np.array_equal(gu, np.zeros((1, 1)))
