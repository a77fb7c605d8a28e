"""Pins of the oracle's graph closure and mass-spring-damper Jacobians."""
import numpy as np
import pytest

from oracle.graph import ball, jacobian_pattern
from oracle.msd import msd_linearize, msd_step
from paper_2602_17601_amd import workloads as wl


def _nnz_closed_form(M, r):
    return sum(min(M - 1, i + r) - max(0, i - r) + 1 for i in range(M))


@pytest.mark.parametrize("M,hops,L,expect", [(10, 1, 1, 28), (100, 2, 2, 880),
                                             (1000, 2, 3, 12958), (1000, 2, 1, 4994)])
def test_pattern_counts(M, hops, L, expect):
    rp, col = wl.chain_csr(M, hops)
    assert len(col) == sum(2 * (M - h) for h in range(1, hops + 1))
    prow, pcol = jacobian_pattern(rp, col, M, L)
    assert prow[-1] == expect == _nnz_closed_form(M, hops * L)
    # every row sorted and contains the diagonal
    for i in range(M):
        r = pcol[prow[i]:prow[i + 1]]
        assert np.all(np.diff(r) > 0) and i in r


def test_ball_by_hand_on_directed_graph():
    # edges (sender -> receiver): 0->1, 1->2, 2->3, 3->1, 4->0 ; N_i = senders into i
    edges = [(0, 1), (1, 2), (2, 3), (3, 1), (4, 0)]
    M = 5
    rows = [[] for _ in range(M)]
    for s, t in edges:
        rows[t].append(s)
    rp = np.zeros(M + 1, np.int32)
    col = []
    for i in range(M):
        col += sorted(rows[i])
        rp[i + 1] = len(col)
    col = np.asarray(col, np.int32)
    assert ball(rp, col, 1, 0) == [1]
    assert ball(rp, col, 1, 1) == [0, 1, 3]
    assert ball(rp, col, 1, 2) == [0, 1, 2, 3, 4]
    assert ball(rp, col, 2, 1) == [1, 2]
    assert ball(rp, col, 4, 3) == [4]          # nothing sends into node 4
    assert ball(rp, col, 0, 2) == [0, 4]


def _dense_A(A, prow, pcol, M):
    D = np.zeros((6 * M, 6 * M))
    for i in range(M):
        for e in range(prow[i], prow[i + 1]):
            j = pcol[e]
            D[6 * i:6 * i + 6, 6 * j:6 * j + 6] = A[e]
    return D


def test_linear_msd_closed_form():
    """Hand-derived Jacobian of the linear chain under semi-implicit Euler:
    off-diagonal [[dt^2 k/m I, dt^2 c/m I],[dt k/m I, dt c/m I]], diagonal
    [[I - dt^2 k d/m I, dt I - dt^2 c d/m I],[-dt k d/m I, I - dt c d/m I]] with
    d = |N_i| + [anchored]; B = [dt^2/m I; dt/m I] on the node's inputs; c = 0."""
    P = wl.msd10_fp64()
    prm = P.msd
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, prm)
    dt, k, cc, m = prm.dt, prm.k, prm.c, prm.m
    I = np.eye(3)
    for i in range(P.M):
        d = (P.row_ptr[i + 1] - P.row_ptr[i]) + (1 if i == prm.anchor else 0)
        for e in range(prow[i], prow[i + 1]):
            j = pcol[e]
            if j == i:
                ref = np.block([[I - dt * dt * k * d / m * I, dt * I - dt * dt * cc * d / m * I],
                                [-dt * k * d / m * I, I - dt * cc * d / m * I]])
            else:
                ref = np.block([[dt * dt * k / m * I, dt * dt * cc / m * I],
                                [dt * k / m * I, dt * cc / m * I]])
            for kk in range(P.N):
                np.testing.assert_allclose(A[kk, e], ref, rtol=0, atol=1e-15)
        for a_idx, a in enumerate(P.act):
            if a == i:
                Bref = np.zeros((6, P.nu))
                Bref[:3, 3 * a_idx:3 * a_idx + 3] = dt * dt / m * I
                Bref[3:, 3 * a_idx:3 * a_idx + 3] = dt / m * I
                np.testing.assert_allclose(B[0, i], Bref, atol=1e-16)
    np.testing.assert_allclose(c, 0.0, atol=1e-14)
    # a damped anchored chain under symplectic Euler is stable
    rho = np.abs(np.linalg.eigvals(_dense_A(A[0], prow, pcol, P.M))).max()
    assert rho <= 1.0 + 1e-12


def test_nonlinear_msd_matches_central_differences():
    rng = np.random.default_rng(11)
    M, N = 6, 2
    rp, col = wl.chain_csr(M, 2)
    act = wl.actuated_nodes(M, 2)
    prm = wl.MSDParams(k3=50.0, gravity=9.81, anchor=0)
    xhat = rng.normal(0, 0.2, size=(N + 1, M, 6))
    uhat = rng.uniform(-1, 1, size=(N, 6))
    prow, pcol, A, B, c = msd_linearize(xhat, uhat, rp, col, act, prm)
    for k in range(N):
        Ad = _dense_A(A[k], prow, pcol, M)
        x = xhat[k].reshape(-1)
        h = 1e-6
        J = np.zeros((6 * M, 6 * M))
        for a in range(6 * M):
            xp = x.copy(); xp[a] += h
            xm = x.copy(); xm[a] -= h
            fp = msd_step(xp.reshape(M, 6), uhat[k], rp, col, act, prm).reshape(-1)
            fm = msd_step(xm.reshape(M, 6), uhat[k], rp, col, act, prm).reshape(-1)
            J[:, a] = (fp - fm) / (2 * h)
        np.testing.assert_allclose(Ad, J, atol=1e-8)
        JB = np.zeros((6 * M, 6))
        for a in range(6):
            up = uhat[k].copy(); up[a] += h
            um = uhat[k].copy(); um[a] -= h
            JB[:, a] = (msd_step(xhat[k], up, rp, col, act, prm)
                        - msd_step(xhat[k], um, rp, col, act, prm)).reshape(-1) / (2 * h)
        np.testing.assert_allclose(B[k].reshape(6 * M, 6), JB, atol=1e-9)
        # offset reproduces the nonlinear step at the nominal point
        f = msd_step(xhat[k], uhat[k], rp, col, act, prm).reshape(-1)
        np.testing.assert_allclose(Ad @ x + B[k].reshape(6 * M, 6) @ uhat[k] + c[k].reshape(-1),
                                   f, atol=1e-12)
