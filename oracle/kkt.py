"""Uncondensed OCP solved through its KKT system (oracle; test infrastructure only).

The linear time-varying OCP of Sec. III-B eq. (2) without inequality rows,
with all states and inputs as unknowns z = [x_0; ...; x_N; u_0; ...; u_{N-1}]:
    minimize 1/2 z' blkdiag(Qbar, Rbar) z + [qbar; rbar]' z
    s.t.     x_0 = x0,  x_{k+1} - A_k x_k - B_k u_k = c_k
Optional extra equality rows E_u u = e_u (an active set found elsewhere) and
E_x x = e_x (active state rows).  Solved by one dense LU of the KKT matrix;
condensing must give the same input trajectory (Sec. III-B).
"""
from __future__ import annotations

import numpy as np

from .condense import dense_dynamics, stacked_costs


def solve_uncondensed(A, B, c, prow, pcol, x0, Q, q, R, r, Eu=None, eu=None, Ex=None, ex=None):
    """Returns (x [N+1][n_x], u [N][nu], nu_dyn multipliers)."""
    M = x0.shape[0]
    N = A.shape[0]
    nu = B.shape[3]
    nx = 6 * M
    Ad, Bd, cd = dense_dynamics(A, B, c, prow, pcol, M)
    Qb, qb, Rb, rb = stacked_costs(Q, q, R, r)
    nzx = (N + 1) * nx
    nz = nzx + N * nu
    P = np.zeros((nz, nz))
    P[:nzx, :nzx] = Qb
    P[nzx:, nzx:] = Rb
    p = np.concatenate([qb, rb])
    rows, rhs = [], []
    E0 = np.zeros((nx, nz))
    E0[:, :nx] = np.eye(nx)
    rows.append(E0); rhs.append(x0.reshape(-1))
    for k in range(N):
        Ek = np.zeros((nx, nz))
        Ek[:, (k + 1) * nx:(k + 2) * nx] = np.eye(nx)
        Ek[:, k * nx:(k + 1) * nx] = -Ad[k]
        Ek[:, nzx + k * nu:nzx + (k + 1) * nu] = -Bd[k]
        rows.append(Ek); rhs.append(cd[k])
    if Eu is not None and len(Eu):
        Z = np.zeros((len(Eu), nz))
        Z[:, nzx:] = Eu
        rows.append(Z); rhs.append(np.asarray(eu))
    if Ex is not None and len(Ex):
        Z = np.zeros((len(Ex), nz))
        Z[:, :nzx] = Ex
        rows.append(Z); rhs.append(np.asarray(ex))
    Eq = np.vstack(rows)
    e = np.concatenate(rhs)
    m = Eq.shape[0]
    K = np.block([[P, Eq.T], [Eq, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-p, e]))
    z = sol[:nz]
    return z[:nzx].reshape(N + 1, M, 6), z[nzx:].reshape(N, nu), sol[nz:]
