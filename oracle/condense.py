"""Condensing of the linear time-varying OCP (oracle; test infrastructure only).

Two independent computations of the same quantities:

* ``condense_dense`` -- the plain definition (Sec. III-B eq. condensed_matrices):
  dense prediction matrices with x = Gamma_u u + Gamma_x, then
  H = Gu' Qbar Gu + Rbar, g = Gu' Qbar Gx + Gu' qbar + rbar,
  Ct = Cbar_x Gu, dt = dbar_x - Cbar_x Gx.
* ``condense_local`` -- the paper's per-node recursion (Sec. V-B, proof of
  Thm. 1, eqs. sparse_gamma_i_xb / sparse_gamma_i_u, H, g and the stacked
  constraint rows): Gamma_x^i and Gamma_u^i are grown stage by stage from the
  last block rows of the neighbours j in tilde N_i, then H^i, g^i, Ct^i, dt^i
  are formed per node and summed / stacked.

Shapes: the Jacobian blocks follow a block pattern (prow, pcol) that contains
the diagonal; A is [N][nnz][6][6], B [N][M][6][nu], c [N][M][6], x0 [M][6];
Q is [N+1][M][6] (diagonal) or [N+1][M][6][6]; q [N+1][M][6]; R [N][nu][nu];
r [N][nu].  Stage-0 state rows are not allowed (they do not depend on u).
Stacked states are stage-major then node-major: x = [x_0; ...; x_N],
x_k = [x^1_k; ...; x^M_k].
"""
from __future__ import annotations

import numpy as np


def _qblock(Q, k, i):
    q = Q[k, i]
    return np.diag(q) if q.ndim == 1 else q


def dense_dynamics(A, B, c, prow, pcol, M):
    """Dense A_k [n_x][n_x], B_k [n_x][nu], c_k [n_x] from the block form."""
    N = A.shape[0]
    nx = 6 * M
    Ad = np.zeros((N, nx, nx))
    for k in range(N):
        for i in range(M):
            for e in range(prow[i], prow[i + 1]):
                j = int(pcol[e])
                Ad[k, 6 * i:6 * i + 6, 6 * j:6 * j + 6] = A[k, e]
    Bd = B.reshape(N, nx, -1)
    cd = c.reshape(N, nx)
    return Ad, Bd, cd


def prediction_matrices(Ad, Bd, cd, x0):
    """Gamma_u [(N+1)n_x][N nu] and Gamma_x [(N+1)n_x] with x = Gamma_u u + Gamma_x.

    Block (k, j) of Gamma_u is A_{k-1} ... A_{j+1} B_j for j < k and zero
    otherwise; Gamma_x_k = A_{k-1}...A_0 x0 + sum_{j<k} A_{k-1}...A_{j+1} c_j.
    """
    N, nx, nu = Bd.shape
    Gu = np.zeros(((N + 1) * nx, N * nu))
    Gx = np.zeros((N + 1) * nx)
    for k in range(N + 1):
        for j in range(k):
            P = np.eye(nx)
            for l in range(j + 1, k):
                P = Ad[l] @ P
            Gu[k * nx:(k + 1) * nx, j * nu:(j + 1) * nu] = P @ Bd[j]
        P = np.eye(nx)
        for l in range(k):
            P = Ad[l] @ P
        v = P @ x0.reshape(-1)
        for j in range(k):
            P = np.eye(nx)
            for l in range(j + 1, k):
                P = Ad[l] @ P
            v = v + P @ cd[j]
        Gx[k * nx:(k + 1) * nx] = v
    return Gu, Gx


def stacked_costs(Q, q, R, r):
    N1, M = Q.shape[0], Q.shape[1]
    nx = 6 * M
    Qb = np.zeros((N1 * nx, N1 * nx))
    for k in range(N1):
        for i in range(M):
            o = k * nx + 6 * i
            Qb[o:o + 6, o:o + 6] = _qblock(Q, k, i)
    N, nu = r.shape
    Rb = np.zeros((N * nu, N * nu))
    for k in range(N):
        Rb[k * nu:(k + 1) * nu, k * nu:(k + 1) * nu] = R[k]
    return Qb, q.reshape(-1), Rb, r.reshape(-1)


def state_row_matrix(rows, M, N):
    """Cbar_x [n_c][(N+1) n_x] and dbar_x [n_c] of single-node half-spaces."""
    nx = 6 * M
    C = np.zeros((rows.n, (N + 1) * nx))
    for t in range(rows.n):
        o = int(rows.stage[t]) * nx + 6 * int(rows.node[t])
        C[t, o:o + 6] = rows.C[t]
    return C, np.asarray(rows.d, dtype=np.float64)


def condense_dense(A, B, c, prow, pcol, x0, Q, q, R, r, rows):
    """Plain-definition condensing.  Returns dict(H, g, Ct, dt, Gu, Gx)."""
    M = x0.shape[0]
    N = A.shape[0]
    Ad, Bd, cd = dense_dynamics(A, B, c, prow, pcol, M)
    Gu, Gx = prediction_matrices(Ad, Bd, cd, x0)
    Qb, qb, Rb, rb = stacked_costs(Q, q, R, r)
    H = Gu.T @ Qb @ Gu + Rb
    g = Gu.T @ Qb @ Gx + Gu.T @ qb + rb
    Cx, dx = state_row_matrix(rows, M, N)
    return dict(H=H, g=g, Ct=Cx @ Gu, dt=dx - Cx @ Gx, Gu=Gu, Gx=Gx)


def condense_local(A, B, c, prow, pcol, x0, Q, q, R, r, rows):
    """The per-node recursion of Sec. V-B.  Returns dict(H, g, Ct, dt, S, Gx).

    S[k][i] is the last block row of Gamma_u^i after k steps ([6][N nu], the
    columns of u_j for j >= k are zero) and Gx[k][i] the last block of Gamma_x^i.
    """
    N, nnz = A.shape[0], A.shape[1]
    M = x0.shape[0]
    nu = B.shape[3]
    S = np.zeros((N + 1, M, 6, N * nu))
    Gx = np.zeros((N + 1, M, 6))
    Gx[0] = x0
    for n in range(N):                     # recursion index (stage)
        for i in range(M):                 # node
            s = np.zeros((6, N * nu))
            gx = c[n, i].copy()
            for e in range(prow[i], prow[i + 1]):   # j in tilde N_i
                j = int(pcol[e])
                s += A[n, e] @ S[n, j]
                gx += A[n, e] @ Gx[n, j]
            s[:, n * nu:(n + 1) * nu] = B[n, i]
            S[n + 1, i] = s
            Gx[n + 1, i] = gx
    H = np.zeros((N * nu, N * nu))
    g = np.zeros(N * nu)
    for i in range(M):                     # H^i and g^i, aggregated
        for k in range(N + 1):
            Qk = _qblock(Q, k, i)
            H += S[k, i].T @ Qk @ S[k, i]
            g += S[k, i].T @ (Qk @ Gx[k, i] + q[k, i])
    for k in range(N):
        H[k * nu:(k + 1) * nu, k * nu:(k + 1) * nu] += R[k]
        g[k * nu:(k + 1) * nu] += r[k]
    Ct = np.zeros((rows.n, N * nu))
    dt = np.zeros(rows.n)
    for t in range(rows.n):
        i, k = int(rows.node[t]), int(rows.stage[t])
        Ct[t] = rows.C[t] @ S[k, i]
        dt[t] = rows.d[t] - rows.C[t] @ Gx[k, i]
    return dict(H=H, g=g, Ct=Ct, dt=dt, S=S, Gx=Gx)


def rollout(A, B, c, prow, pcol, x0, u):
    """Simulate x_{k+1} = A_k x_k + B_k u_k + c_k (Sec. III-B eq. 2b) block-wise."""
    N = A.shape[0]
    M = x0.shape[0]
    nu = B.shape[3]
    x = np.zeros((N + 1, M, 6))
    x[0] = x0
    uu = u.reshape(N, nu)
    for k in range(N):
        for i in range(M):
            v = B[k, i] @ uu[k] + c[k, i]
            for e in range(prow[i], prow[i + 1]):
                v = v + A[k, e] @ x[k, int(pcol[e])]
            x[k + 1, i] = v
    return x


def ocp_cost(x, u, Q, q, R, r):
    """Sum over stages of 1/2 x'Qx + q'x (k = 0..N) and 1/2 u'Ru + r'u (k < N)."""
    N1, M = Q.shape[0], Q.shape[1]
    N, nu = r.shape
    uu = u.reshape(N, nu)
    J = 0.0
    for k in range(N1):
        for i in range(M):
            Qk = _qblock(Q, k, i)
            J += 0.5 * x[k, i] @ Qk @ x[k, i] + q[k, i] @ x[k, i]
    for k in range(N):
        J += 0.5 * uu[k] @ R[k] @ uu[k] + r[k] @ uu[k]
    return J
