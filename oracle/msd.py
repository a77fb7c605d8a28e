"""Mass-spring-damper chain dynamics and analytic Jacobians (oracle; test
infrastructure only).

The stand-in plant of the plain (analytic-Jacobian) form.  It is a local,
homogeneous, differentiable node dynamics in the sense of Assumption 1
(Sec. IV-A), integrated with the same semi-implicit Euler scheme as the GNN
model of Sec. V-A eq. (forward_dynamics): v+ = v + dt a, p+ = p + dt v+.

Node acceleration (states are displacements from rest):
  a^i = 1/m [ sum_{j in N_i} ( F(p^j - p^i) + c (v^j - v^i) )
              + [i anchored] ( -F(p^i) - c v^i ) + f^i ] - gravity e_z
with the spring force F(d) = k d + k3 |d|^2 d and f^i the 3D input force on an
actuated node (zero elsewhere).
"""
from __future__ import annotations

import numpy as np

from .graph import in_neighbours, jacobian_pattern


def _force(d, k, k3):
    return k * d + k3 * float(d @ d) * d


def _dforce(d, k, k3):
    """d F / d d = k I + k3 (|d|^2 I + 2 d d^T)."""
    return k * np.eye(3) + k3 * (float(d @ d) * np.eye(3) + 2.0 * np.outer(d, d))


def input_force(u, i, act):
    """Force on node i from the stacked input u = [f_a1; f_a2; ...]."""
    hit = np.nonzero(np.asarray(act) == i)[0]
    if hit.size == 0:
        return np.zeros(3)
    a = int(hit[0])
    return np.asarray(u[3 * a:3 * a + 3], dtype=np.float64)


def msd_step(x, u, row_ptr, col, act, prm):
    """One step x -> x+ of the whole chain; x is [M][6]."""
    M = x.shape[0]
    xn = np.empty_like(x, dtype=np.float64)
    for i in range(M):
        p, v = x[i, :3], x[i, 3:]
        acc = np.zeros(3)
        for j in in_neighbours(row_ptr, col, i):
            acc += _force(x[j, :3] - p, prm.k, prm.k3) + prm.c * (x[j, 3:] - v)
        if i == prm.anchor:
            acc += -_force(p, prm.k, prm.k3) - prm.c * v
        acc += input_force(u, i, act)
        acc = acc / prm.m
        acc[2] -= prm.gravity
        vn = v + prm.dt * acc
        xn[i, :3] = p + prm.dt * vn
        xn[i, 3:] = vn
    return xn


def msd_linearize(xhat, uhat, row_ptr, col, act, prm):
    """Analytic A^{ij}_k, B^i_k, c^i_k at the nominal (xhat_k, uhat_k).

    Returns (prow, pcol, A [N][nnz][6][6], B [N][M][6][nu], c [N][M][6]) where
    (prow, pcol) is the 1-hop pattern (tilde N_i, ascending) and c follows the
    linearization offset of Sec. V-A: c = f(xhat, uhat) - sum_j A^{ij} xhat^j - B uhat.
    """
    N = uhat.shape[0]
    M = xhat.shape[1]
    nu = uhat.shape[1]
    prow, pcol = jacobian_pattern(row_ptr, col, M, 1)
    A = np.zeros((N, len(pcol), 6, 6))
    B = np.zeros((N, M, 6, nu))
    c = np.zeros((N, M, 6))
    dt, m = prm.dt, prm.m
    for k in range(N):
        x = xhat[k]
        fx = msd_step(x, uhat[k], row_ptr, col, act, prm)
        for i in range(M):
            p = x[i, :3]
            # d a^i / d x^j as 3x6 blocks
            dadx = {}
            diag_p = np.zeros((3, 3))
            diag_v = np.zeros((3, 3))
            for j in in_neighbours(row_ptr, col, i):
                Kj = _dforce(x[j, :3] - p, prm.k, prm.k3) / m
                dadx[j] = np.hstack([Kj, prm.c / m * np.eye(3)])
                diag_p -= Kj
                diag_v -= prm.c / m * np.eye(3)
            if i == prm.anchor:
                diag_p -= _dforce(p, prm.k, prm.k3) / m
                diag_v -= prm.c / m * np.eye(3)
            dadx[i] = np.hstack([diag_p, diag_v])
            for e in range(prow[i], prow[i + 1]):
                j = int(pcol[e])
                dv = dt * dadx[j]
                if j == i:
                    dv = dv + np.hstack([np.zeros((3, 3)), np.eye(3)])
                dp = dt * dv
                if j == i:
                    dp = dp + np.hstack([np.eye(3), np.zeros((3, 3))])
                A[k, e] = np.vstack([dp, dv])
            hit = np.nonzero(np.asarray(act) == i)[0]
            if hit.size:
                a = int(hit[0])
                B[k, i, 3:, 3 * a:3 * a + 3] = dt / m * np.eye(3)
                B[k, i, :3, 3 * a:3 * a + 3] = dt * dt / m * np.eye(3)
            lin = B[k, i] @ uhat[k]
            for e in range(prow[i], prow[i + 1]):
                lin = lin + A[k, e] @ x[int(pcol[e])]
            c[k, i] = fx[i] - lin
    return prow, pcol, A, B, c
