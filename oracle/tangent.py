"""Tangent maps of the linearized dynamics (oracle; test infrastructure only).

The linearization of Sec. V-A gives, per stage k, the block Jacobians
A_k = d f / d x (blocks A^{ij}_k on the pattern j in tilde N_i) and
B_k = d f / d u (blocks B^i_k) of the one-step model x_{k+1} = f(x_k, u_k).
Their forward- and reverse-mode products are

* jvp: t_k = A_k dx_k + B_k du_k  (the directional derivative of f),
* vjp: (A_k' g_k, B_k' g_k)       (the gradient of g_k . f).

Both are written here as their plain definitions: the blocks are placed in the
dense matrices of ``condense.dense_dynamics`` and multiplied.  Shapes: A
[N][nnz][6][6], B [N][M][6][nu], dx and g [N][M][6], du [N][nu].
"""
from __future__ import annotations

import numpy as np

from .condense import dense_dynamics


def jvp_blocks(A, B, prow, pcol, dx, du):
    """t [N][M][6] with t_k = A_k dx_k + B_k du_k."""
    N, M = B.shape[0], B.shape[1]
    Ad, Bd, _ = dense_dynamics(A, B, np.zeros((N, M, 6)), prow, pcol, M)
    t = np.stack([Ad[k] @ dx[k].reshape(-1) + Bd[k] @ du[k] for k in range(N)])
    return t.reshape(N, M, 6)


def vjp_blocks(A, B, prow, pcol, g):
    """(gx [N][M][6], gu [N][nu]) with gx_k = A_k' g_k and gu_k = B_k' g_k."""
    N, M = B.shape[0], B.shape[1]
    Ad, Bd, _ = dense_dynamics(A, B, np.zeros((N, M, 6)), prow, pcol, M)
    gx = np.stack([Ad[k].T @ g[k].reshape(-1) for k in range(N)]).reshape(N, M, 6)
    gu = np.stack([Bd[k].T @ g[k].reshape(-1) for k in range(N)])
    return gx, gu
