"""The paper's own dynamics model, an interaction network (Sec. V-A eq.
forward_dynamics), and its linearization (Sec. V-A "Linearization", eq.
linearized_dynamics) in FP64.  Oracle; test infrastructure only.

Node i's next state: with e^{ij} = x^i - x^j and a^i = sum_{j in N_i} psi(e^{ij}),
    v^i+ = v^i + phi([x^i; a^i; u]),   p^i+ = p^i + dt v^i+,
psi and phi being MLPs with a ReLU after every layer but the last, u the global
input.  The linearization is forward mode: a tangent matrix is carried through
every layer (z = W h + b gives dz = W dh; a ReLU keeps the rows whose
pre-activation is > 0, the subgradient 0 at the kink).
"""
from __future__ import annotations

import numpy as np

from oracle.graph import in_neighbours, jacobian_pattern


def _mlp(Ws, bs, h, T=None):
    """Forward pass of an MLP; with T (d input / d seed) also the output's tangents."""
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = W @ h + b
        if T is not None:
            T = W @ T
        if l < len(Ws) - 1:
            on = z > 0
            h = np.where(on, z, 0.0)
            if T is not None:
                T = T * on[:, None]
        else:
            h = z
    return h, T


def inet_forward(x, u, W, row_ptr, col):
    """f(x, u) for all nodes: x [M][6], u [nu] -> [M][6]."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    M = x.shape[0]
    out = np.empty((M, 6))
    for i in range(M):
        a = np.zeros(W.d_m)
        for j in in_neighbours(row_ptr, col, i):
            a += _mlp(W.psi_W, W.psi_b, x[i] - x[j])[0]
        dv = _mlp(W.phi_W, W.phi_b, np.concatenate([x[i], a, u]))[0]
        vn = x[i, 3:] + dv
        out[i, :3] = x[i, :3] + W.dt * vn
        out[i, 3:] = vn
    return out


def inet_linearize(xhat, uhat, W, row_ptr, col):
    """A^{ij}_k (1-hop pattern, ascending), B^i_k, c^i_k at (xhat_k, uhat_k).

    Returns (prow, pcol, A [N][nnz][6][6], B [N][M][6][nu], c [N][M][6], f [N][M][6])."""
    uhat = np.asarray(uhat, dtype=np.float64)
    N, nu = uhat.shape
    M = np.asarray(xhat).shape[1]
    prow, pcol = jacobian_pattern(row_ptr, col, M, 1)
    A = np.zeros((N, len(pcol), 6, 6))
    B = np.zeros((N, M, 6, nu))
    c = np.zeros((N, M, 6))
    f = np.zeros((N, M, 6))
    dm = W.d_m
    for k in range(N):
        x = np.asarray(xhat[k], dtype=np.float64)
        u = uhat[k]
        for i in range(M):
            # d v+ / d x^j for every j in the pattern row, and d v+ / d u
            nbrs = list(in_neighbours(row_ptr, col, i))
            a = np.zeros(dm)
            Jpsi = {}
            for j in nbrs:
                m, T = _mlp(W.psi_W, W.psi_b, x[i] - x[j], np.eye(6))
                a += m
                Jpsi[j] = T                     # d psi / d e^{ij}, [d_m][6]
            h = np.concatenate([x[i], a, u])
            dv, J = _mlp(W.phi_W, W.phi_b, h, np.eye(h.shape[0]))
            Jx, Ja, Ju = J[:, :6], J[:, 6:6 + dm], J[:, 6 + dm:]
            dvdx = {i: np.hstack([np.zeros((3, 3)), np.eye(3)]) + Jx}
            for j in nbrs:
                dvdx[i] = dvdx[i] + Ja @ Jpsi[j]    # e^{ij} grows with x^i
                dvdx[j] = dvdx.get(j, np.zeros((3, 6))) - Ja @ Jpsi[j]
            vn = x[i, 3:] + dv
            f[k, i, :3] = x[i, :3] + W.dt * vn
            f[k, i, 3:] = vn
            for e in range(prow[i], prow[i + 1]):
                j = int(pcol[e])
                dv_j = dvdx.get(j, np.zeros((3, 6)))
                dp_j = W.dt * dv_j + (np.hstack([np.eye(3), np.zeros((3, 3))]) if j == i else 0.0)
                A[k, e, :3] = dp_j
                A[k, e, 3:] = dv_j
            B[k, i, :3] = W.dt * Ju
            B[k, i, 3:] = Ju
            lin = B[k, i] @ u
            for e in range(prow[i], prow[i + 1]):
                lin = lin + A[k, e] @ x[int(pcol[e])]
            c[k, i] = f[k, i] - lin
    return prow, pcol, A, B, c, f
