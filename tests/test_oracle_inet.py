"""Pins of the oracle's interaction network (the paper's own model, Sec. V-A)
and its linearization: central differences of the forward model, and exactness
of the linearization where every ReLU is active (the model is then affine in
(x, u), so A x + B u + c reproduces f away from the linearization point)."""
import copy

import numpy as np

from oracle.inet import inet_forward, inet_linearize
from paper_2602_17601_amd import workloads as wl


def _fd_blocks(P, W, k, eps=1e-6):
    """Central differences of f at (xhat[k], uhat[k]): dF[i][j] [6][6] and dU[i] [6][nu]."""
    x, u = P.xhat[k].copy(), P.uhat[k].copy()
    M, nu = P.M, P.nu
    dF = np.zeros((M, M, 6, 6))
    dU = np.zeros((M, 6, nu))
    for j in range(M):
        for a in range(6):
            xp, xm = x.copy(), x.copy()
            xp[j, a] += eps
            xm[j, a] -= eps
            dF[:, j, :, a] = (inet_forward(xp, u, W, P.row_ptr, P.col) - inet_forward(xm, u, W, P.row_ptr, P.col)) / (2 * eps)
    for d in range(nu):
        up, um = u.copy(), u.copy()
        up[d] += eps
        um[d] -= eps
        dU[:, :, d] = (inet_forward(x, up, W, P.row_ptr, P.col) - inet_forward(x, um, W, P.row_ptr, P.col)) / (2 * eps)
    return dF, dU


def test_inet_linearization_matches_central_differences():
    P = wl.trunk_inet(N=3, seed=11, x0_sigma=0.3, walk=0.05)
    W = P.inet
    prow, pcol, A, B, c, f = inet_linearize(P.xhat, P.uhat, W, P.row_ptr, P.col)
    for k in range(P.N):
        np.testing.assert_allclose(f[k], inet_forward(P.xhat[k], P.uhat[k], W, P.row_ptr, P.col), rtol=0, atol=1e-14)
        dF, dU = _fd_blocks(P, W, k)
        for i in range(P.M):
            blocks = {int(pcol[e]): A[k, e] for e in range(prow[i], prow[i + 1])}
            for j in range(P.M):
                Aij = blocks.get(j, np.zeros((6, 6)))
                assert np.abs(Aij - dF[i, j]).max() <= 1e-6 * max(1.0, np.abs(dF[i, j]).max()), (k, i, j)
            assert np.abs(B[k, i] - dU[i]).max() <= 1e-6 * max(1.0, np.abs(dU[i]).max())


def test_inet_linearization_is_exact_where_every_relu_is_on():
    P = wl.trunk_inet(N=2, seed=12)
    W = copy.deepcopy(P.inet)
    # nonnegative weights and biases >= 1 keep every pre-activation positive for
    # small states and inputs: the model is then affine in (x, u)
    W.psi_W = [np.abs(w) for w in W.psi_W]
    W.phi_W = [np.abs(w) for w in W.phi_W]
    W.psi_b = [np.abs(b) + 1.0 for b in W.psi_b]
    W.phi_b = [np.abs(b) + 1.0 for b in W.phi_b]
    prow, pcol, A, B, c, f = inet_linearize(P.xhat, P.uhat, W, P.row_ptr, P.col)
    rng = np.random.default_rng(3)
    for k in range(P.N):
        x = P.xhat[k] + 0.05 * rng.normal(size=P.xhat[k].shape)
        u = P.uhat[k] + 0.05 * rng.normal(size=P.nu)
        ref = inet_forward(x, u, W, P.row_ptr, P.col)
        for i in range(P.M):
            lin = B[k, i] @ u + c[k, i]
            for e in range(prow[i], prow[i + 1]):
                lin = lin + A[k, e] @ x[int(pcol[e])]
            assert np.abs(lin - ref[i]).max() <= 1e-11 * max(1.0, np.abs(ref[i]).max()), (k, i)


def test_trunk_graph_has_two_neighbours_per_node():
    rp, col = wl.nearest_csr(4, 2)
    assert list(np.diff(rp)) == [2, 2, 2, 2]
    assert [list(col[rp[i]:rp[i + 1]]) for i in range(4)] == [[1, 2], [0, 2], [1, 3], [1, 2]]
