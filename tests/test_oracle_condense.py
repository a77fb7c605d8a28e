"""Pins of the oracle's condensing: dense definition vs the per-node recursion,
closed forms, the rollout identity, constraint identity and the uncondensed KKT."""
import numpy as np
import pytest

from oracle.condense import (condense_dense, condense_local, ocp_cost, rollout)
from oracle.graph import jacobian_pattern
from oracle.kkt import solve_uncondensed
from paper_2602_17601_amd import workloads as wl


def _random_lti_blocks(rng, M, hops, L, N, nu, scale=0.3, time_varying=True):
    rp, col = wl.chain_csr(M, hops)
    prow, pcol = jacobian_pattern(rp, col, M, L)
    nnz = len(pcol)
    if time_varying:
        A = rng.normal(0, scale, size=(N, nnz, 6, 6))
        B = rng.normal(size=(N, M, 6, nu))
        c = rng.normal(size=(N, M, 6))
    else:
        A = np.broadcast_to(rng.normal(0, scale, size=(nnz, 6, 6)), (N, nnz, 6, 6)).copy()
        B = np.broadcast_to(rng.normal(size=(M, 6, nu)), (N, M, 6, nu)).copy()
        c = np.broadcast_to(rng.normal(size=(M, 6)), (N, M, 6)).copy()
    return prow, pcol, A, B, c


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("full_Q", [False, True])
def test_dense_definition_equals_local_recursion(full_Q):
    rng = np.random.default_rng(1)
    M, N, nu = 7, 5, 4
    prow, pcol, A, B, c = _random_lti_blocks(rng, M, 2, 2, N, nu)
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu, full_Q=full_Q)
    rows = wl.random_rows(rng, M, N, 9)
    d = condense_dense(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, rows)
    l = condense_local(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, rows)
    for key in ("H", "g", "Ct", "dt"):
        assert _rel(l[key], d[key]) < 1e-12, key
    nx = 6 * M
    for k in range(N + 1):
        np.testing.assert_allclose(l["S"][k].reshape(nx, -1), d["Gu"][k * nx:(k + 1) * nx], atol=1e-9)
        np.testing.assert_allclose(l["Gx"][k].reshape(-1), d["Gx"][k * nx:(k + 1) * nx], atol=1e-9)


def test_lti_closed_form_prediction_matrices():
    """Constant A, B, c: block (k, j) of Gamma_u is A^{k-1-j} B and
    Gamma_x_k = A^k x0 + sum_{j<k} A^{k-1-j} c (matrix powers)."""
    rng = np.random.default_rng(2)
    M, N, nu = 5, 6, 3
    prow, pcol, A, B, c = _random_lti_blocks(rng, M, 1, 1, N, nu, time_varying=False)
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu)
    l = condense_local(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, wl.no_rows())
    nx = 6 * M
    Ad = np.zeros((nx, nx))
    for i in range(M):
        for e in range(prow[i], prow[i + 1]):
            Ad[6 * i:6 * i + 6, 6 * pcol[e]:6 * pcol[e] + 6] = A[0, e]
    Bd = B[0].reshape(nx, nu)
    cd = c[0].reshape(nx)
    mp = np.linalg.matrix_power
    for k in range(N + 1):
        Sk = l["S"][k].reshape(nx, N * nu)
        for j in range(N):
            blk = Sk[:, j * nu:(j + 1) * nu]
            ref = mp(Ad, k - 1 - j) @ Bd if j < k else np.zeros((nx, nu))
            np.testing.assert_allclose(blk, ref, atol=1e-10)
        gx = mp(Ad, k) @ x0.reshape(-1) + sum((mp(Ad, k - 1 - j) @ cd for j in range(k)), np.zeros(nx))
        np.testing.assert_allclose(l["Gx"][k].reshape(-1), gx, atol=1e-10)


def test_horizon_one_matches_the_written_out_case():
    """N = 1: Gamma_u^i = [0; B^i_0], Gamma_x^i = [x0^i; sum_j A^{ij}_0 x0^j + c^i_0],
    so H = sum_i B^i' Q^i_1 B^i + R_0 and g = sum_i B^i' (Q^i_1 Gx^i_1 + q^i_1) + r_0."""
    rng = np.random.default_rng(3)
    M, N, nu = 6, 1, 4
    prow, pcol, A, B, c = _random_lti_blocks(rng, M, 2, 1, N, nu)
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu, full_Q=True)
    l = condense_local(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, wl.no_rows())
    H = cost.R[0].copy()
    g = cost.r[0].copy()
    for i in range(M):
        gx1 = c[0, i] + sum(A[0, e] @ x0[pcol[e]] for e in range(prow[i], prow[i + 1]))
        H += B[0, i].T @ cost.Q[1, i] @ B[0, i]
        g += B[0, i].T @ (cost.Q[1, i] @ gx1 + cost.q[1, i])
    np.testing.assert_allclose(l["H"], H, atol=1e-12)
    np.testing.assert_allclose(l["g"], g, atol=1e-12)


def test_edgeless_graph_decouples_into_textbook_single_node_condensing():
    """With no edges each node is an independent 6-state system; H is R plus the
    sum of the single-node (M = 1) condensed Hessians."""
    rng = np.random.default_rng(4)
    M, N, nu = 4, 4, 2
    prow = np.arange(M + 1, dtype=np.int32)
    pcol = np.arange(M, dtype=np.int32)
    A = rng.normal(0, 0.4, size=(N, M, 6, 6))
    B = rng.normal(size=(N, M, 6, nu))
    c = rng.normal(size=(N, M, 6))
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu)
    full = condense_dense(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, wl.no_rows())
    H = np.zeros((N * nu, N * nu))
    g = np.zeros(N * nu)
    for k in range(N):
        H[k * nu:(k + 1) * nu, k * nu:(k + 1) * nu] += cost.R[k]
        g[k * nu:(k + 1) * nu] += cost.r[k]
    one = np.array([0, 1], np.int32)
    zeroR = np.zeros_like(cost.R)
    zeror = np.zeros_like(cost.r)
    for i in range(M):
        sub = condense_dense(A[:, i:i + 1], B[:, i:i + 1], c[:, i:i + 1], one, np.array([0], np.int32),
                             x0[i:i + 1], cost.Q[:, i:i + 1], cost.q[:, i:i + 1], zeroR, zeror, wl.no_rows())
        H += sub["H"]
        g += sub["g"]
    np.testing.assert_allclose(full["H"], H, atol=1e-10)
    np.testing.assert_allclose(full["g"], g, atol=1e-10)


def test_rollout_identity_cost_and_constraint_rows():
    """For any u: the simulated states equal S_k u + Gx_k, the OCP cost equals
    1/2 u'Hu + g'u + const, and C x^i_k(u) - d = Ct u - dt for every state row."""
    rng = np.random.default_rng(5)
    M, N, nu = 6, 5, 3
    prow, pcol, A, B, c = _random_lti_blocks(rng, M, 2, 2, N, nu)
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu, full_Q=True)
    rows = wl.random_rows(rng, M, N, 7)
    l = condense_local(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, rows)
    consts = []
    for trial in range(3):
        u = rng.normal(size=N * nu)
        x = rollout(A, B, c, prow, pcol, x0, u)
        for k in range(N + 1):
            np.testing.assert_allclose(x[k], l["S"][k] @ u + l["Gx"][k], atol=1e-9)
        J = ocp_cost(x, u, cost.Q, cost.q, cost.R, cost.r)
        consts.append(J - (0.5 * u @ l["H"] @ u + l["g"] @ u))
        lhs = np.array([rows.C[t] @ x[rows.stage[t], rows.node[t]] - rows.d[t] for t in range(rows.n)])
        np.testing.assert_allclose(lhs, l["Ct"] @ u - l["dt"], atol=1e-9)
    assert np.ptp(consts) < 1e-8 * max(1.0, abs(consts[0]))


def test_hessian_symmetric_and_dominates_input_weight():
    rng = np.random.default_rng(6)
    M, N, nu = 5, 4, 3
    prow, pcol, A, B, c = _random_lti_blocks(rng, M, 1, 1, N, nu)
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu)
    l = condense_local(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, wl.no_rows())
    H = l["H"]
    assert np.abs(H - H.T).max() < 1e-12 * np.abs(H).max()
    Rb = np.zeros_like(H)
    for k in range(N):
        Rb[k * nu:(k + 1) * nu, k * nu:(k + 1) * nu] = cost.R[k]
    assert np.linalg.eigvalsh(H - Rb).min() > -1e-10 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() >= np.linalg.eigvalsh(Rb).min() - 1e-10


def test_node_relabelling_invariance():
    rng = np.random.default_rng(7)
    M, N, nu = 6, 4, 2
    prow, pcol, A, B, c = _random_lti_blocks(rng, M, 2, 1, N, nu)
    x0 = rng.normal(size=(M, 6))
    cost = wl.random_costs(rng, M, N, nu)
    base = condense_local(A, B, c, prow, pcol, x0, cost.Q, cost.q, cost.R, cost.r, wl.no_rows())
    perm = rng.permutation(M)
    inv = np.argsort(perm)
    # new row p holds old row inv[p]; its blocks point to new labels perm[j]
    prow2 = np.zeros(M + 1, np.int32)
    pcol2, eidx = [], []
    for p in range(M):
        i = inv[p]
        ent = sorted((perm[pcol[e]], e) for e in range(prow[i], prow[i + 1]))
        pcol2 += [a for a, _ in ent]
        eidx += [e for _, e in ent]
        prow2[p + 1] = len(pcol2)
    A2 = A[:, eidx]
    out = condense_local(A2, B[:, inv], c[:, inv], prow2, np.asarray(pcol2, np.int32), x0[inv],
                         cost.Q[:, inv], cost.q[:, inv], cost.R, cost.r, wl.no_rows())
    np.testing.assert_allclose(out["H"], base["H"], atol=1e-10)
    np.testing.assert_allclose(out["g"], base["g"], atol=1e-10)


def test_uncondensed_kkt_matches_condensed_unconstrained_minimizer():
    P = wl.msd10_fp64()
    from oracle.msd import msd_linearize
    prow, pcol, A, B, c = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    cst = P.costs
    l = condense_local(A, B, c, prow, pcol, P.x0, cst.Q, cst.q, cst.R, cst.r, wl.no_rows())
    x, u, _ = solve_uncondensed(A, B, c, prow, pcol, P.x0, cst.Q, cst.q, cst.R, cst.r)
    u_cond = np.linalg.solve(l["H"], -l["g"])
    assert _rel(u.reshape(-1), u_cond) < 1e-9
    assert x.shape == (P.N + 1, P.M, 6)
