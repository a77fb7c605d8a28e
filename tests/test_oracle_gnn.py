"""Pins of the oracle's GNN model and its per-node forward-mode linearization."""
import numpy as np
import pytest

from oracle.gnn import gnn_forward, gnn_linearize
from oracle.graph import ball
from paper_2602_17601_amd import workloads as wl


def _small(M=7, hops=2, Hd=12, L=2, seed=5, bias_scale=0.0):
    rp, col = wl.chain_csr(M, hops)
    act = wl.actuated_nodes(M, 2)
    W = wl.gnn_weights(seed, Hd, L, bias_scale=bias_scale)
    rng = np.random.default_rng(seed + 100)
    x = rng.normal(0, 0.5, size=(M, 6))
    u = rng.uniform(-1, 1, size=6)
    return rp, col, act, W, x, u


def _dense_jac(prow, pcol, A, M):
    D = np.zeros((6 * M, 6 * M))
    for i in range(M):
        for e in range(prow[i], prow[i + 1]):
            D[6 * i:6 * i + 6, 6 * pcol[e]:6 * pcol[e] + 6] = A[e]
    return D


def test_forward_mode_matches_central_differences():
    rp, col, act, W, x, u = _small()
    M = x.shape[0]
    prow, pcol, A, B, c, f = gnn_linearize(x[None], u[None], W, rp, col, act)
    J = _dense_jac(prow, pcol, A[0], M)
    h = 1e-6
    xv = x.reshape(-1)
    Jfd = np.zeros_like(J)
    for a in range(6 * M):
        xp = xv.copy(); xp[a] += h
        xm = xv.copy(); xm[a] -= h
        Jfd[:, a] = (gnn_forward(xp.reshape(M, 6), u, W, rp, col, act)
                     - gnn_forward(xm.reshape(M, 6), u, W, rp, col, act)).reshape(-1) / (2 * h)
    np.testing.assert_allclose(J, Jfd, atol=1e-8)
    Bfd = np.zeros((6 * M, 6))
    for a in range(6):
        up = u.copy(); up[a] += h
        um = u.copy(); um[a] -= h
        Bfd[:, a] = (gnn_forward(x, up, W, rp, col, act)
                     - gnn_forward(x, um, W, rp, col, act)).reshape(-1) / (2 * h)
    np.testing.assert_allclose(B[0].reshape(6 * M, 6), Bfd, atol=1e-8)
    # the per-node value equals the whole-graph forward
    np.testing.assert_allclose(f[0], gnn_forward(x, u, W, rp, col, act), atol=1e-14)
    # something is actually nonzero off the diagonal at L hops
    assert np.abs(J - np.eye(6 * M)).max() > 1e-4


def test_identity_activation_matches_kronecker_closed_form():
    """With every activation the identity the model is affine, and its state
    Jacobian is a product of per-layer Kronecker operators:
      encoder  E  = I_M (x) W_enc[:, :6]
      layer l  T_l = I_M (x) W_n1 + D (x) (W_n2 (W_a + W_b)) - Adj (x) (W_n2 W_b)
      decoder  O  = I_M (x) W_dec
    with W_e = [W_a W_b], W_n = [W_n1 W_n2], D = diag(in-degree), Adj[i, j] = 1 for j in N_i;
    then dv+ = [0 I] + dt O[3:6] T_L ... T_1 E and dp+ = [I 0] + dt dv+."""
    M, Hd, L = 6, 10, 2
    rp, col, act, W, x, u = _small(M=M, Hd=Hd, L=L, seed=9)
    prow, pcol, A, B, c, f = gnn_linearize(x[None], u[None], W, rp, col, act, activation="identity")
    J = _dense_jac(prow, pcol, A[0], M)
    Adj = np.zeros((M, M))
    for i in range(M):
        for j in col[rp[i]:rp[i + 1]]:
            Adj[i, j] = 1.0
    D = np.diag(Adj.sum(1))
    I = np.eye(M)
    Z = np.kron(I, W.W_enc[:, :6])
    for l in range(L):
        Wa, Wb = W.W_edge[l][:, :Hd], W.W_edge[l][:, Hd:]
        Wn1, Wn2 = W.W_node[l][:, :Hd], W.W_node[l][:, Hd:]
        T = np.kron(I, Wn1) + np.kron(D, Wn2 @ (Wa + Wb)) - np.kron(Adj, Wn2 @ Wb)
        Z = T @ Z
    O = np.kron(I, W.W_dec) @ Z                      # [6M][6M], rows (node, channel)
    sel_v = np.kron(I, np.hstack([np.zeros((3, 3)), np.eye(3)]))
    sel_p = np.kron(I, np.hstack([np.eye(3), np.zeros((3, 3))]))
    dO_v = O.reshape(M, 6, 6 * M)[:, 3:6, :].reshape(3 * M, 6 * M)
    dv = sel_v + W.dt * dO_v
    dp = sel_p + W.dt * dv
    ref = np.stack([dp.reshape(M, 3, 6 * M), dv.reshape(M, 3, 6 * M)], axis=1)
    ref = ref.transpose(0, 1, 2, 3).reshape(M, 6, 6 * M).reshape(6 * M, 6 * M)
    np.testing.assert_allclose(J, ref, atol=1e-12)


def test_locality_outside_receptive_field_is_exact_zero():
    rp, col, act, W, x, u = _small(M=12, L=2)
    M = 12
    base = gnn_forward(x, u, W, rp, col, act)
    for i in (0, 5, 11):
        inside = set(ball(rp, col, i, W.L))
        for j in range(M):
            if j in inside:
                continue
            x2 = x.copy()
            x2[j] += 0.37
            assert np.array_equal(gnn_forward(x2, u, W, rp, col, act)[i], base[i])


def test_permutation_equivariance():
    """Relabelling the nodes (and the graph and actuators with them) permutes
    the next states and conjugates the Jacobian blocks."""
    rp, col, act, W, x, u = _small(M=8, L=2)
    M = 8
    perm = np.random.default_rng(3).permutation(M)        # new label of old node
    inv = np.argsort(perm)
    rows = [[] for _ in range(M)]
    for i in range(M):
        for j in col[rp[i]:rp[i + 1]]:
            rows[perm[i]].append(perm[j])
    rp2 = np.zeros(M + 1, np.int32)
    col2 = []
    for i in range(M):
        col2 += sorted(rows[i])
        rp2[i + 1] = len(col2)
    col2 = np.asarray(col2, np.int32)
    # actuator order must keep u's layout: actuator a is old node act[a], new label perm[act[a]]
    act2 = perm[act]
    x2 = x[inv]
    f1 = gnn_forward(x, u, W, rp, col, act)
    f2 = gnn_forward(x2, u, W, rp2, col2, act2)
    np.testing.assert_allclose(f2[perm], f1, atol=1e-13)


def test_bf16_rounding_is_round_to_nearest_even():
    vals = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -3.140625, 1e-3])
    r = wl.bf16_round(vals)
    # 1 + 2^-8 is exactly halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert r[1] == 1.0
    # 1 + 1.5*2^-8 rounds up to 1 + 2^-7
    assert r[2] == 1.0078125
    assert r[3] == 1.0078125
    assert r[4] == -3.140625
    assert abs(r[5] - 1e-3) / 1e-3 < 2 ** -8


def _encoder_pre(x, u, W, act, j):
    """Encoder pre-activation of node j (the test builds its input from the model's definition)."""
    from oracle.gnn import node_input
    return W.W_enc @ node_input(x, u, j, act) + W.b_enc


@pytest.mark.parametrize("j,L", [(0, 2), (6, 2), (4, 3)])
def test_kink_margin_finds_a_zero_encoder_preactivation_in_exactly_the_downstream_fields(j, L):
    """Shift one encoder bias so that node j's pre-activation of feature 3 is
    zero: the margin must vanish for exactly the nodes whose L-hop receptive
    field contains j, and stay clear of zero elsewhere."""
    from oracle.gnn import gnn_kink_margin
    rp, col, act, W, x, u = _small(M=11, hops=1, Hd=12, L=L, seed=21)
    W.b_enc = W.b_enc.copy()
    W.b_enc[3] -= _encoder_pre(x, u, W, act, j)[3]
    mg = gnn_kink_margin(x, u, W, rp, col, act)
    for i in range(11):
        if j in ball(rp, col, i, L):
            assert mg[i] < 1e-14, (i, mg[i])
        else:
            assert mg[i] > 1e-6, (i, mg[i])


def test_kink_margin_finds_a_zero_edge_preactivation_of_the_first_round():
    """Zero the round-0 pre-activation of edge (r <- s): with L = 2 it is in
    the field of every node within one hop downstream of r, and no other."""
    from oracle.gnn import gnn_kink_margin
    rp, col, act, W, x, u = _small(M=10, hops=2, Hd=8, L=2, seed=4)
    M, r, s, f = 10, 5, 3, 2
    h = np.stack([np.maximum(_encoder_pre(x, u, W, act, n), 0) for n in range(M)])
    ze = W.W_edge[0] @ np.concatenate([h[r], h[r] - h[s]]) + W.b_edge[0]
    W.b_edge = [b.copy() for b in W.b_edge]
    W.b_edge[0][f] -= ze[f]
    mg = gnn_kink_margin(x, u, W, rp, col, act)
    for i in range(M):
        if r in ball(rp, col, i, 1):
            assert mg[i] < 1e-14, (i, mg[i])
        else:
            assert mg[i] > 1e-6, (i, mg[i])


def test_kink_margin_is_scale_invariant_without_biases():
    """With zero biases the model is positively homogeneous: scaling x and u by
    a > 0 scales every pre-activation and every term by a, so no margin moves."""
    from oracle.gnn import gnn_kink_margin
    rp, col, act, W, x, u = _small(M=9, L=2, seed=7)
    m1 = gnn_kink_margin(x, u, W, rp, col, act)
    m2 = gnn_kink_margin(3.5 * x, 3.5 * u, W, rp, col, act)
    np.testing.assert_allclose(m1, m2, rtol=1e-12)
    assert np.all(m1 > 0) and np.all(np.isfinite(m1))


# ----------------------------------------------------------------------------- reverse mode

@pytest.mark.parametrize("M,hops,Hd,L,bias", [(7, 2, 12, 2, 0.0), (9, 1, 8, 3, 0.3), (6, 2, 10, 1, 0.5)])
def test_reverse_mode_is_the_transpose_of_the_forward_mode_jacobian(M, hops, Hd, L, bias):
    """gnn_vjp (reverse mode, whole graph) against the dense transpose of the
    per-node forward-mode Jacobian (a separate algorithm): gx = A' g, gu = B' g."""
    from oracle.gnn import gnn_vjp
    rp, col, act, W, x, u = _small(M, hops, Hd, L, seed=M + L, bias_scale=bias)
    prow, pcol, A, B, c, f = gnn_linearize(x[None], u[None], W, rp, col, act)
    g = np.random.default_rng(3).normal(size=(M, 6))
    gx, gu = gnn_vjp(x, u, W, rp, col, act, g)
    D = _dense_jac(prow, pcol, A[0], M)
    np.testing.assert_allclose(gx.reshape(-1), D.T @ g.reshape(-1), rtol=0, atol=1e-12)
    np.testing.assert_allclose(gu, B[0].reshape(6 * M, -1).T @ g.reshape(-1), rtol=0, atol=1e-12)


def test_reverse_mode_matches_central_differences_of_g_dot_f():
    """d/dt g . f(x + t dx, u + t du) at t = 0 equals gx . dx + gu . du."""
    from oracle.gnn import gnn_vjp
    rp, col, act, W, x, u = _small(8, 2, 12, 2, seed=21, bias_scale=0.2)
    rng = np.random.default_rng(4)
    g = rng.normal(size=x.shape)
    gx, gu = gnn_vjp(x, u, W, rp, col, act, g)
    for _ in range(3):
        dx, du = rng.normal(size=x.shape), rng.normal(size=u.shape)
        h = 1e-6
        fp = gnn_forward(x + h * dx, u + h * du, W, rp, col, act)
        fm = gnn_forward(x - h * dx, u - h * du, W, rp, col, act)
        fd = np.sum(g * (fp - fm)) / (2 * h)
        assert abs(fd - (np.sum(gx * dx) + gu @ du)) < 1e-7 * max(1.0, abs(fd))


def test_reverse_mode_of_the_affine_model_is_the_weight_product_transposed():
    """With identity activations the model is affine, so g . f is linear in g and
    the reverse mode must give exactly the transposed forward-mode products."""
    from oracle.gnn import gnn_vjp
    rp, col, act, W, x, u = _small(7, 2, 6, 2, seed=8)
    prow, pcol, A, B, c, f = gnn_linearize(x[None], u[None], W, rp, col, act, activation="identity")
    D = _dense_jac(prow, pcol, A[0], 7)
    for s in range(2):
        g = np.random.default_rng(10 + s).normal(size=(7, 6))
        gx, gu = gnn_vjp(x, u, W, rp, col, act, g, activation="identity")
        np.testing.assert_allclose(gx.reshape(-1), D.T @ g.reshape(-1), rtol=0, atol=1e-12)
        np.testing.assert_allclose(gu, B[0].reshape(42, -1).T @ g.reshape(-1), rtol=0, atol=1e-12)
