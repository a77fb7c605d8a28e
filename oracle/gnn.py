"""GNN dynamics model and its per-node linearization (oracle; test
infrastructure only).

Model (Sec. V-A eq. forward_dynamics; message passing as Sec. III-A eq. 1,
sum aggregation, ReLU MLPs, edge feature built from the relative state):
  h0_i      = act(W_enc [x^i; P^i u] + b_enc)             P^i u: node i's force, 0 if not actuated
  m_ij      = act(W_e^l [h_i; h_i - h_j] + b_e^l)         j in N_i (senders of edges j -> i)
  h_i       <- act(W_n^l [h_i; sum_{j in N_i} m_ij] + b_n^l)   for l = 0..L-1
  o_i       = W_dec h_i + b_dec                            o_i[3:6] is the velocity increment / dt
  v+        = v + dt o_i[3:6],   p+ = p + dt v+            (semi-implicit Euler)

Linearization (Sec. V-A "Linearization" and eq. linearized_dynamics): each node's
local dynamics are differentiated independently by forward-mode automatic
differentiation (value, tangent) pairs seeded on the states of every node of
its L-hop receptive set and on u.  ReLU uses the subgradient 0 at 0 (the
derivative mask is z > 0).  The offset is c = f(xhat,uhat) - sum_j A^{ij} xhat^j - B uhat.

``activation='identity'`` replaces every ReLU by the identity; it exists only
so the tests can compare against a closed-form affine model.

``gnn_vjp`` is reverse mode through the same network: the gradient of g . f,
pinned in the tests against the forward-mode Jacobian above (a separate
algorithm) and against central differences.

``gnn_kink_margin`` reports, per node, how close the model is to a ReLU kink
anywhere in the node's receptive field: the smallest ratio |z| / scale(z) over
every pre-activation z that f^i depends on, scale(z) being the sum of the
absolute values of the terms of z (|W| |operand| summed, plus |b|).  A
computation that carries the activations with relative rounding error eps can
take a different ReLU decision only where this ratio is of order eps.
"""
from __future__ import annotations

import numpy as np

from .graph import ball, in_neighbours, jacobian_pattern


def _act(z, activation):
    if activation == "identity":
        return z, np.ones_like(z)
    mask = (z > 0).astype(np.float64)
    return z * mask, mask


def node_input(x, u, i, act):
    """[x^i; P^i u] with P^i selecting node i's 3 force inputs (zero if unactuated)."""
    f = np.zeros(3)
    hit = np.nonzero(np.asarray(act) == i)[0]
    if hit.size:
        a = int(hit[0])
        f = np.asarray(u[3 * a:3 * a + 3], dtype=np.float64)
    return np.concatenate([x[i], f])


def _edges(row_ptr, col):
    """Receiver and sender of every edge, in CSR order (edge e runs col[e] -> its row)."""
    recv = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    return recv, np.asarray(col, dtype=np.int64)


def gnn_forward(x, u, W, row_ptr, col, act, activation="relu", margins=False):
    """One step x -> x+ for every node; x is [M][6], returns [M][6].

    With ``margins=True`` also returns the margin |z| / scale(z) of every
    pre-activation: a dict with 'enc' [M][Hd] and, per round l, 'edge'[l]
    [E][Hd] (CSR edge order) and 'node'[l] [M][Hd].
    """
    M = x.shape[0]
    inp = np.stack([node_input(x, u, i, act) for i in range(M)])
    z = inp @ W.W_enc.T + W.b_enc
    out = {"enc": np.abs(z) / (np.abs(inp) @ np.abs(W.W_enc).T + np.abs(W.b_enc)), "edge": [], "node": []}
    h, _ = _act(z, activation)
    recv, send = _edges(row_ptr, col)
    for l in range(W.L):
        e_in = np.concatenate([h[recv], h[recv] - h[send]], axis=1)   # [h_i; h_i - h_j] per edge
        ze = e_in @ W.W_edge[l].T + W.b_edge[l]
        m, _ = _act(ze, activation)
        agg = np.zeros_like(h)
        np.add.at(agg, recv, m)                                         # sum over j in N_i
        # terms of z_e: W1 h_i + W2 h_i - W2 h_j + b, each taken in absolute value
        W1, W2 = np.abs(W.W_edge[l][:, :W.Hd]), np.abs(W.W_edge[l][:, W.Hd:])
        se = np.abs(h[recv]) @ (W1 + W2).T + np.abs(h[send]) @ W2.T + np.abs(W.b_edge[l])
        out["edge"].append(np.abs(ze) / se)
        n_in = np.concatenate([h, agg], axis=1)
        zn = n_in @ W.W_node[l].T + W.b_node[l]
        out["node"].append(np.abs(zn) / (np.abs(n_in) @ np.abs(W.W_node[l]).T + np.abs(W.b_node[l])))
        h, _ = _act(zn, activation)
    o = h @ W.W_dec.T + W.b_dec
    vn = x[:, 3:] + W.dt * o[:, 3:6]
    pn = x[:, :3] + W.dt * vn
    f = np.concatenate([pn, vn], axis=1)
    return (f, out) if margins else f


def gnn_vjp(x, u, W, row_ptr, col, act, g, activation="relu"):
    """Reverse mode of one step: the gradient of g . f(x, u) (Sec. V-A's model).

    x [M][6], u [nu], g [M][6] -> (gx [M][6], gu [nu]).  The forward pass keeps
    each layer's derivative masks; the cotangents then run back through the
    decoder and integrator, the L message-passing rounds in reverse order and
    the encoder, each written out from the layer's definition.
    """
    M, nu, Hd = x.shape[0], u.shape[0], W.Hd
    inp = np.stack([node_input(x, u, i, act) for i in range(M)])
    h, m_enc = _act(inp @ W.W_enc.T + W.b_enc, activation)
    recv, send = _edges(row_ptr, col)
    m_edge, m_node = [], []
    for l in range(W.L):
        e_in = np.concatenate([h[recv], h[recv] - h[send]], axis=1)
        m, de = _act(e_in @ W.W_edge[l].T + W.b_edge[l], activation)
        agg = np.zeros_like(h)
        np.add.at(agg, recv, m)
        h, dn = _act(np.concatenate([h, agg], axis=1) @ W.W_node[l].T + W.b_node[l], activation)
        m_edge.append(de)
        m_node.append(dn)
    # integrator: p+ = p + dt v+, v+ = v + dt o[3:6]
    vb = g[:, 3:] + W.dt * g[:, :3]               # cotangent of v+
    gx = np.concatenate([g[:, :3], vb], axis=1)   # direct dependence on p and v
    ob = np.zeros((M, 6))
    ob[:, 3:6] = W.dt * vb                        # cotangent of o
    hb = ob @ W.W_dec                             # of h^L
    for l in reversed(range(W.L)):
        nb = (m_node[l] * hb) @ W.W_node[l]       # of [h; agg] at the node update
        hb_new, ab = nb[:, :Hd].copy(), nb[:, Hd:]
        eb = (m_edge[l] * ab[recv]) @ W.W_edge[l]  # of [h_i; h_i - h_j] per edge (every edge feeds agg_i)
        np.add.at(hb_new, recv, eb[:, :Hd] + eb[:, Hd:])
        np.add.at(hb_new, send, -eb[:, Hd:])
        hb = hb_new
    ib = (m_enc * hb) @ W.W_enc                   # of the node inputs [x^i; P^i u]
    gx = gx + ib[:, :6]
    gu = np.zeros(nu)
    for a, node in enumerate(act):
        gu[3 * a:3 * a + 3] += ib[int(node), 6:9]
    return gx, gu


def gnn_vjp_stages(xhat, uhat, W, row_ptr, col, act, g, activation="relu"):
    """gnn_vjp at every stage k < N: (gx [N][M][6], gu [N][nu])."""
    N = uhat.shape[0]
    out = [gnn_vjp(xhat[k], uhat[k], W, row_ptr, col, act, g[k], activation) for k in range(N)]
    return np.stack([o[0] for o in out]), np.stack([o[1] for o in out])


def gnn_kink_margin(x, u, W, row_ptr, col, act, nodes=None):
    """Smallest pre-activation margin in the receptive field of each node.

    f^i depends on the encoder of every node within L hops of i and, in round
    l (0-based), on the node update of every node within L-1-l hops of i and
    on the edges into those nodes.  Returns an array over ``nodes`` (all by
    default).  A zero scale (every term zero) counts as margin +inf.
    """
    M = x.shape[0]
    _, mg = gnn_forward(x, u, W, row_ptr, col, act, margins=True)
    recv, _ = _edges(row_ptr, col)
    with np.errstate(invalid="ignore"):
        enc = np.nan_to_num(mg["enc"].min(axis=1), nan=np.inf)
        edge = [np.nan_to_num(e.min(axis=1), nan=np.inf) for e in mg["edge"]]
        node = [np.nan_to_num(n.min(axis=1), nan=np.inf) for n in mg["node"]]
    res = []
    for i in (range(M) if nodes is None else nodes):
        best = enc[ball(row_ptr, col, i, W.L)].min()
        for l in range(W.L):
            near = ball(row_ptr, col, i, W.L - 1 - l)
            best = min(best, node[l][near].min())
            sel = np.isin(recv, near)
            if sel.any():
                best = min(best, edge[l][sel].min())
        res.append(best)
    return np.asarray(res)


def gnn_linearize_node(x, u, W, row_ptr, col, act, i, activation="relu"):
    """Forward-mode derivative of f^i on node i's receptive subgraph.

    Returns (f_i [6], S (sorted receptive nodes), J [6][6|S| + nu]) where the
    columns of J are the seeds x^{S[0]}, x^{S[1]}, ..., then u.
    """
    L = W.L
    nu = u.shape[0]
    S = ball(row_ptr, col, i, L)
    T = 6 * len(S) + nu
    pos = {j: p for p, j in enumerate(S)}
    du = np.zeros((nu, T))
    du[:, 6 * len(S):] = np.eye(nu)

    def seed_x(j):
        t = np.zeros((6, T))
        t[:, 6 * pos[j]:6 * pos[j] + 6] = np.eye(6)
        return t

    # encoder on every node of the receptive set
    h, dh = {}, {}
    for j in S:
        inp = node_input(x, u, j, act)
        dinp = np.vstack([seed_x(j), np.zeros((3, T))])
        hit = np.nonzero(np.asarray(act) == j)[0]
        if hit.size:
            a = int(hit[0])
            dinp[6:9] = du[3 * a:3 * a + 3]
        z = W.W_enc @ inp + W.b_enc
        hv, mask = _act(z, activation)
        h[j], dh[j] = hv, mask[:, None] * (W.W_enc @ dinp)
    # message-passing rounds: after round l only nodes within L-1-l hops are needed
    for l in range(L):
        keep = ball(row_ptr, col, i, L - 1 - l)
        nh, ndh = {}, {}
        for n in keep:
            agg = np.zeros(W.Hd)
            dagg = np.zeros((W.Hd, T))
            for j in in_neighbours(row_ptr, col, n):
                e = np.concatenate([h[n], h[n] - h[j]])
                de = np.vstack([dh[n], dh[n] - dh[j]])
                m, mask = _act(W.W_edge[l] @ e + W.b_edge[l], activation)
                agg += m
                dagg += mask[:, None] * (W.W_edge[l] @ de)
            z = W.W_node[l] @ np.concatenate([h[n], agg]) + W.b_node[l]
            hv, mask = _act(z, activation)
            nh[n] = hv
            ndh[n] = mask[:, None] * (W.W_node[l] @ np.vstack([dh[n], dagg]))
        h, dh = nh, ndh
    o = W.W_dec @ h[i] + W.b_dec
    do = W.W_dec @ dh[i]
    dx_i = seed_x(i)
    vn = x[i, 3:] + W.dt * o[3:6]
    dvn = dx_i[3:] + W.dt * do[3:6]
    pn = x[i, :3] + W.dt * vn
    dpn = dx_i[:3] + W.dt * dvn
    return np.concatenate([pn, vn]), S, np.vstack([dpn, dvn])


def gnn_linearize(xhat, uhat, W, row_ptr, col, act, stages=None, nodes=None,
                  activation="relu"):
    """A^{ij}_k (L-hop pattern, ascending), B^i_k, c^i_k and f^i_k.

    Only the requested (stage, node) pairs are computed (all by default); the
    remaining entries are left as NaN so that accidental use is visible.
    Returns (prow, pcol, A [N][nnz][6][6], B [N][M][6][nu], c [N][M][6], f [N][M][6]).
    """
    N, nu = uhat.shape
    M = xhat.shape[1]
    prow, pcol = jacobian_pattern(row_ptr, col, M, W.L)
    A = np.full((N, len(pcol), 6, 6), np.nan)
    B = np.full((N, M, 6, nu), np.nan)
    c = np.full((N, M, 6), np.nan)
    f = np.full((N, M, 6), np.nan)
    for k in (range(N) if stages is None else stages):
        for i in (range(M) if nodes is None else nodes):
            fi, S, J = gnn_linearize_node(xhat[k], uhat[k], W, row_ptr, col, act, i, activation)
            assert list(pcol[prow[i]:prow[i + 1]]) == S
            lin = J[:, 6 * len(S):] @ uhat[k]
            for p, j in enumerate(S):
                A[k, prow[i] + p] = J[:, 6 * p:6 * p + 6]
                lin = lin + J[:, 6 * p:6 * p + 6] @ xhat[k, j]
            B[k, i] = J[:, 6 * len(S):]
            c[k, i] = fi - lin
            f[k, i] = fi
    return prow, pcol, A, B, c, f
