"""Training objective of the GNN dynamics model and its optimizer (oracle; test
infrastructure only), Sec. V-A "Training":

  L(theta) = 1/S sum_t || x_{t+1} - F_theta(x_t, u_t) ||_O^2 + lambda ||theta||^2,

||r||_O^2 = r' O r summed over the nodes with O diagonal (one weight per state
component), theta every weight and bias of the model of ``oracle.gnn``.
``loss_grad`` returns L and dL/dtheta by reverse mode: the forward pass keeps
each layer's input and derivative mask, the cotangent of F runs back through the
decoder, the node and edge MLPs of every round and the encoder, and every
layer's weight gradient is the sum over nodes (edges) of cotangent times input.
``adam_step`` is the update of Kingma and Ba (Adam, 2015) with bias correction.
"""
from __future__ import annotations

import copy

import numpy as np

from .gnn import _edges, node_input


def _forward(x, u, W, row_ptr, col, act):
    """F(x, u) with the values the reverse pass needs."""
    M = x.shape[0]
    inp = np.stack([node_input(x, u, i, act) for i in range(M)])
    z0 = inp @ W.W_enc.T + W.b_enc
    h = np.maximum(z0, 0.0)
    tape = {"inp": inp, "z0": z0, "rounds": []}
    recv, send = _edges(row_ptr, col)
    for l in range(W.L):
        e_in = np.concatenate([h[recv], h[recv] - h[send]], axis=1)
        ze = e_in @ W.W_edge[l].T + W.b_edge[l]
        m = np.maximum(ze, 0.0)
        agg = np.zeros_like(h)
        np.add.at(agg, recv, m)
        n_in = np.concatenate([h, agg], axis=1)
        zn = n_in @ W.W_node[l].T + W.b_node[l]
        tape["rounds"].append({"e_in": e_in, "ze": ze, "n_in": n_in, "zn": zn})
        h = np.maximum(zn, 0.0)
    o = h @ W.W_dec.T + W.b_dec
    vn = x[:, 3:] + W.dt * o[:, 3:6]
    pn = x[:, :3] + W.dt * vn
    tape["hL"] = h
    return np.concatenate([pn, vn], axis=1), tape


def _zeros_like(W):
    G = copy.deepcopy(W)
    G.W_enc, G.b_enc = np.zeros_like(W.W_enc), np.zeros_like(W.b_enc)
    G.W_edge = [np.zeros_like(a) for a in W.W_edge]
    G.b_edge = [np.zeros_like(a) for a in W.b_edge]
    G.W_node = [np.zeros_like(a) for a in W.W_node]
    G.b_node = [np.zeros_like(a) for a in W.b_node]
    G.W_dec, G.b_dec = np.zeros_like(W.W_dec), np.zeros_like(W.b_dec)
    return G


def params(W):
    """Every parameter array of W, in the library's packing order."""
    out = [W.W_enc, W.b_enc]
    for l in range(W.L):
        out += [W.W_edge[l], W.b_edge[l], W.W_node[l], W.b_node[l]]
    return out + [W.W_dec, W.b_dec]


def loss_grad(W, x, u, x_next, row_ptr, col, act, O, lam):
    """L and dL/dtheta (a GNNWeights of gradients) over the S samples
    x [S][M][6], u [S][nu], x_next [S][M][6]; O [6] the diagonal weights."""
    S = x.shape[0]
    O = np.asarray(O, dtype=np.float64)
    G = _zeros_like(W)
    recv, send = _edges(row_ptr, col)
    loss = 0.0
    for t in range(S):
        F, tape = _forward(np.asarray(x[t], np.float64), np.asarray(u[t], np.float64), W, row_ptr, col, act)
        r = F - x_next[t]
        loss += float(np.sum(O * r * r)) / S
        gF = 2.0 * O * r / S                     # dL/dF
        gv = gF[:, 3:] + W.dt * gF[:, :3]        # p+ = p + dt v+ feeds the velocity too
        go = np.zeros((F.shape[0], 6))
        go[:, 3:6] = W.dt * gv                   # v+ = v + dt o[3:6]
        G.W_dec += go.T @ tape["hL"]
        G.b_dec += go.sum(axis=0)
        gh = go @ W.W_dec
        for l in range(W.L - 1, -1, -1):
            rd = tape["rounds"][l]
            gzn = gh * (rd["zn"] > 0)
            G.W_node[l] += gzn.T @ rd["n_in"]
            G.b_node[l] += gzn.sum(axis=0)
            gin = gzn @ W.W_node[l]
            Hd = W.Hd
            gh = gin[:, :Hd].copy()
            gagg = gin[:, Hd:]
            gze = gagg[recv] * (rd["ze"] > 0)   # each edge's message feeds its receiver's sum
            G.W_edge[l] += gze.T @ rd["e_in"]
            G.b_edge[l] += gze.sum(axis=0)
            ge = gze @ W.W_edge[l]               # [E][2 Hd]: cotangents of h_i and of h_i - h_j
            np.add.at(gh, recv, ge[:, :Hd] + ge[:, Hd:])
            np.add.at(gh, send, -ge[:, Hd:])
        gz0 = gh * (tape["z0"] > 0)
        G.W_enc += gz0.T @ tape["inp"]
        G.b_enc += gz0.sum(axis=0)
    for p, gp in zip(params(W), params(G)):
        loss += lam * float(np.sum(p * p))
        gp += 2.0 * lam * p
    return loss, G


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the flat parameter vector (step counts from 1); returns
    (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
