"""Pins of the oracle's training objective and optimizer: the gradient of every
parameter block against central differences of the loss, the regularizer alone
where the model fits the data exactly, and Adam's first step and convergence on
a quadratic."""
import copy

import numpy as np

from oracle.gnn import gnn_forward
from oracle.train import adam_step, loss_grad, params
from paper_2602_17601_amd import workloads as wl


def _data(seed=3, M=9, S=3, Hd=16, L=2):
    P = wl.make_problem("train", M=M, hops=2, N=S, n_act=2, model="gnn", seed=seed, Hd=Hd, L=L, x0_sigma=0.3,
                        walk=0.05, bias_scale=0.2)
    rng = np.random.default_rng(seed)
    x = P.xhat[:S]
    u = P.uhat
    xn = x + 0.05 * rng.normal(size=x.shape)
    return P, x, u, xn


def test_loss_gradient_matches_central_differences_in_every_block():
    P, x, u, xn = _data()
    W = P.gnn
    O = np.array([1.0, 2.0, 0.5, 0.1, 0.3, 0.7])
    lam = 1e-3
    loss, G = loss_grad(W, x, u, xn, P.row_ptr, P.col, P.act, O, lam)
    rng = np.random.default_rng(0)
    eps = 1e-6
    for bi, (p, gp) in enumerate(zip(params(W), params(G))):
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in p.shape)
            pp, pm = copy.deepcopy(W), copy.deepcopy(W)
            params(pp)[bi][idx] += eps
            params(pm)[bi][idx] -= eps
            lp = loss_grad(pp, x, u, xn, P.row_ptr, P.col, P.act, O, lam)[0]
            lm = loss_grad(pm, x, u, xn, P.row_ptr, P.col, P.act, O, lam)[0]
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - gp[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (bi, idx, fd, gp[idx])


def test_exact_fit_leaves_only_the_regularizer():
    P, x, u, _ = _data(seed=4)
    W = P.gnn
    xn = np.stack([gnn_forward(x[t], u[t], W, P.row_ptr, P.col, P.act) for t in range(x.shape[0])])
    lam = 0.01
    loss, G = loss_grad(W, x, u, xn, P.row_ptr, P.col, P.act, np.ones(6), lam)
    assert abs(loss - lam * sum(float(np.sum(p * p)) for p in params(W))) < 1e-12
    for p, gp in zip(params(W), params(G)):
        np.testing.assert_allclose(gp, 2 * lam * p, rtol=0, atol=1e-12)


def test_adam_first_step_is_lr_times_the_gradient_sign_and_it_minimizes_a_quadratic():
    g = np.array([3.0, -0.2, 1e-3])
    th, m, v = adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=1e-12)
    np.testing.assert_allclose(th, -0.1 * np.sign(g), rtol=1e-8)  # eps / |g| of the smallest entry
    th, m, v = np.array([10.0, -4.0]), np.zeros(2), np.zeros(2)
    target = np.array([3.0, 1.0])
    for step in range(1, 3001):
        th, m, v = adam_step(th, 2 * (th - target), m, v, step, lr=0.05)
    np.testing.assert_allclose(th, target, atol=1e-3)
