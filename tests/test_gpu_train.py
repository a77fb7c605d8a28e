"""GNN training on the GPU: the loss and its gradient (gnmpc_gnn_loss_grad)
against the oracle's reverse mode, Adam (gnmpc_adam_step) against the oracle's
update, and a short training run on spring-damper simulator data (the loop of
paper_2602_17601_amd.train) that lowers the loss."""
import numpy as np
import pytest
import torch

from oracle.gnn import gnn_forward
from oracle.train import adam_step, loss_grad, params
from paper_2602_17601_amd import workloads as wl

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")
tr = pytest.importorskip("paper_2602_17601_amd.train")


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _plan(P, S):
    plan = gn.Plan(P.M, P.nu, S, 0, gn.F32)
    plan.graph_set(P.row_ptr, P.col, P.gnn.L)
    plan.model_set_gnn(P.gnn, P.act, dtype=gn.F32)
    return plan


def _min_margin(P, W, x, u):
    m = np.inf
    for t in range(x.shape[0]):
        _, mg = gnn_forward(x[t], u[t], W, P.row_ptr, P.col, P.act, margins=True)
        with np.errstate(invalid="ignore"):
            for v in [mg["enc"]] + list(mg["edge"]) + list(mg["node"]):
                m = min(m, float(np.nan_to_num(v, nan=np.inf).min()))
    return m


@pytest.mark.parametrize("M,L,Hd,S,bias", [(14, 2, 64, 4, 0.2), (11, 1, 192, 3, 0.3), (9, 3, 128, 2, 0.1)])
def test_loss_and_gradient_match_the_oracle(M, L, Hd, S, bias):
    """FP32 on the device against FP64 reverse mode on the FP32-rounded inputs, per
    parameter block within 1e-4 (where no pre-activation is within 2^-16 of its
    terms' scale of a ReLU kink; 1e-2 otherwise) and the loss within 1e-5."""
    P = wl.make_problem("train_g", M=M, hops=2, N=S, n_act=2, model="gnn", seed=M + Hd, Hd=Hd, L=L, x0_sigma=0.3,
                        walk=0.05, bias_scale=bias)
    r32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    x, u = r32(P.xhat[:S]), r32(P.uhat)
    xn = r32(x + 0.05 * np.random.default_rng(M).normal(size=x.shape))
    O = np.array([1.0, 1.0, 1.0, 0.1, 0.1, 0.1])
    lam = 1e-3
    theta64 = gn.gnn_flat(P.gnn)
    W = P.gnn.__class__(**{**P.gnn.__dict__})  # the same weights rounded to FP32 for the oracle
    W.W_enc, W.b_enc = r32(W.W_enc), r32(W.b_enc)
    W.W_edge, W.b_edge = [r32(a) for a in W.W_edge], [r32(a) for a in W.b_edge]
    W.W_node, W.b_node = [r32(a) for a in W.W_node], [r32(a) for a in W.b_node]
    W.W_dec, W.b_dec = r32(W.W_dec), r32(W.b_dec)
    plan = _plan(P, S)
    n, wb = plan.gnn_train_sizes()
    assert n == theta64.size
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    loss = torch.full((1,), float("nan"), device="cuda")
    grad = torch.full((n,), float("nan"), device="cuda")
    plan.gnn_loss_grad(_t(theta64), _t(x), _t(u), _t(xn), O, lam, ws, loss, grad)
    torch.cuda.synchronize()
    rl, G = loss_grad(W, x, u, xn, P.row_ptr, P.col, P.act, O, lam)
    g = grad.double().cpu().numpy()
    assert np.all(np.isfinite(g))
    assert abs(float(loss.item()) - rl) <= 1e-5 * abs(rl)
    tol = 1e-4 if _min_margin(P, W, x, u) > 2.0 ** -16 else 1e-2
    off = 0
    for bi, gp in enumerate(params(G)):
        k = gp.size
        assert _rel(g[off:off + k], gp.reshape(-1)) < tol, (bi, _rel(g[off:off + k], gp.reshape(-1)))
        off += k
    # repeatable bit for bit
    grad2 = torch.empty_like(grad)
    plan.gnn_loss_grad(_t(theta64), _t(x), _t(u), _t(xn), O, lam, ws, loss, grad2)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)


def test_adam_step_matches_the_oracle():
    rng = np.random.default_rng(1)
    n = 1000
    th = rng.normal(size=n)
    m, v = np.zeros(n), np.zeros(n)
    dth, dm, dv = _t(th), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    for step in range(1, 4):
        g = rng.normal(size=n)
        th, m, v = adam_step(th, np.asarray(g, np.float32).astype(np.float64), m, v, step, lr=1e-2)
        gn.adam_step(dth, _t(g), dm, dv, step, 1e-2)
    torch.cuda.synchronize()
    assert np.abs(dth.double().cpu().numpy() - th).max() < 1e-5


def test_training_on_simulator_data_lowers_the_loss():
    """A 20-node chain simulated for 16 trajectories x 8 steps; a GNN (Hd 64, L 2)
    trained with Adam on mini-batches of 32 samples for 30 epochs."""
    M, B, T, S = 20, 16, 8, 32
    sim = wl.simulator_batch(B, T, M=M, hops=2, n_act=2, seed=3, x0_sigma=0.05, step=0.1)
    splan = gn.Plan(M, sim.nu, 1, 0, gn.F32)
    splan.graph_set(sim.row_ptr, sim.col, 1)
    splan.model_set_msd(sim.msd, sim.act)
    X = torch.empty(B, T + 1, M, 6, device="cuda")
    splan.msd_simulate(_t(sim.x0), _t(sim.u), X)
    x = X[:, :T].reshape(B * T, M, 6)
    xn = X[:, 1:].reshape(B * T, M, 6)
    u = _t(sim.u).reshape(B * T, sim.nu)
    batches = [(x[i:i + S].contiguous(), u[i:i + S].contiguous(), xn[i:i + S].contiguous())
               for i in range(0, B * T, S)]
    W = wl.gnn_weights(7, 64, 2, dt=sim.msd.dt)
    plan = gn.Plan(M, sim.nu, S, 0, gn.F32)
    plan.graph_set(sim.row_ptr, sim.col, 2)
    plan.model_set_gnn(W, sim.act, dtype=gn.F32)
    theta = _t(gn.gnn_flat(W))
    hist = tr.train(plan, theta, batches, epochs=30, O=[1, 1, 1, 1, 1, 1], lam=1e-6, lr=1e-2)
    print("loss per epoch", [round(h, 8) for h in hist[::5]], hist[-1])
    assert all(np.isfinite(hist))
    assert hist[-1] < 0.7 * hist[0]
