"""The learned-surrogate pipeline end to end (Sec. V-A "Dataset Generation" and
"Training", Algorithm 1's outer loop in Sec. V-C): trajectories of the nonlinear
spring-damper chain from the simulator kernel, the GNN trained on them with the
library's reverse-mode loss gradient and Adam, then the closed loop run twice on
the same plant, once with the trained GNN's Jacobians and once with the analytic
spring-damper Jacobians.  Every step of the method runs in the library
(gnmpc_msd_simulate, gnmpc_gnn_loss_grad, gnmpc_adam_step, gnmpc_linearize,
gnmpc_rti_step); this module only draws mini-batches, moves tensors and forms
the reported error norms.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import gnmpc as gn
from . import workloads as wl
from .train import PatienceScheduler


def gnn_unflat(theta: np.ndarray, like: wl.GNNWeights) -> wl.GNNWeights:
    """GNN weights from the flat packing of gnmpc.gnn_flat, shaped like `like`."""
    theta = np.asarray(theta, np.float64).reshape(-1)
    pos = 0

    def take(shape):
        nonlocal pos
        n = int(np.prod(shape))
        out = theta[pos:pos + n].reshape(shape).copy()
        pos += n
        return out

    W_enc, b_enc = take(like.W_enc.shape), take(like.b_enc.shape)
    W_edge, b_edge, W_node, b_node = [], [], [], []
    for l in range(like.L):
        W_edge.append(take(like.W_edge[l].shape))
        b_edge.append(take(like.b_edge[l].shape))
        W_node.append(take(like.W_node[l].shape))
        b_node.append(take(like.b_node[l].shape))
    W_dec, b_dec = take(like.W_dec.shape), take(like.b_dec.shape)
    if pos != theta.size:
        raise ValueError(f"gnn_unflat: {theta.size} parameters for a model of {pos}")
    return wl.GNNWeights(like.Hd, like.L, W_enc, b_enc, W_edge, b_edge, W_node, b_node, W_dec, b_dec, like.dt)


@dataclass
class SurrogateConfig:
    M: int = 1000            # nodes of the chain
    B: int = 4096            # trajectories
    T: int = 100             # steps per trajectory
    B_test: int = 256        # trajectories held out for evaluation
    Hd: int = 128
    L: int = 3
    batch: int = 20          # samples per Adam step
    steps: int = 2000        # Adam steps
    epoch_steps: int = 100   # steps between scheduler updates (and progress lines)
    lr: float = 1e-3
    lam: float = 1e-8
    N: int = 20              # MPC horizon
    loop_steps: int = 500    # closed-loop iterations per controller
    umax: float = 1.0
    seed: int = 5
    weight_seed: int = 11
    gnn_dtype: int = gn.BF16


def _dense_blocks(A, prow, pcol, M):
    """[N][6M][6M] from block-sparse A [N][nnz][6][6] (pattern prow, pcol)."""
    N = A.shape[0]
    rows = torch.repeat_interleave(torch.arange(M, device=A.device),
                                   torch.as_tensor(np.diff(prow), device=A.device).long())
    cols = torch.as_tensor(pcol, device=A.device).long()
    D = torch.zeros(M, M, N, 6, 6, dtype=A.dtype, device=A.device)
    D[rows, cols] = A.permute(1, 0, 2, 3)
    return D.permute(2, 0, 3, 1, 4).reshape(N, 6 * M, 6 * M)


def run(cfg: SurrogateConfig, log=print) -> dict:
    dev = "cuda"
    t0 = time.time()
    f32 = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev).contiguous()
    # ---- data set: B trajectories of T steps from the simulator kernel
    sim = wl.simulator_batch(cfg.B, cfg.T, M=cfg.M, seed=cfg.seed)
    M, nu = cfg.M, sim.nu
    splan = gn.Plan(M, nu, 1, 0, gn.F32)
    splan.graph_set(sim.row_ptr, sim.col, 1)
    splan.model_set_msd(sim.msd, sim.act)
    U = f32(sim.u)
    X = torch.empty(cfg.B, cfg.T + 1, M, 6, device=dev)
    splan.msd_simulate(f32(sim.x0), U, X)
    torch.cuda.synchronize()
    data_s = time.time() - t0
    log(f"[surrogate] data set: {cfg.B} x {cfg.T} steps of the {M}-node chain ({data_s:.1f} s)")
    B_train = cfg.B - cfg.B_test

    def samples(b_idx, t_idx):
        x = X[b_idx, t_idx].contiguous()
        xn = X[b_idx, t_idx + 1].contiguous()
        u = U[b_idx, t_idx].contiguous()
        return x, u, xn

    # ---- training: Adam on mini-batches of (x_t, u_t, x_{t+1}) from the training trajectories
    W0 = wl.gnn_weights(cfg.weight_seed, cfg.Hd, cfg.L, dt=sim.msd.dt)
    S = cfg.batch
    tplan = gn.Plan(M, nu, S, 0, gn.F32)
    tplan.graph_set(sim.row_ptr, sim.col, cfg.L)
    tplan.model_set_gnn(W0, sim.act, dtype=cfg.gnn_dtype)
    n, wb = tplan.gnn_train_sizes()
    theta = f32(gn.gnn_flat(W0))
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    grad, m, v = (torch.zeros(n, device=dev) for _ in range(3))
    loss = torch.empty(1, device=dev)
    O = [1.0] * 6
    gen = np.random.default_rng(cfg.seed + 1)
    # held-out samples (every trajectory of the test set at seeded steps)
    nt_eval = max(S, (min(cfg.B_test * cfg.T, 1024) // S) * S)
    eb = torch.as_tensor(B_train + gen.integers(0, cfg.B_test, nt_eval), device=dev)
    et = torch.as_tensor(gen.integers(0, cfg.T, nt_eval), device=dev)

    def eval_rmse(th):
        tot = 0.0
        for i in range(0, nt_eval, S):
            x, u, xn = samples(eb[i:i + S], et[i:i + S])
            tplan.gnn_loss_grad(th, x, u, xn, O, 0.0, ws, loss, grad)
            tot += float(loss) * S
        return float(np.sqrt(tot / nt_eval / (M * 6)))

    # spread of the one-step increment, the scale the RMSE is read against
    x, u, xn = samples(eb, et)
    incr_rms = float(torch.sqrt(((xn - x) ** 2).mean()))
    rmse0 = eval_rmse(theta)
    sched = PatienceScheduler(cfg.lr, factor=0.5, patience=3, threshold=1e-3)
    history = []
    ep_loss = 0.0
    t_train = time.time()
    for step in range(1, cfg.steps + 1):
        b_idx = torch.as_tensor(gen.integers(0, B_train, S), device=dev)
        t_idx = torch.as_tensor(gen.integers(0, cfg.T, S), device=dev)
        x, u, xn = samples(b_idx, t_idx)
        tplan.gnn_loss_grad(theta, x, u, xn, O, cfg.lam, ws, loss, grad)
        gn.adam_step(theta, grad, m, v, step, sched.lr)
        ep_loss += float(loss)
        if step % cfg.epoch_steps == 0:
            ep_loss /= cfg.epoch_steps
            history.append(ep_loss)
            sched.step(ep_loss)
            log(f"[surrogate] step {step}: mean training loss {ep_loss:.4e}, lr {sched.lr:.2e}")
            ep_loss = 0.0
    torch.cuda.synchronize()
    train_s = time.time() - t_train
    rmse1 = eval_rmse(theta)
    W1 = gnn_unflat(theta.double().cpu().numpy(), W0)
    log(f"[surrogate] one-step RMSE on held-out samples: {rmse0:.4e} -> {rmse1:.4e} (increment rms {incr_rms:.4e})")

    # ---- Jacobian error at held-out states: GNN (trained and initial) against the analytic model
    N = cfg.N
    jb = B_train  # first held-out trajectory, stages 0..N-1
    xh = X[jb, :N + 1].contiguous()
    uh = U[jb, :N].contiguous()

    def jac(model, W=None):
        p = gn.Plan(M, nu, N, 0, gn.F32)
        if model == "gnn":
            p.graph_set(sim.row_ptr, sim.col, cfg.L)
            p.model_set_gnn(W, sim.act, dtype=cfg.gnn_dtype)
        else:
            p.graph_set(sim.row_ptr, sim.col, 1)
            p.model_set_msd(sim.msd, sim.act)
        A = torch.empty(N, p.nnz, 6, 6, device=dev)
        Bm = torch.empty(N, M, 6, nu, device=dev)
        c = torch.empty(N, M, 6, device=dev)
        p.linearize(xh, uh, A, Bm, c)
        prow, pcol = p.graph_pattern()
        return _dense_blocks(A, prow, pcol, M), Bm

    Am, Bmsd = jac("msd")
    eye = torch.eye(6 * M, device=dev)
    nA = float(torch.linalg.norm(Am - eye))
    nB = float(torch.linalg.norm(Bmsd))
    jac_err = {}
    for name, W in (("initial", W0), ("trained", W1)):
        Ag, Bg = jac("gnn", W)
        jac_err[name] = {"A_minus_I": float(torch.linalg.norm(Ag - Am)) / nA,
                         "B": float(torch.linalg.norm(Bg - Bmsd)) / nB}
        del Ag, Bg
    del Am
    log(f"[surrogate] Jacobian error (rel. Frobenius, {N} held-out stages): {jac_err}")

    # ---- closed loop: the same plant, GNN Jacobians against analytic Jacobians
    P = wl.make_problem("surrogate_loop", M=M, hops=sim.hops, N=N, n_act=len(sim.act), model="msd", seed=3,
                        msd=sim.msd, x0_sigma=0.02, umax=cfg.umax)
    assert np.array_equal(P.act, sim.act)
    x_start = X[jb, 0].clone()

    def loop(model):
        n_u = N * nu
        plan = gn.Plan(M, nu, N, 0, gn.F32)
        if model == "gnn":
            plan.graph_set(sim.row_ptr, sim.col, cfg.L)
            plan.model_set_gnn(W1, sim.act, dtype=cfg.gnn_dtype)
        else:
            plan.graph_set(sim.row_ptr, sim.col, 1)
            plan.model_set_msd(sim.msd, sim.act)
        e = lambda *sh: torch.empty(*sh, device=dev)
        b = dict(xhat=x_start.expand(N + 1, M, 6).contiguous(), uhat=torch.zeros(N, nu, device=dev),
                 x0=x_start.clone(), Q=f32(P.costs.Q), q=f32(P.costs.q), R=f32(P.costs.R), r=f32(P.costs.r),
                 lb=f32(P.lb), ub=f32(P.ub), A=e(N, plan.nnz, 6, 6), B=e(N, M, 6, nu), c=e(N, M, 6),
                 H=e(n_u, n_u), g=e(n_u), u=e(n_u), info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8,
                                                                      device=dev))
        xpred, Xs = e(N + 1, M, 6), e(1, 2, M, 6)
        traj = e(cfg.loop_steps + 1, M, 6)
        uapp = e(cfg.loop_steps, nu)
        traj[0] = b["x0"]
        settings = gn.default_admm_settings()
        unsolved = 0
        check = max(1, cfg.loop_steps // 5)   # QP status read (and progress line) every `check` iterations
        torch.cuda.synchronize()
        t1 = time.time()
        for it in range(cfg.loop_steps):
            gn.rti_step(plan, b, xpred, settings=settings)
            uapp[it] = b["u"][:nu]
            splan.msd_simulate(b["x0"].view(1, M, 6), b["u"][:nu].view(1, 1, nu), Xs)
            b["x0"].copy_(Xs[0, 1])
            traj[it + 1] = b["x0"]
            if (it + 1) % check == 0:
                unsolved += int(gn.qp_info(b["info"]).status != gn.QP_SOLVED)
                log(f"[surrogate] {model} loop: {it + 1} iterations")
        torch.cuda.synchronize()
        ms = (time.time() - t1) * 1e3 / cfg.loop_steps
        return traj, uapp, ms, unsolved

    tr_g, u_g, ms_g, uns_g = loop("gnn")
    tr_m, u_m, ms_m, uns_m = loop("msd")
    Qd = torch.as_tensor(np.asarray(P.costs.Q)[0].reshape(M, 6), dtype=torch.float32, device=dev)
    Rd = float(np.asarray(P.costs.R).reshape(-1)[0])

    def cost(tr, ua):
        return float((tr[1:] ** 2 * Qd).sum() + Rd * (ua ** 2).sum())

    out = {
        "workload": (f"{cfg.B} x {cfg.T}-step trajectories of the {M}-node nonlinear chain (cubic springs "
                     f"k3={sim.msd.k3}, gravity {sim.msd.gravity}); GNN Hd={cfg.Hd} L={cfg.L} trained "
                     f"{cfg.steps} Adam steps x {S} samples; {cfg.loop_steps}-step closed loop, N={N}, |u|<={cfg.umax}"),
        "data_s": data_s,
        "train_s": train_s,
        "train_ms_per_step": train_s * 1e3 / cfg.steps,
        "loss_history": history,
        "one_step_rmse": {"initial": rmse0, "trained": rmse1, "increment_rms": incr_rms,
                          "held_out_samples": nt_eval},
        "jacobian_rel_error": jac_err,
        "closed_loop": {
            "gnn": {"ms_per_iteration": ms_g, "cost": cost(tr_g, u_g), "qp_unsolved_at_checks": uns_g,
                    "checks": cfg.loop_steps // max(1, cfg.loop_steps // 5)},
            "analytic": {"ms_per_iteration": ms_m, "cost": cost(tr_m, u_m), "qp_unsolved_at_checks": uns_m,
                         "checks": cfg.loop_steps // max(1, cfg.loop_steps // 5)},
            "state_rel_diff": float(torch.linalg.norm(tr_g - tr_m) / torch.linalg.norm(tr_m)),
            "input_rel_diff": float(torch.linalg.norm(u_g - u_m) / max(float(torch.linalg.norm(u_m)), 1e-30)),
            "finite": bool(torch.isfinite(tr_g).all() and torch.isfinite(tr_m).all()),
        },
        "total_s": time.time() - t0,
    }
    return out
