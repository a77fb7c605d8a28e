"""Training loop of the GNN dynamics model (Sec. V-A "Training"): mini-batches of
(x_t, u_t, x_{t+1}) samples, the library's loss and gradient
(gnmpc_gnn_loss_grad), Adam (gnmpc_adam_step) and a learning rate reduced on a
plateau of the monitored loss ("a learning rate scheduler based on patience").
Every array stays on the device; the host reads one loss value per epoch.
"""
from __future__ import annotations

import torch

from . import gnmpc as gn


class PatienceScheduler:
    """Multiply the learning rate by `factor` once the monitored loss has not improved
    on its best value by more than `threshold` (relative) for `patience` epochs;
    never below `min_lr`."""

    def __init__(self, lr, factor=0.5, patience=5, threshold=1e-4, min_lr=1e-6):
        if not (0 < factor < 1) or patience < 0 or lr <= 0:
            raise ValueError("factor in (0, 1), patience >= 0, lr > 0")
        self.lr, self.factor, self.patience, self.threshold, self.min_lr = lr, factor, patience, threshold, min_lr
        self.best = float("inf")
        self.bad = 0

    def step(self, loss):
        if loss < self.best * (1.0 - self.threshold):
            self.best = loss
            self.bad = 0
        else:
            self.bad += 1
            if self.bad > self.patience:
                self.lr = max(self.min_lr, self.lr * self.factor)
                self.bad = 0
        return self.lr


def train(plan, theta, batches, epochs, O, lam, lr=1e-3, scheduler=None, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam on the plan's GNN from parameters `theta` (FP32 device, gnmpc.gnn_flat
    packing; updated in place) over `batches`, a list of (x [N][M][6], u [N][nu],
    x_next [N][M][6]) device tensors with N the plan's horizon.  Returns the mean
    loss of every epoch (the loss of each batch before its update)."""
    n, wb = plan.gnn_train_sizes()
    dev = theta.device
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    grad = torch.empty(n, dtype=torch.float32, device=dev)
    m = torch.zeros(n, dtype=torch.float32, device=dev)
    v = torch.zeros(n, dtype=torch.float32, device=dev)
    losses = torch.empty(len(batches), dtype=torch.float32, device=dev)
    sched = scheduler or PatienceScheduler(lr)
    history, step = [], 0
    for _ in range(epochs):
        for bi, (x, u, xn) in enumerate(batches):
            plan.gnn_loss_grad(theta, x, u, xn, O, lam, ws, losses[bi:bi + 1], grad)
            step += 1
            gn.adam_step(theta, grad, m, v, step, sched.lr, beta1, beta2, eps)
        epoch_loss = float(losses.mean())
        history.append(epoch_loss)
        sched.step(epoch_loss)
    return history
