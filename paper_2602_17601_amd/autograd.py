"""The plan's one-step model x_{k+1} = f(x_k, u_k) (Sec. V-A) as a differentiable
torch op over all N stages.  The forward pass is gnmpc_linearize, which also forms
the block Jacobians A_k, B_k at (x_k, u_k) with the forward-mode kernel; the
backward pass applies gnmpc_vjp to those saved blocks, and ``dynamics_jvp`` applies
gnmpc_jvp.  Argument marshalling only: every product runs in the library."""
from __future__ import annotations

import torch

from . import gnmpc as gn


def _blocks(plan, x, u):
    N, M, nu = plan.N, plan.M, plan.nu
    kw = dict(device=x.device, dtype=x.dtype)
    A = torch.empty(N, plan.nnz, 6, 6, **kw)
    B = torch.empty(N, M, 6, nu, **kw)
    c = torch.empty(N, M, 6, **kw)
    f = torch.empty(N, M, 6, **kw)
    plan.linearize(x.detach().contiguous(), u.detach().contiguous(), A, B, c, f)
    return A, B, f


class Dynamics(torch.autograd.Function):
    """f(x_k, u_k) for k < N: x [N+1][M][6] (stage N is not read), u [N][nu] -> [N][M][6].

    The gradient with respect to x[N] is zero; ReLU takes the subgradient 0 at 0."""

    @staticmethod
    def forward(ctx, plan, x, u):
        A, B, f = _blocks(plan, x, u)
        ctx.plan = plan
        ctx.save_for_backward(A, B)
        return f

    @staticmethod
    def backward(ctx, grad):
        A, B = ctx.saved_tensors
        plan = ctx.plan
        N, M, nu = plan.N, plan.M, plan.nu
        gx = torch.zeros(N + 1, M, 6, device=grad.device, dtype=grad.dtype)
        gu = torch.empty(N, nu, device=grad.device, dtype=grad.dtype)
        plan.vjp(A, B, grad.contiguous(), gx[:N], gu)
        return None, gx, gu


def dynamics_jvp(plan: "gn.Plan", x, u, dx, du):
    """(f(x_k, u_k), A_k dx[k] + B_k du[k]) for k < N; dx [N][M][6], du [N][nu]."""
    A, B, f = _blocks(plan, x, u)
    t = torch.empty_like(f)
    plan.jvp(A, B, dx.contiguous(), du.contiguous(), t)
    return f, t
