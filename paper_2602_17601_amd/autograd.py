"""The plan's one-step model x_{k+1} = f(x_k, u_k) (Sec. V-A) as a differentiable
torch op over all N stages.  For a GNN model the forward pass is gnmpc_gnn_forward
and the backward pass gnmpc_gnn_vjp, reverse mode through the network's layers
(the forward pass is recomputed at the saved point for its ReLU masks; no
Jacobian blocks are formed).  For the mass-spring-damper model the forward pass is
gnmpc_linearize, whose analytic blocks A_k, B_k are saved and multiplied by
gnmpc_vjp.  ``dynamics_jvp`` applies gnmpc_jvp to the linearization's blocks.
Argument marshalling only: every product runs in the library."""
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
        ctx.plan = plan
        xd, ud = x.detach().contiguous(), u.detach().contiguous()
        if getattr(plan, "model", None) == "gnn":
            f = torch.empty(plan.N, plan.M, 6, device=x.device, dtype=x.dtype)
            plan.gnn_forward(xd, ud, f)
            ctx.save_for_backward(xd, ud)
            ctx.reverse = True
            return f
        A, B, f = _blocks(plan, x, u)
        ctx.save_for_backward(A, B)
        ctx.reverse = False
        return f

    @staticmethod
    def backward(ctx, grad):
        plan = ctx.plan
        N, M, nu = plan.N, plan.M, plan.nu
        gx = torch.zeros(N + 1, M, 6, device=grad.device, dtype=grad.dtype)
        gu = torch.empty(N, nu, device=grad.device, dtype=grad.dtype)
        if ctx.reverse:
            xd, ud = ctx.saved_tensors
            gxs = torch.empty(N, M, 6, device=grad.device, dtype=grad.dtype)
            plan.gnn_vjp(xd, ud, grad.contiguous(), gxs, gu)
            gx[:N] = gxs
        else:
            A, B = ctx.saved_tensors
            plan.vjp(A, B, grad.contiguous(), gx[:N], gu)
        return None, gx, gu


def dynamics_jvp(plan: "gn.Plan", x, u, dx, du):
    """(f(x_k, u_k), A_k dx[k] + B_k du[k]) for k < N; dx [N][M][6], du [N][nu]."""
    A, B, f = _blocks(plan, x, u)
    t = torch.empty_like(f)
    plan.jvp(A, B, dx.contiguous(), du.contiguous(), t)
    return f, t
