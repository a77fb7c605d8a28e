"""Tangent maps of the linearized model on the GPU (gnmpc_jvp / gnmpc_vjp and the
autograd op): against the oracle's analytic spring-damper blocks in FP64,
against the oracle's products of the device's own GNN blocks, against central
differences of the device's GNN forward pass, and the adjoint identity."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle.msd import msd_linearize
from oracle.tangent import jvp_blocks, vjp_blocks
from paper_2602_17601_amd import workloads as wl

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")
ag = pytest.importorskip("paper_2602_17601_amd.autograd")


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _msd_plan():
    P = wl.make_problem("tan_msd", M=23, hops=2, N=5, n_act=3, model="msd", seed=8, x0_sigma=0.3, walk=0.1,
                        msd=wl.MSDParams(k3=40.0, gravity=9.81))
    plan = gn.Plan(P.M, P.nu, P.N, 1, gn.F64)
    plan.graph_set(P.row_ptr, P.col, 1)
    plan.model_set_msd(P.msd, P.act)
    return P, plan


def _gnn_plan():
    P = wl.gnn100_fp32()
    plan = gn.Plan(P.M, P.nu, P.N, 1, gn.F32)
    plan.graph_set(P.row_ptr, P.col, P.gnn.L)
    plan.model_set_gnn(P.gnn, P.act, dtype=gn.F32)
    return P, plan


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_msd_jvp_vjp_match_the_analytic_blocks_fp64():
    P, plan = _msd_plan()
    prow, pcol, A, B, _ = msd_linearize(P.xhat, P.uhat, P.row_ptr, P.col, P.act, P.msd)
    rng = np.random.default_rng(3)
    dx, du = rng.normal(size=(P.N, P.M, 6)), rng.normal(size=(P.N, P.nu))
    g = rng.normal(size=(P.N, P.M, 6))
    x, u = _t(P.xhat, torch.float64), _t(P.uhat, torch.float64)
    f, t = ag.dynamics_jvp(plan, x, u, _t(dx, torch.float64), _t(du, torch.float64))
    assert _rel(t.cpu().numpy(), jvp_blocks(A, B, prow, pcol, dx, du)) < 1e-12
    xg = x.clone().requires_grad_(True)
    ug = u.clone().requires_grad_(True)
    y = ag.Dynamics.apply(plan, xg, ug)
    assert torch.equal(y.detach(), f)
    (y * _t(g, torch.float64)).sum().backward()
    gx, gu = vjp_blocks(A, B, prow, pcol, g)
    assert _rel(xg.grad[:P.N].cpu().numpy(), gx) < 1e-12
    assert torch.count_nonzero(xg.grad[P.N]) == 0
    assert _rel(ug.grad.cpu().numpy(), gu) < 1e-12


def test_gnn_products_match_the_oracle_on_the_device_blocks():
    P, plan = _gnn_plan()
    N, M, nu = P.N, P.M, P.nu
    x, u = _t(P.xhat, torch.float32), _t(P.uhat, torch.float32)
    A = torch.empty(N, plan.nnz, 6, 6, device="cuda")
    B = torch.empty(N, M, 6, nu, device="cuda")
    c = torch.empty(N, M, 6, device="cuda")
    plan.linearize(x, u, A, B, c)
    rng = np.random.default_rng(4)
    dx, du = rng.normal(size=(N, M, 6)), rng.normal(size=(N, nu))
    g = rng.normal(size=(N, M, 6))
    out = torch.empty(N, M, 6, device="cuda")
    plan.jvp(A, B, _t(dx, torch.float32), _t(du, torch.float32), out)
    gx = torch.empty(N, M, 6, device="cuda")
    gu = torch.empty(N, nu, device="cuda")
    plan.vjp(A, B, _t(g, torch.float32), gx, gu)
    torch.cuda.synchronize()
    # the pattern of the device blocks: the L-hop closure of the graph, as the oracle builds it
    from oracle.graph import jacobian_pattern
    prow, pcol = jacobian_pattern(P.row_ptr, P.col, M, P.gnn.L)
    Ah, Bh = A.double().cpu().numpy(), B.double().cpu().numpy()
    assert _rel(out.cpu().numpy(), jvp_blocks(Ah, Bh, prow, pcol, dx, du)) < 1e-5
    rx, ru = vjp_blocks(Ah, Bh, prow, pcol, g)
    assert _rel(gx.cpu().numpy(), rx) < 1e-5
    assert _rel(gu.cpu().numpy(), ru) < 1e-5
    # repeated calls give the same bits
    out2 = torch.empty_like(out)
    plan.jvp(A, B, _t(dx, torch.float32), _t(du, torch.float32), out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)


def test_gnn_jvp_matches_central_differences_and_the_adjoint_identity():
    P, plan = _gnn_plan()
    N, M, nu = P.N, P.M, P.nu
    x, u = _t(P.xhat, torch.float32), _t(P.uhat, torch.float32)
    rng = np.random.default_rng(6)
    dx = _t(rng.normal(size=(N + 1, M, 6)), torch.float32)
    du = _t(rng.normal(size=(N, nu)), torch.float32)
    f, t = ag.dynamics_jvp(plan, x, u, dx[:N], du)
    h = 1e-3
    fp = ag.Dynamics.apply(plan, x + h * dx, u + h * du)
    fm = ag.Dynamics.apply(plan, x - h * dx, u - h * du)
    fd = ((fp - fm) / (2 * h)).double().cpu().numpy()
    # FP32 model: rounding of the differences and ReLU kinks crossed within +-h bound the agreement
    assert _rel(t.double().cpu().numpy(), fd) < 1e-2
    w = _t(rng.normal(size=(N, M, 6)), torch.float32)
    xg = x.clone().requires_grad_(True)
    ug = u.clone().requires_grad_(True)
    (ag.Dynamics.apply(plan, xg, ug) * w).sum().backward()
    lhs = float((w.double() * t.double()).sum())
    rhs = float((xg.grad.double() * dx.double()).sum() + (ug.grad.double() * du.double()).sum())
    assert abs(lhs - rhs) <= 1e-4 * max(1.0, abs(lhs))


def test_tangent_calls_reject_bad_arguments():
    P, plan = _msd_plan()
    N, M, nu = P.N, P.M, P.nu
    A = torch.zeros(N, plan.nnz, 6, 6, device="cuda", dtype=torch.float64)
    B = torch.zeros(N, M, 6, nu, device="cuda", dtype=torch.float64)
    v = torch.zeros(N, M, 6, device="cuda", dtype=torch.float64)
    w = torch.zeros(N, nu, device="cuda", dtype=torch.float64)
    with pytest.raises(gn.GnmpcError):
        plan.jvp(A, B, v, w[:, :1].contiguous(), v.clone())  # du of the wrong shape
    lib = gn.lib()
    ptr = lambda t: C.c_void_p(t.data_ptr())
    assert lib.gnmpc_jvp(plan._h, ptr(A), ptr(B), None, ptr(w), ptr(v), None) == gn.INVALID_ARG
    assert lib.gnmpc_vjp(plan._h, ptr(A), ptr(B), ptr(v), ptr(v.clone()), None, None) == gn.INVALID_ARG
    torch.cuda.synchronize()
