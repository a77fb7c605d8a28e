"""The paper's own model on the GPU (gnmpc_model_set_inet + gnmpc_linearize):
linearization of the interaction network against the oracle's forward mode, in
FP64 and FP32, and one GNN-MPC loop iteration with it against the oracle's."""
import copy

import numpy as np
import pytest
import torch

from oracle.inet import inet_linearize
from oracle.mpc import initial_trajectory, rti_step
from paper_2602_17601_amd import workloads as wl

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _plan(P, dtype, n_c_max=0):
    plan = gn.Plan(P.M, P.nu, P.N, n_c_max, dtype)
    plan.graph_set(P.row_ptr, P.col, 1)
    plan.model_set_inet(P.inet)
    return plan


def _linearize(plan, P, tdt):
    N, M, nu = P.N, P.M, P.nu
    A = torch.full((N, plan.nnz, 6, 6), float("nan"), dtype=tdt, device="cuda")
    B = torch.full((N, M, 6, nu), float("nan"), dtype=tdt, device="cuda")
    c = torch.full((N, M, 6), float("nan"), dtype=tdt, device="cuda")
    f = torch.full((N, M, 6), float("nan"), dtype=tdt, device="cuda")
    plan.linearize(_t(P.xhat, tdt), _t(P.uhat, tdt), A, B, c, f)
    torch.cuda.synchronize()
    return _np(A), _np(B), _np(c), _np(f)


def test_inet_linearize_fp64_matches_the_oracle():
    """The robot's shape: 4 nodes, 2 neighbours each, psi 4 x 50, phi 8 x 250, nu = 6, N = 20."""
    P = wl.trunk_inet(seed=41, x0_sigma=0.2, walk=0.02)
    plan = _plan(P, gn.F64)
    A, B, c, f = _linearize(plan, P, torch.float64)
    prow, pcol, rA, rB, rc, rf = inet_linearize(P.xhat, P.uhat, P.inet, P.row_ptr, P.col)
    dprow, dpcol = plan.graph_pattern()
    assert np.array_equal(dprow, prow) and np.array_equal(dpcol, pcol)
    for got, ref in ((A, rA), (B, rB), (c, rc), (f, rf)):
        assert _rel(got, ref) < 1e-12


def test_inet_linearize_fp32_wider_graph_matches_the_oracle():
    """FP32 on a 37-node graph with 3 neighbours per node and narrower layers
    (psi 2 x 32 -> 24, phi 3 x 96, nu = 5), the oracle on the FP32-rounded weights."""
    P = wl.trunk_inet(M=37, d=3, N=4, nu=5, seed=42, x0_sigma=0.2, walk=0.02, psi_hidden=2, psi_width=32,
                      d_m=24, phi_hidden=3, phi_width=96)
    plan = _plan(P, gn.F32)
    A, B, c, f = _linearize(plan, P, torch.float32)
    W = copy.deepcopy(P.inet)
    r32 = lambda v: np.asarray(v, np.float32).astype(np.float64)
    W.psi_W, W.psi_b = [r32(v) for v in W.psi_W], [r32(v) for v in W.psi_b]
    W.phi_W, W.phi_b = [r32(v) for v in W.phi_W], [r32(v) for v in W.phi_b]
    _, _, rA, rB, rc, rf = inet_linearize(r32(P.xhat), r32(P.uhat), W, P.row_ptr, P.col)
    assert _rel(A, rA) < 2e-5 and _rel(B, rB) < 2e-5 and _rel(f, rf) < 2e-5
    assert _rel(c, rc) < 1e-4  # c = f - A x - B u cancels


def test_rti_step_with_the_paper_model_matches_the_oracle():
    """One GNN-MPC iteration (FP64) with the interaction network from Algorithm 1's
    initial trajectory; u* by ADMM against the interior-point oracle."""
    P = wl.trunk_inet(N=10, seed=43, x0_sigma=0.05, umax=0.5)
    N, M, nu, n = P.N, P.M, P.nu, P.N * P.nu
    plan = _plan(P, gn.F64)
    xh, uh = initial_trajectory(P.x0, N, nu)
    e = lambda *s: torch.empty(*s, dtype=torch.float64, device="cuda")
    b = dict(xhat=_t(xh, torch.float64), uhat=_t(uh, torch.float64), x0=_t(P.x0, torch.float64),
             Q=_t(P.costs.Q, torch.float64), q=_t(P.costs.q, torch.float64), R=_t(P.costs.R, torch.float64),
             r=_t(P.costs.r, torch.float64), lb=_t(P.lb, torch.float64), ub=_t(P.ub, torch.float64),
             A=e(N, plan.nnz, 6, 6), B=e(N, M, 6, nu), c=e(N, M, 6), H=e(n, n), g=e(n), u=e(n),
             info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda"))
    xpred = e(N + 1, M, 6)
    gn.rti_step(plan, b, xpred)
    torch.cuda.synchronize()
    assert gn.qp_info(b["info"]).status == gn.QP_SOLVED

    def lin(x, u):
        prow, pcol, A, B, c, _ = inet_linearize(x, u, P.inet, P.row_ptr, P.col)
        return prow, pcol, A, B, c

    ref = rti_step(P.x0, xh, uh, lin, P.costs, wl.no_rows(), P.lb, P.ub)
    assert _rel(_np(b["H"]), ref["H"]) < 1e-10 and _rel(_np(b["g"]), ref["g"]) < 1e-10
    assert _rel(_np(b["u"]), ref["u"]) < 1e-3
    assert _rel(_np(xpred), ref["x"]) < 1e-4
    # the same condensed QP by the interior-point solver, the paper's kind of QP solver
    u_ipm = e(n)
    info = torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda")
    plan.solve_qp_ipm(b["H"], b["g"], b["lb"], b["ub"], None, None, None, u_ipm, info, tol=1e-12)
    torch.cuda.synchronize()
    inf = gn.qp_info(info)
    assert inf.status == gn.QP_SOLVED, (inf.status, inf.iters)
    assert _rel(_np(u_ipm), ref["u"]) < max(1e-6, 10 * np.sqrt(inf.kappa_est))


def test_model_set_inet_rejects_bad_calls():
    P = wl.trunk_inet(N=2, seed=44)
    plan = gn.Plan(P.M, P.nu + 1, P.N, 0, gn.F32)  # nu differs from the model's
    plan.graph_set(P.row_ptr, P.col, 1)
    with pytest.raises(gn.GnmpcError) as e:
        plan.model_set_inet(P.inet)
    assert e.value.status == gn.SHAPE
    plan2 = gn.Plan(P.M, P.nu, P.N, 0, gn.F32)
    plan2.graph_set(P.row_ptr, P.col, 2)  # the interaction network has one round
    with pytest.raises(gn.GnmpcError) as e:
        plan2.model_set_inet(P.inet)
    assert e.value.status == gn.SHAPE
    plan3 = _plan(P, gn.F32)
    xh = torch.zeros(P.N + 1, P.M, 6, device="cuda")
    with pytest.raises(gn.GnmpcError) as e:  # only the GNN has the layer-wise reverse mode
        plan3.gnn_forward(xh, torch.zeros(P.N, P.nu, device="cuda"), torch.zeros(P.N, P.M, 6, device="cuda"))
    assert e.value.status == gn.NOT_READY
