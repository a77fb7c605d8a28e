"""Algorithm 1 on the GPU (gnmpc_rti_step): closed loops against the oracle's
loop iteration (FP64 spring-damper controller, and a GNN controller in FP32),
with the spring-damper simulator (gnmpc_msd_simulate) as the plant."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle.gnn import gnn_linearize
from oracle.mpc import initial_trajectory, rti_step
from oracle.msd import msd_linearize, msd_step
from paper_2602_17601_amd import workloads as wl

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _t(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _bufs(plan, P, tdt, x0, xhat, uhat):
    N, M, nu, n = P.N, P.M, P.nu, P.N * P.nu
    e = lambda *s: torch.empty(*s, dtype=tdt, device="cuda")
    return dict(xhat=_t(xhat, tdt), uhat=_t(uhat, tdt), x0=_t(x0, tdt), Q=_t(P.costs.Q, tdt), q=_t(P.costs.q, tdt),
                R=_t(P.costs.R, tdt), r=_t(P.costs.r, tdt), lb=_t(P.lb, tdt), ub=_t(P.ub, tdt),
                A=e(N, plan.nnz, 6, 6), B=e(N, M, 6, nu), c=e(N, M, 6), H=e(n, n), g=e(n), u=e(n),
                info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda"))


def _msd_plan(P, dtype):
    plan = gn.Plan(P.M, P.nu, P.N, 0, dtype)
    plan.graph_set(P.row_ptr, P.col, 1)
    plan.model_set_msd(P.msd, P.act)
    return plan


def _plant_step(plant, b, x_next, nu):
    """x_next <- f(x0, u*[0]) on the simulator; returns nothing (device)."""
    M = b["x0"].shape[0]
    X = torch.empty(1, 2, M, 6, dtype=b["x0"].dtype, device="cuda")
    plant.msd_simulate(b["x0"].view(1, M, 6), b["u"][:nu].view(1, 1, nu), X)
    x_next.copy_(X[0, 1])


def test_rti_closed_loop_fp64_spring_damper_matches_the_oracle():
    """40-node nonlinear chain (cubic springs), N = 15, |u| <= 0.5 (active at some
    steps): 12 closed-loop iterations on each side; the QP is solved by ADMM on the
    device and by the interior-point oracle, so u agrees to ADMM's accuracy."""
    prm = wl.MSDParams(k=10.0, c=0.1, m=1.0, dt=0.05, k3=50.0)
    P = wl.make_problem("rti64", M=40, hops=2, N=15, n_act=2, model="msd", seed=31, msd=prm, x0_sigma=0.05,
                        umax=0.5, qdiag=(100, 100, 100, 1, 1, 1), rho_r=1e-3)
    N, M, nu = P.N, P.M, P.nu
    plan = _msd_plan(P, gn.F64)
    xh, uh = initial_trajectory(P.x0, N, nu)
    b = _bufs(plan, P, torch.float64, P.x0, xh, uh)
    xpred = torch.empty(N + 1, M, 6, dtype=torch.float64, device="cuda")
    lin = lambda a, c: msd_linearize(a, c, P.row_ptr, P.col, P.act, prm)
    x = P.x0.copy()
    active = 0
    for t in range(12):
        gn.rti_step(plan, b, xpred)
        torch.cuda.synchronize()
        assert gn.qp_info(b["info"]).status == gn.QP_SOLVED
        ref = rti_step(x, xh, uh, lin, P.costs, wl.no_rows(), P.lb, P.ub)
        u = _np(b["u"])
        assert _rel(u, ref["u"]) < 1e-3, (t, _rel(u, ref["u"]))
        assert _rel(_np(xpred), ref["x"]) < 1e-4
        assert _rel(_np(b["xhat"]), ref["xhat"]) < 1e-4
        assert _rel(_np(b["uhat"]), ref["uhat"]) < 1e-3
        active += int(np.any(np.abs(ref["u"][:nu]) > 0.5 - 1e-6))
        _plant_step(plan, b, b["x0"], nu)
        x = msd_step(x, ref["u"][:nu], P.row_ptr, P.col, P.act, prm)
        xh, uh = ref["xhat"], ref["uhat"]
        torch.cuda.synchronize()
        assert _rel(_np(b["x0"]), x) < 1e-4
    assert active > 0


def test_rti_with_the_interior_point_qp_matches_the_oracle_loop():
    """The spring-damper closed loop of the test above with gnmpc_rti_step_ipm: the
    condensed QPs solved by the device's interior-point method (tol 1e-12), so u*
    follows the oracle's interior-point solution to the IPM's own accuracy
    (max(1e-6, 10 sqrt(mu)) at its last duality measure mu), not ADMM's."""
    prm = wl.MSDParams(k=10.0, c=0.1, m=1.0, dt=0.05, k3=50.0)
    P = wl.make_problem("rti64ipm", M=40, hops=2, N=15, n_act=2, model="msd", seed=31, msd=prm, x0_sigma=0.05,
                        umax=0.5, qdiag=(100, 100, 100, 1, 1, 1), rho_r=1e-3)
    N, M, nu = P.N, P.M, P.nu
    plan = _msd_plan(P, gn.F64)
    xh, uh = initial_trajectory(P.x0, N, nu)
    b = _bufs(plan, P, torch.float64, P.x0, xh, uh)
    xpred = torch.empty(N + 1, M, 6, dtype=torch.float64, device="cuda")
    lin = lambda a, c: msd_linearize(a, c, P.row_ptr, P.col, P.act, prm)
    x = P.x0.copy()
    active = 0
    for t in range(8):
        gn.rti_step_ipm(plan, b, xpred, tol=1e-12)
        torch.cuda.synchronize()
        inf = gn.qp_info(b["info"])
        assert inf.status == gn.QP_SOLVED, (t, inf.status, inf.iters)
        ref = rti_step(x, xh, uh, lin, P.costs, wl.no_rows(), P.lb, P.ub)
        tol_u = max(1e-6, 10 * np.sqrt(inf.kappa_est))
        assert _rel(_np(b["u"]), ref["u"]) < tol_u, (t, _rel(_np(b["u"]), ref["u"]))
        assert _rel(_np(xpred), ref["x"]) < 1e-4
        active += int(np.any(np.abs(ref["u"][:nu]) > 0.5 - 1e-6))
        _plant_step(plan, b, b["x0"], nu)
        x = msd_step(x, ref["u"][:nu], P.row_ptr, P.col, P.act, prm)
        xh, uh = ref["xhat"], ref["uhat"]
        torch.cuda.synchronize()
        assert _rel(_np(b["x0"]), x) < 1e-4
    assert active > 0
    with pytest.raises(gn.GnmpcError) as e:
        gn.rti_step_ipm(plan, b, xpred, tol=0.0)
    assert e.value.status == gn.INVALID_ARG


def test_rti_gnn_controller_fp32_matches_the_oracle_on_the_measured_states():
    """A GNN controller (FP32 weights, Hd = 64, L = 2, 14 nodes, N = 5) on the
    spring-damper plant: at every iteration the oracle runs the same loop
    iteration from the device's measured state and linearization trajectory."""
    prm = wl.MSDParams(k=10.0, c=0.1, m=1.0, dt=0.05, k3=50.0)
    P = wl.make_problem("rtignn", M=14, hops=2, N=5, n_act=2, model="gnn", seed=32, Hd=64, L=2, msd=prm,
                        x0_sigma=0.05, umax=0.5, qdiag=(100, 100, 100, 1, 1, 1), rho_r=1e-3)
    N, M, nu = P.N, P.M, P.nu
    plan = gn.Plan(M, nu, N, 0, gn.F32)
    plan.graph_set(P.row_ptr, P.col, P.gnn.L)
    plan.model_set_gnn(P.gnn, P.act, dtype=gn.F32)
    plant = _msd_plan(P, gn.F32)
    xh, uh = initial_trajectory(P.x0, N, nu)
    b = _bufs(plan, P, torch.float32, P.x0, xh, uh)
    xpred = torch.empty(N + 1, M, 6, device="cuda")
    f64 = lambda a: np.asarray(a, np.float32).astype(np.float64)

    def lin(a, c):
        prow, pcol, A, B, cc, _ = gnn_linearize(a, c, P.gnn, P.row_ptr, P.col, P.act)
        return prow, pcol, A, B, cc

    for t in range(4):
        x0, xh, uh = _np(b["x0"]), _np(b["xhat"]), _np(b["uhat"])
        gn.rti_step(plan, b, xpred)
        torch.cuda.synchronize()
        ref = rti_step(f64(x0), f64(xh), f64(uh), lin, P.costs, wl.no_rows(), P.lb, P.ub)
        assert _rel(_np(b["u"]), ref["u"]) < 1e-3, (t, _rel(_np(b["u"]), ref["u"]))
        assert _rel(_np(xpred), ref["x"]) < 1e-4
        _plant_step(plant, b, b["x0"], nu)
        torch.cuda.synchronize()


def test_rti_step_rejects_aliased_prediction_buffers():
    P = wl.make_problem("rtibad", M=9, hops=1, N=3, n_act=1, model="msd", seed=1)
    plan = _msd_plan(P, gn.F32)
    xh, uh = initial_trajectory(P.x0, P.N, P.nu)
    b = _bufs(plan, P, torch.float32, P.x0, xh, uh)
    with pytest.raises(gn.GnmpcError) as e:
        gn.rti_step(plan, b, b["xhat"])
    assert e.value.status == gn.INVALID_ARG
    L = gn.lib()
    s = gn.default_admm_settings()
    assert L.gnmpc_rti_step(None, None, None, None, C.byref(s), None) == gn.INVALID_ARG
