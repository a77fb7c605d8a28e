"""Trajectories of the nonlinear mass-spring-damper chain on the GPU
(gnmpc_msd_simulate) against the oracle's step applied T times."""
import numpy as np
import pytest
import torch

from oracle.msd import msd_step
from paper_2602_17601_amd import workloads as wl

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _run(S, dtype):
    B, T = S.u.shape[0], S.u.shape[1]
    gdt = gn.F64 if dtype == torch.float64 else gn.F32
    plan = gn.Plan(S.M, S.nu, 1, 1, gdt)
    plan.graph_set(S.row_ptr, S.col, 1)
    plan.model_set_msd(S.msd, S.act)
    t = lambda a: torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()
    X = torch.full((B, T + 1, S.M, 6), float("nan"), dtype=dtype, device="cuda")
    x0, u = t(S.x0), t(S.u)
    plan.msd_simulate(x0, u, X)
    torch.cuda.synchronize()
    assert torch.equal(X[:, 0], x0)
    npd = np.float64 if dtype == torch.float64 else np.float32
    return X.double().cpu().numpy(), np.asarray(S.x0, npd).astype(np.float64), np.asarray(S.u, npd).astype(np.float64)


def _oracle(S, x0, u):
    B, T = u.shape[0], u.shape[1]
    X = np.zeros((B, T + 1, S.M, 6))
    for b in range(B):
        X[b, 0] = x0[b]
        for t in range(T):
            X[b, t + 1] = msd_step(X[b, t], u[b, t], S.row_ptr, S.col, S.act, S.msd)
    return X


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_msd_simulate_matches_the_oracle_step(dtype, tol):
    """Cubic springs, gravity, an anchored node, 3 actuated nodes, uneven node
    count (more nodes than the 256 lanes of a workgroup): every state of every
    trajectory."""
    S = wl.simulator_batch(B=3, T=12, M=301, hops=2, n_act=3, seed=7, x0_sigma=0.2, step=0.3)
    X, x0, u = _run(S, dtype)
    R = _oracle(S, x0, u)
    rel = np.linalg.norm(X - R) / np.linalg.norm(R)
    print(dtype, "rel", rel)
    assert rel < tol


def test_msd_simulate_zero_steps_and_argument_errors():
    S = wl.simulator_batch(B=2, T=0, M=20, hops=1, n_act=2, seed=8)
    X, x0, _ = _run(S, torch.float64)
    assert np.array_equal(X[:, 0], x0)
    P = wl.make_problem("sim_gnn", M=20, hops=1, N=2, n_act=2, model="gnn", seed=1, Hd=64, L=1)
    plan = gn.Plan(P.M, P.nu, P.N, 1, gn.F32)
    plan.graph_set(P.row_ptr, P.col, 1)
    plan.model_set_gnn(P.gnn, P.act)
    x = torch.zeros(1, P.M, 6, device="cuda")
    with pytest.raises(gn.GnmpcError) as e:  # a GNN plan has no spring-damper model to simulate
        plan.msd_simulate(x, torch.zeros(1, 1, P.nu, device="cuda"), torch.zeros(1, 2, P.M, 6, device="cuda"))
    assert e.value.status == gn.NOT_READY
