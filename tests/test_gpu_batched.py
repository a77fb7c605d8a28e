"""Batched steps of independent instances of uneven size (gnmpc_step_batched):
every instance's outputs must equal those of its own single-instance step bit
for bit, run eagerly and as replays of a captured HIP graph."""
import numpy as np
import pytest
import torch

from paper_2602_17601_amd import workloads as wl
from tests.tolerance import U32, h_err

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")

OUTS = ("A", "B", "c", "H", "g", "u", "info")


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()


def _setup(P):
    plan = gn.Plan(P.M, P.nu, P.N, 1, gn.F32)
    plan.graph_set(P.row_ptr, P.col, P.gnn.L)
    plan.model_set_gnn(P.gnn, P.act, dtype=gn.BF16)
    n = P.N * P.nu
    b = dict(xhat=_t(P.xhat), uhat=_t(P.uhat), x0=_t(P.x0), Q=_t(P.costs.Q), q=_t(P.costs.q), R=_t(P.costs.R),
             r=_t(P.costs.r), lb=_t(P.lb), ub=_t(P.ub),
             A=torch.empty(P.N, plan.nnz, 6, 6, device="cuda"), B=torch.empty(P.N, P.M, 6, P.nu, device="cuda"),
             c=torch.empty(P.N, P.M, 6, device="cuda"), H=torch.empty(n, n, device="cuda"),
             g=torch.empty(n, device="cuda"), u=torch.empty(n, device="cuda"),
             info=torch.zeros(gn.QP_INFO_BYTES, dtype=torch.uint8, device="cuda"))
    return plan, b


def _single(plan, b):
    plan.linearize(b["xhat"], b["uhat"], b["A"], b["B"], b["c"])
    plan.condense(b["A"], b["B"], b["c"], b["x0"], b["Q"], b["q"], b["R"], b["r"], None, None, b["H"], b["g"],
                  None, None)
    plan.solve_box_qp(b["H"], b["g"], b["lb"], b["ub"], None, None, None, b["u"], b["info"])


def _scribble(setups):
    for _, b in setups:
        for k in OUTS:
            if b[k].dtype == torch.uint8:
                b[k][:12].fill_(0xFF)
                b[k][16:].fill_(0xFF)
            else:
                b[k].fill_(float("nan"))


def _check(setups, refs, what):
    for i, ((_, b), ref) in enumerate(zip(setups, refs)):
        for k in OUTS:
            assert torch.equal(b[k], ref[k]), f"{what}: instance {i} {k} differs from its single step"


def test_batched_step_matches_single_instances():
    probs = wl.batch_instances(6, seed=4, M_range=(50, 300), N_range=(5, 14))
    setups = [_setup(P) for P in probs]
    refs = []
    for plan, b in setups:
        _single(plan, b)
        torch.cuda.synchronize()
        refs.append({k: b[k].clone() for k in OUTS})
        assert torch.isfinite(b["u"]).all()
    descs = [gn.step_desc(plan, b) for plan, b in setups]
    _scribble(setups)
    gn.step_batched(descs)
    torch.cuda.synchronize()
    _check(setups, refs, "eager batch")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gn.step_batched(descs)
    for rep in range(3):
        _scribble(setups)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _check(setups, refs, f"graph replay {rep}")


def test_batched_step_rejects_bad_descriptors():
    P = wl.batch_instances(1, seed=5, M_range=(50, 60), N_range=(5, 6))[0]
    plan, b = _setup(P)
    d = gn.step_desc(plan, b)
    d.H = None  # a missing array is reported before anything runs for that instance
    with pytest.raises(gn.GnmpcError):
        gn.step_batched([d])
    torch.cuda.synchronize()


def test_batched_step_matches_oracle_on_serving_shapes():
    """Four instances of the serving workload (uneven M, N up to 30, n_u up to
    12; shared BF16 GNN Hd=128, L=2) in one batched step, each against the FP64
    oracle: condensing of the device's own A, B, c (H - Rbar and g within
    1e-5), the QP solution against the interior-point oracle (1e-4), and the
    Jacobians of 8 nodes at 3 stages against the exact model by the BF16 gate."""
    from oracle.condense import condense_local
    from oracle.gnn import gnn_kink_margin, gnn_linearize
    from oracle.qp import qp_ipm
    from tests.gnn_gate import bf16_gate, delta_A
    every = wl.batch_instances(52, seed=4)
    probs = [every[i] for i in (23, 51, 24, 34)]   # (M, N, n_u) = (304, 30, 12), (117, 30, 12), (75, 20, 9), (212, 10, 6)
    setups = [_setup(P) for P in probs]
    gn.step_batched([gn.step_desc(plan, b) for plan, b in setups])
    torch.cuda.synchronize()
    f64 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    for P, (plan, b) in zip(probs, setups):
        A, B, c = (b[k].double().cpu().numpy() for k in ("A", "B", "c"))
        H, g, u = (b[k].double().cpu().numpy() for k in ("H", "g", "u"))
        prow, pcol = plan.graph_pattern()
        cs = P.costs
        ref = condense_local(A, B, c, prow, pcol, f64(P.x0), f64(cs.Q), f64(cs.q), f64(cs.R), f64(cs.r), wl.no_rows())
        n = P.N * P.nu
        Rb = np.zeros((n, n))
        for k in range(P.N):
            Rb[k * P.nu:(k + 1) * P.nu, k * P.nu:(k + 1) * P.nu] = f64(cs.R[k])
        eh = h_err(H, ref["H"], Rb, U32)
        eg = np.linalg.norm(g - ref["g"]) / np.linalg.norm(ref["g"])
        assert eh < 1e-5 and eg < 1e-5, (P.name, eh, eg)
        uref, *_ = qp_ipm(ref["H"], ref["g"], P.lb, P.ub)
        info = gn.qp_info(b["info"])
        eu = np.linalg.norm(u - uref) / max(np.linalg.norm(uref), 1e-12)
        print(P.name, (P.M, P.N, P.nu), "H", eh, "g", eg, "u", eu, "QP", info.status, info.iters)
        assert info.status == gn.QP_SOLVED and eu < 1e-4, (P.name, info.status, eu)
        Wr = P.gnn.rounded_bf16(biases="f32")
        xh, uh = f64(P.xhat), f64(P.uhat)
        stages = [0, P.N // 2, P.N - 1]
        nodes = sorted({0, 1, int(P.act[0]), int(P.act[-1]), P.M // 3, P.M // 2, P.M - 2, P.M - 1})
        _, _, Ar, Br, _, _ = gnn_linearize(xh, uh, Wr, P.row_ptr, P.col, P.act, stages=stages, nodes=nodes)
        margin = {}
        for k in stages:
            for i, m in zip(nodes, gnn_kink_margin(xh[k], uh[k], Wr, P.row_ptr, P.col, P.act, nodes=nodes)):
                margin[(k, i)] = m
        pairs = [(k, i) for k in stages for i in nodes]
        bf16_gate(delta_A(A, prow, pcol), delta_A(Ar, prow, pcol), B, Br, prow, margin, pairs)


def test_batched_step_rejects_a_repeated_plan():
    """A plan's workspace serves one instance at a time: two descriptors of the
    same plan are refused (INVALID_ARG) before anything is enqueued."""
    P = wl.batch_instances(1, seed=6, M_range=(50, 60), N_range=(5, 6))[0]
    plan, b = _setup(P)
    d = gn.step_desc(plan, b)
    with pytest.raises(gn.GnmpcError) as e:
        gn.step_batched([d, d])
    assert e.value.status == gn.INVALID_ARG
    assert "two descriptors" in gn.lib().gnmpc_plan_last_error(plan._h).decode()
