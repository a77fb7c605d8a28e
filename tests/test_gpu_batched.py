"""Batched steps of independent instances of uneven size (gnmpc_step_batched):
every instance's outputs must equal those of its own single-instance step bit
for bit, run eagerly and as replays of a captured HIP graph."""
import numpy as np
import pytest
import torch

from paper_2602_17601_amd import workloads as wl

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
