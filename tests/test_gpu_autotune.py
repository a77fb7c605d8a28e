"""The condensing autotuner (gnmpc_autotune_condense) and the propagation variants
it chooses between: every variant against the oracle's per-node recursion, and the
tuner's choice (the fastest measured) kept by the plan."""
import numpy as np
import pytest
import torch

from oracle.condense import condense_local
from paper_2602_17601_amd import workloads as wl
from tests.tolerance import U32, h_err, rbar

pytestmark = pytest.mark.gpu

gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda").contiguous()


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _setup(P, L):
    """A plan on P's graph with random rounded-to-FP32 blocks in its pattern (so every
    variant sees the same inputs) and the condensing arrays."""
    plan = gn.Plan(P.M, P.nu, P.N, max(P.rows.n, 1), gn.F32)
    plan.graph_set(P.row_ptr, P.col, L)
    plan.rows_set(P.rows.node, P.rows.stage)
    prow, pcol = plan.graph_pattern()
    rng = np.random.default_rng(P.M + L)
    r32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    A = r32(rng.normal(scale=0.3, size=(P.N, len(pcol), 6, 6)) / np.sqrt(np.diff(prow).max()))
    B = r32(rng.normal(scale=0.1, size=(P.N, P.M, 6, P.nu)))
    c = r32(rng.normal(scale=0.01, size=(P.N, P.M, 6)))
    x0, Q, q, R, r = (r32(v) for v in (P.x0, P.costs.Q, P.costs.q, P.costs.R, P.costs.r))
    rows = wl.StateRows(P.rows.node, P.rows.stage, r32(P.rows.C), r32(P.rows.d))
    n = P.N * P.nu
    e = lambda *s: torch.empty(*s, device="cuda")
    dev = dict(A=_t(A), B=_t(B), c=_t(c), x0=_t(x0), Q=_t(Q), q=_t(q), R=_t(R), r=_t(r), rowC=_t(rows.C),
               rowd=_t(rows.d), H=e(n, n), g=e(n), Ct=e(P.rows.n, n), dt=e(P.rows.n))
    ref = condense_local(A, B, c, prow, pcol, x0, Q, q, R, r, rows)
    return plan, dev, ref, rbar(R, P.N, P.nu)


def _condense(plan, d):
    plan.condense(d["A"], d["B"], d["c"], d["x0"], d["Q"], d["q"], d["R"], d["r"], d["rowC"], d["rowd"], d["H"],
                  d["g"], d["Ct"], d["dt"])
    torch.cuda.synchronize()
    return {k: _np(d[k]) for k in ("H", "g", "Ct", "dt")}


def _check(out, ref, Rb):
    assert h_err(out["H"], ref["H"], Rb, U32) < 1e-5
    for k in ("g", "Ct", "dt"):
        assert _rel(out[k], ref[k]) < 1e-5, k


@pytest.mark.parametrize("M,hops,L,N,nu", [(300, 2, 1, 12, 6), (120, 2, 2, 10, 6)])
def test_every_propagation_variant_matches_the_oracle(M, hops, L, N, nu):
    P = wl.make_problem("tune", M=M, hops=hops, N=N, n_act=nu // 3, model="msd", seed=M, n_random_rows=40)
    plan, d, ref, Rb = _setup(P, L)
    tried = 0
    for variant, nb in [(0, 0), (1, 16), (1, 8), (1, 4), (1, 2), (1, 1), (2, 16), (2, 8), (2, 4), (2, 2), (2, 1)]:
        try:
            plan.condense_variant(variant, nb)
        except gn.GnmpcError as e:
            assert e.status == gn.UNSUPPORTED  # these blocks do not fit LDS
            continue
        got = plan.condense_variant()
        assert got[0] == variant and (variant == 0 or got[1] == nb)
        _check(_condense(plan, d), ref, Rb)
        tried += 1
    assert tried >= 4


def test_autotuner_keeps_the_fastest_variant_and_it_matches_the_oracle():
    P = wl.make_problem("tune_gnn", M=400, hops=2, N=16, n_act=4, model="msd", seed=9, n_random_rows=60)
    plan, d, ref, Rb = _setup(P, 3)  # the 3-hop pattern of a GNN with three rounds
    chosen, entries = plan.autotune_condense(d["A"], d["B"], d["c"], d["x0"], d["Q"], d["q"], d["R"], d["r"],
                                             d["rowC"], d["rowd"], d["H"], d["g"], d["Ct"], d["dt"], reps=3)
    assert len(entries) >= 2
    assert entries[chosen]["us"] == min(e["us"] for e in entries)
    v, nb = plan.condense_variant()
    assert v == entries[chosen]["variant"]
    if v >= 1:
        assert nb == entries[chosen]["block_nodes"]
    print("tuning", entries, "chosen", chosen)
    a = _condense(plan, d)
    b = _condense(plan, d)
    _check(a, ref, Rb)
    for k in a:
        assert np.array_equal(a[k], b[k])  # the kept choice is deterministic
