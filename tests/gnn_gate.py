"""Parity gate of BF16 GNN Jacobians against the exact FP64 oracle.

The device runs the GNN with bfloat16 weights.  Its forward pass carries the
activations at FP32 accuracy, so its ReLU decisions equal the exact model's
except where a pre-activation z is within FP32 accumulation error of zero;
its tangents are rounded to bfloat16.  The oracle is the exact FP64 model on
the same (bf16-rounded) weights, with no rounding of its own.

Rule, per (stage, node) pair:
  * error = rel-Frobenius of the node's A row minus its identity part, and
    of its B row (B rows that are exactly zero in the oracle must be exactly
    zero on the device);
  * a pair above the bound is excused only if the oracle finds, in the node's
    receptive field, a pre-activation with |z| <= KINK * sum|terms of z|, the
    worst-case FP32 accumulation error of the 2 Hd + 1 terms (n u = 256 *
    2^-24 = 2^-16): there the two sides may legitimately take different
    decisions (the Jacobian of a ReLU network jumps across a kink);
  * excused pairs are counted and may be at most 1% of the pairs checked;
    a pair above the bound that is not near a kink fails the gate;
  * the rel-Frobenius over all checked pairs of each stage, excused ones
    included, stays within the bound.
"""
import numpy as np

BOUND = 2e-2
KINK = 2.0 ** -16
MAX_EXCUSED = 0.01


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def delta_A(A, prow, pcol):
    """A with the identity removed from the diagonal blocks (the part the model learns)."""
    D = A.copy()
    M = len(prow) - 1
    for i in range(M):
        for e in range(prow[i], prow[i + 1]):
            if pcol[e] == i:
                D[..., e, :, :] -= np.eye(6)
    return D


def bf16_gate(dA, dAr, B, Br, prow, margin, pairs):
    """dA/dAr: device / oracle A - I [N][nnz][6][6]; B/Br [N][M][6][nu];
    margin[(k, i)] from oracle.gnn.gnn_kink_margin; pairs: list of (k, i).
    Returns a report dict; raises AssertionError when the gate fails."""
    bad, excused = [], []
    worst = 0.0
    for k, i in pairs:
        sl = slice(prow[i], prow[i + 1])
        ea = rel(dA[k, sl], dAr[k, sl])
        if np.abs(Br[k, i]).sum() == 0:
            assert np.all(B[k, i] == 0), ("B must be exactly zero", k, i)
            eb = 0.0
        else:
            eb = rel(B[k, i], Br[k, i])
        e = max(ea, eb)
        if e > BOUND:
            (excused if margin[(k, i)] <= KINK else bad).append((k, i, e, margin[(k, i)]))
        else:
            worst = max(worst, e)
    stages = sorted({k for k, _ in pairs})
    agg = {}
    for k in stages:
        nodes = [i for kk, i in pairs if kk == k]
        sel = np.concatenate([np.arange(prow[i], prow[i + 1]) for i in nodes])
        agg[k] = (rel(dA[k, sel], dAr[k, sel]), rel(B[k, nodes], Br[k, nodes]))
    near = sum(1 for p in pairs if margin[p] <= KINK)
    report = dict(pairs=len(pairs), near_kink=near, excused=excused, unexcused=bad,
                  worst_kept=worst, worst_stage=max(max(v) for v in agg.values()))
    print("BF16 gate:", {k: v for k, v in report.items() if k not in ("excused",)},
          "excused:", [(k, i, round(e, 4)) for k, i, e, _ in excused])
    assert not bad, ("pairs above the bound with no near-kink pre-activation", bad)
    assert len(excused) <= MAX_EXCUSED * len(pairs), ("too many excused pairs", excused)
    for k, (ea, eb) in agg.items():
        assert ea < BOUND and eb < BOUND, ("stage aggregate above the bound", k, ea, eb)
    return report
