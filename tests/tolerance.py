"""Error measure for the condensed Hessian H returned in a device precision.

H = Rbar + sum_k S_k' Q_k S_k is compared without Rbar (for the chains used
here Rbar dominates H, so a relative error on H itself would hide errors in
the state part).  But the device stores H itself, not H - Rbar, in its own
precision: every entry carries the rounding of that final store, up to
u |H_ij| with u the unit roundoff (2^-24 for FP32, 2^-53 for FP64), and when
Rbar dominates, that rounding alone can exceed 1e-5 of |H - Rbar|.  No
arithmetic can avoid it, so it is discounted entry by entry:

    e_ij = max(0, |H_ij - Href_ij| - u |Href_ij|)
    h_err = |e|_F / |Href - Rbar|_F

Everywhere Rbar is zero (the off-diagonal stage blocks) the discount is the
rounding of the entry's own value, so the measure is the plain relative error
there up to one unit roundoff per entry.
"""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def h_err(H, Href, Rb, unit):
    """Relative error of H - Rbar after discounting the storage rounding of H."""
    e = np.maximum(0.0, np.abs(H - Href) - unit * np.abs(Href))
    nb = np.linalg.norm(Href - Rb)
    return float(np.linalg.norm(e) / (nb if nb > 0 else 1.0))


def rbar(R, N, nu):
    """Block-diagonal Rbar [N nu][N nu] of the stage input costs R [N][nu][nu]."""
    Rb = np.zeros((N * nu, N * nu))
    for k in range(N):
        Rb[k * nu:(k + 1) * nu, k * nu:(k + 1) * nu] = R[k]
    return Rb
