"""One iteration of the GNN-MPC loop (Algorithm 1) in FP64 (oracle; test
infrastructure only).

``rti_step`` takes the loop body's steps in the paper's order: linearize the
model around the linearization trajectory {xhat_k, uhat_k} (Sec. V-A
"Linearization"), condense with the measured initial state x0 (Sec. V-B), solve
the condensed QP (Sec. III-B eq. condensed_matrices, box bounds and state rows),
then update the linearization trajectory with the shifted optimal solution.
The optimal states are x* = Gamma_u u* + Gamma_x, i.e. the linearized dynamics
rolled forward from x0 with u*.  The shift {xhat_k, uhat_k} <- {x*_{k+1}, u*_{k+1}}
leaves the last stage open; the reading taken here repeats the last one:
xhat'[N] = x*[N] and uhat'[N-1] = u*[N-1].  Algorithm 1 initializes the
trajectory with xhat_k = x(t) for every k and uhat_k = 0 (``initial_trajectory``).
"""
from __future__ import annotations

import numpy as np

from oracle.condense import condense_local, rollout
from oracle.qp import qp_ipm


def initial_trajectory(x, N, nu):
    """Algorithm 1's initialization: every stage at the current state, zero inputs."""
    x = np.asarray(x, dtype=np.float64)
    return np.repeat(x[None], N + 1, axis=0), np.zeros((N, nu))


def rti_step(x0, xhat, uhat, linearize, costs, rows, lb, ub):
    """One loop iteration.  linearize(xhat, uhat) -> (prow, pcol, A, B, c).

    Returns dict(u, x, xhat, uhat, H, g, Ct, dt): the QP solution u* [N nu], the
    optimal predicted states x* [N+1][M][6], the shifted trajectory for the next
    iteration, and the condensed QP data."""
    N, nu = np.asarray(uhat).shape
    prow, pcol, A, B, c = linearize(xhat, uhat)
    cd = condense_local(A, B, c, prow, pcol, x0, costs.Q, costs.q, costs.R, costs.r, rows)
    if rows.n:
        u = qp_ipm(cd["H"], cd["g"], lb, ub, cd["Ct"], None, cd["dt"])[0]
    else:
        u = qp_ipm(cd["H"], cd["g"], lb, ub)[0]
    x = rollout(A, B, c, prow, pcol, x0, u)
    U = u.reshape(N, nu)
    return dict(u=u, x=x, xhat=np.concatenate([x[1:], x[N:]]), uhat=np.concatenate([U[1:], U[N - 1:]]),
                H=cd["H"], g=cd["g"], Ct=cd["Ct"], dt=cd["dt"])
