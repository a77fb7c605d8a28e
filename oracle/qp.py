"""Strictly convex QP solvers (oracle; test infrastructure only).

Problem (the condensed QP of Sec. III-B, with box input bounds kept native and
the condensed state rows as two-sided general rows):
    minimize 1/2 u'Hu + g'u   s.t.  lb <= u <= ub,  lc <= Ct u <= uc
H is symmetric positive definite, so the minimizer is unique.

``qp_ipm``        primal-dual interior-point method with Mehrotra's
                  predictor-corrector (Mehrotra 1992; the paper's condensed QPs
                  are solved by an IPM, Sec. V-C and VI-A).
``qp_enumerate``  brute force over every active pattern (tiny problems only):
                  the unique minimizer is the lowest-objective feasible
                  stationary point among all faces.
``kkt_residuals`` optimality residuals of a primal-dual pair.
"""
from __future__ import annotations

import itertools

import numpy as np


def _inequalities(n, lb, ub, Ct, lc, uc):
    """Stack the finite bounds as G u <= h."""
    G, h = [], []
    I = np.eye(n)
    for a in range(n):
        if np.isfinite(ub[a]):
            G.append(I[a]); h.append(ub[a])
        if np.isfinite(lb[a]):
            G.append(-I[a]); h.append(-lb[a])
    if Ct is not None:
        for t in range(Ct.shape[0]):
            if np.isfinite(uc[t]):
                G.append(Ct[t]); h.append(uc[t])
            if np.isfinite(lc[t]):
                G.append(-Ct[t]); h.append(-lc[t])
    if not G:
        return np.zeros((0, n)), np.zeros(0)
    return np.asarray(G, dtype=np.float64), np.asarray(h, dtype=np.float64)


def qp_ipm(H, g, lb, ub, Ct=None, lc=None, uc=None, tol=1e-10, max_iter=200):
    """Returns (u, lam, G, h): minimizer, multipliers of G u <= h, and G, h.

    The interior-point iterations drive the residuals and the duality measure
    towards zero; the final iterate is then refined on its active set (the
    constraints whose multiplier exceeds their slack) by one equality-constrained
    KKT solve, which is accepted only if it is primal feasible with nonnegative
    multipliers -- for a nondegenerate problem that point is the exact minimizer.
    """
    H = np.asarray(H, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = g.shape[0]
    G, h = _inequalities(n, lb, ub, Ct, lc, uc)
    m = G.shape[0]
    if m == 0:
        return np.linalg.solve(H, -g), np.zeros(0), G, h
    u = np.zeros(n)
    s = np.maximum(h - G @ u, 1.0)
    lam = np.ones(m)
    scale = max(1.0, np.abs(g).max(), np.abs(h).max())
    converged = False
    for _ in range(max_iter):
        rd = H @ u + g + G.T @ lam
        rp = G @ u + s - h
        mu = s @ lam / m
        if max(np.abs(rd).max(), np.abs(rp).max()) <= tol * scale and mu <= 1e-3 * tol * scale:
            converged = True
            break
        W = lam / s
        K = H + G.T @ (W[:, None] * G)
        try:
            Lc = np.linalg.cholesky(K)
        except np.linalg.LinAlgError:      # scaling exhausted double precision
            break

        def solve(rc):
            rhs = -rd - G.T @ (W * rp - rc / s)
            du = np.linalg.solve(Lc.T, np.linalg.solve(Lc, rhs))
            dlam = W * (G @ du + rp) - rc / s
            ds = -(rc + s * dlam) / lam
            return du, ds, dlam

        def max_step(v, dv):
            neg = dv < 0
            return min(1.0, float(np.min(-v[neg] / dv[neg]))) if np.any(neg) else 1.0

        # predictor (affine scaling direction)
        du, ds, dlam = solve(s * lam)
        a = min(max_step(s, ds), max_step(lam, dlam))
        mu_aff = (s + a * ds) @ (lam + a * dlam) / m
        sigma = (mu_aff / mu) ** 3
        # centring-corrector direction
        du, ds, dlam = solve(s * lam + ds * dlam - sigma * mu)
        a = min(1.0, 0.995 * min(max_step(s, ds), max_step(lam, dlam)))
        if a < 1e-14:
            break
        u, s, lam = u + a * du, s + a * ds, lam + a * dlam
    # refinement on the identified active set
    act = lam > s
    k = int(act.sum())
    Ga = G[act]
    K = np.block([[H, Ga.T], [Ga, np.zeros((k, k))]])
    try:
        sol = np.linalg.solve(K, np.concatenate([-g, h[act]]))
        up = sol[:n]
        lp = np.zeros(m)
        lp[act] = sol[n:]
        feas = np.all(G @ up <= h + 1e-12 * scale)
        if feas and np.all(lp >= -1e-12 * scale) and np.all(np.isfinite(sol)):
            return up, np.maximum(lp, 0.0), G, h
    except np.linalg.LinAlgError:
        pass
    if converged:
        return u, lam, G, h
    raise RuntimeError("qp_ipm did not converge (infeasible or ill-posed QP)")


def kkt_residuals(H, g, u, lam, G, h):
    """(stationarity, primal infeasibility, complementarity, dual infeasibility)."""
    st = np.abs(H @ u + g + G.T @ lam).max() if G.size else np.abs(H @ u + g).max()
    if G.shape[0] == 0:
        return st, 0.0, 0.0, 0.0
    slack = h - G @ u
    return (st, max(0.0, -slack.min()), np.abs(slack * lam).max(), max(0.0, -lam.min()))


def qp_enumerate(H, g, lb, ub, Ct=None, lc=None, uc=None, feas_tol=1e-10):
    """Brute-force minimizer: try every assignment of each constraint to
    {at lower, inactive, at upper}, solve the equality-constrained QP on that
    face, keep the feasible point of lowest objective."""
    H = np.asarray(H, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = g.shape[0]
    rows = [np.eye(n)[a] for a in range(n)]
    lo = list(lb)
    hi = list(ub)
    if Ct is not None:
        rows += [Ct[t] for t in range(Ct.shape[0])]
        lo += list(lc)
        hi += list(uc)
    best, best_obj = None, np.inf
    for pat in itertools.product((-1, 0, 1), repeat=len(rows)):
        Aeq, beq = [], []
        ok = True
        for t, p in enumerate(pat):
            if p == 0:
                continue
            b = lo[t] if p < 0 else hi[t]
            if not np.isfinite(b):
                ok = False
                break
            Aeq.append(rows[t]); beq.append(b)
        if not ok:
            continue
        k = len(Aeq)
        if k:
            Aeq = np.asarray(Aeq)
            K = np.block([[H, Aeq.T], [Aeq, np.zeros((k, k))]])
            rhs = np.concatenate([-g, beq])
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            if not np.all(np.isfinite(sol)) or np.linalg.cond(K) > 1e12:
                continue
            x = sol[:n]
        else:
            x = np.linalg.solve(H, -g)
        vals = np.array([r @ x for r in rows])
        if np.any(vals < np.asarray(lo) - feas_tol) or np.any(vals > np.asarray(hi) + feas_tol):
            continue
        obj = 0.5 * x @ H @ x + g @ x
        if obj < best_obj - 1e-14:
            best, best_obj = x, obj
    return best
