"""Projected Newton for a convex function over a box x >= lo.  Test
infrastructure only.

Bertsekas, "Projected Newton methods for optimization problems with simple
constraints" (SIAM J. Control Optim. 20, 1982): coordinates at (or within one
diagonally scaled projected-gradient step of) their bound whose gradient
pushes them out of the box form the active set and take a scaled gradient
step; the free coordinates take a Newton step; the step is searched along the
projection arc x(a) = max(x + a d, lo) with the Armijo rule of that paper
(predicted decrease: the directional derivative on the free set plus the
gradient times the actual move on the active set).

The Newton system on the free set is regularised by diag(|g_i| / x_i) (a
Levenberg-Marquardt term proportional to the gradient, which keeps local
convergence quadratic and is invariant to the scale of each coordinate), so
that it stays solvable where the function is linear along a direction (a
flat or sloped shift of the eigenvalue model: a step of the order of x is then
taken along it) and tends to the plain Newton system as the gradient
vanishes (x > 0 on the box here).  Near the solution, where the predicted decrease drops
below the rounding of f, the full Newton step is taken without a test.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def kkt_scaled(x, g, lo, scale):
    """max over coordinates of |g| / scale (free) or max(0, -g) / scale (at the bound)."""
    at = x <= lo * (1.0 + 1e-12)
    r = np.where(at, np.maximum(0.0, -g), np.abs(g)) / scale
    return float(r.max()) if r.size else 0.0


def _solve_spd(A, b):
    try:
        c = scipy.linalg.cho_factor(A, lower=False, check_finite=False)
        return scipy.linalg.cho_solve(c, b, check_finite=False)
    except np.linalg.LinAlgError:
        return np.linalg.lstsq(A, b, rcond=None)[0]


def minimize_box(evaluate, x0, lo, scale, tol, max_iter=500, sigma=1e-3, beta=0.4):
    """Minimise a convex f over x >= lo.

    evaluate(x, need_derivs) returns f, or (f, g, H) with H dense, at x.
    scale: positive per-coordinate scale of the KKT measure.
    Returns (x, iterations, kkt, stalled)."""
    x = np.maximum(np.asarray(x0, dtype=np.float64), lo)
    f, g, H = evaluate(x, True)
    it = 0
    kkt = kkt_scaled(x, g, lo, scale)
    stalled = False
    while kkt > tol and it < max_iter:
        it += 1
        D = np.diag(H).copy()
        tau = np.abs(g) / x
        Ds = D + tau
        reach = np.abs(x - np.maximum(x - g / Ds, lo))
        act = (x - lo <= reach) & (g > 0)
        F = ~act
        d = np.zeros_like(x)
        d[act] = -g[act] / Ds[act]
        if F.any():
            A = H[np.ix_(F, F)] + np.diag(tau[F])
            d[F] = _solve_spd(A, -g[F])
        alpha = 1.0
        accepted = False
        for _ in range(200):
            xt = np.maximum(x + alpha * d, lo)
            pred = alpha * float(g[F] @ d[F]) + float(g[act] @ (xt[act] - x[act]))
            if alpha == 1.0 and abs(pred) <= 64 * np.finfo(float).eps * (abs(f) + 1.0):
                accepted = True          # below the rounding of f: the Newton step stands
                break
            ft = evaluate(xt, False)
            if ft <= f + sigma * pred:
                accepted = True
                break
            alpha *= beta
        if not accepted:
            stalled = True
            break
        x = xt
        f, g, H = evaluate(x, True)
        kkt = kkt_scaled(x, g, lo, scale)
    return x, it, kkt, stalled
