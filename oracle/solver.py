"""Eigenvalue maximum-likelihood estimate.  Test infrastructure only.

Model equation (singular Kronecker-sum normal) with Theorem 1: once the
eigenvectors V_l are fixed to those of S_l, the negative log-likelihood of one
modality gamma = (a, b) in the eigenvalues lambda_a (r_a entries), lambda_b is

    NLL = 1/2 [ sum_i E_a,i lambda_a,i + sum_j E_b,j lambda_b,j
                - sum_{i<=r_a, j<=r_b} log(lambda_a,i + lambda_b,j) ]

(trace identity tr[S_l Psi_l] = sum_i E_l,i lambda_l,i; the pseudo-determinant
of the Kronecker sum restricted to span(V_a (x) V_b) is the product of the
pairwise sums; the derivation appendix gives r_forall = prod r_l).  Several
modalities add their terms, sharing the eigenvalues of shared axes.  The
eigenvalue-gradient Proposition gives

    dNLL/dlambda_l,i = 1/2 ( E_l,i - sum_{gamma containing l} sum_j 1/(lambda_l,i + lambda_m,j) ).

Readings taken here (the paper leaves these open):

* Domain: the per-axis box lambda_l,i >= eps_l of the Existence lemma (on which
  uniqueness is claimed), not Algorithm 1's sum-of-minima test.  Default
  eps_l = 1e-10 / max_i E_l,i.
* Sums over pairs run over the retained ranks (r_a x r_b pairs).
* Shift directions: adding c_l to every eigenvalue of axis l with
  sum_{l in gamma} c_l = 0 for all gamma leaves every log term unchanged
  (Identifiability appendix).  Along such a direction the NLL is linear with
  slope 1/2 sum_l c_l sum_i E_l,i.  When that slope is zero ("balanced", e.g.
  one modality with r_a = r_b and equal spectra) the minimiser is a line; we
  pick the point that keeps the value of sum_l c_l sum_i lambda_l,i that
  Algorithm 1's start lambda^0 = 1/E has (gradient and Newton steps keep it).
  When the slope is nonzero the box stops the descent and some eigenvalues of
  the larger-trace axis end pinned at eps.
* "While not converged" is read as: scaled KKT residual below ``tol``, where a
  free coordinate contributes |g_i| / (E_i / 2) and a coordinate at its bound
  contributes max(0, -g_i) / (E_i / 2).

Method (an optimiser of its own, sharing no step rule with the library):
profile likelihood.  The axes are split into an outer set and an inner set
that no modality joins to itself (an independent set of the modality graph).
For fixed outer eigenvalues the NLL separates into one-dimensional convex
problems, one per inner eigenvalue: lambda_m,j solves
E_m,j = sum_{partners} sum_i 1/(lambda_l,i + lambda_m,j), or sits at eps_m
when the derivative is already non-negative there; each is solved to the last
bit by Newton's method from the left (the right-hand side is convex and
decreasing).  The profiled NLL of the outer eigenvalues is convex; its
gradient is the partial gradient at the inner optimum (envelope theorem) and
its Hessian the Schur complement of the free inner coordinates.  It is
minimised by ``oracle.newton.minimize_box`` (Bertsekas' projected Newton).
Sums over the partner axis are taken in extended precision, so the scaled KKT
residual reaches ~1e-15.  The result is finally moved along the flat
directions to the start's gauge (the rule above).
``projected_gradient`` is a plain projected gradient descent of the same NLL
from Algorithm 1's start, for small cross-checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .newton import minimize_box


@dataclass
class Problem:
    E: list                      # per axis: float64 array, descending, positive
    modalities: list             # list of (axis_a, axis_b) pairs
    eps: list = field(default=None)

    def __post_init__(self):
        self.E = [np.asarray(e, dtype=np.float64) for e in self.E]
        if self.eps is None:
            self.eps = default_eps(self.E)
        self.eps = [float(x) for x in self.eps]
        for e in self.E:
            if e.ndim != 1 or e.size == 0 or not np.all(e > 0) or not np.all(np.isfinite(e)):
                raise ValueError("every E_l must be a nonempty positive finite vector")
        for a, b in self.modalities:
            if a == b or not (0 <= a < len(self.E)) or not (0 <= b < len(self.E)):
                raise ValueError("bad modality")

    @property
    def n_axes(self):
        return len(self.E)

    @property
    def ranks(self):
        return [e.size for e in self.E]


def default_eps(E):
    return [1e-10 / float(np.max(e)) for e in E]


def _pairs(lam, a, b):
    return lam[a][:, None] + lam[b][None, :]


def nll(lam, prob: Problem) -> float:
    lin = sum(float(np.dot(e, l)) for e, l in zip(prob.E, lam))
    logs = 0.0
    for a, b in prob.modalities:
        logs += float(np.sum(np.log(_pairs(lam, a, b))))
    return 0.5 * (lin - logs)


def grad(lam, prob: Problem):
    g = [0.5 * e.copy() for e in prob.E]
    for a, b in prob.modalities:
        inv = 1.0 / _pairs(lam, a, b)
        g[a] -= 0.5 * inv.sum(axis=1)
        g[b] -= 0.5 * inv.sum(axis=0)
    return g


def hess_parts(lam, prob: Problem):
    """Diagonal per axis and cross blocks C[(a,b)][i,j] = 1/2 (lam_a,i + lam_b,j)^-2."""
    diag = [np.zeros_like(e) for e in prob.E]
    cross = {}
    for a, b in prob.modalities:
        inv2 = 0.5 / _pairs(lam, a, b) ** 2
        diag[a] += inv2.sum(axis=1)
        diag[b] += inv2.sum(axis=0)
        if (a, b) in cross:
            cross[(a, b)] = cross[(a, b)] + inv2
        else:
            cross[(a, b)] = inv2
    return diag, cross


def hess_dense(lam, prob: Problem):
    """The full Hessian as one dense matrix (small problems, for checks)."""
    off = np.concatenate([[0], np.cumsum(prob.ranks)])
    H = np.zeros((off[-1], off[-1]))
    diag, cross = hess_parts(lam, prob)
    for l in range(prob.n_axes):
        H[off[l]:off[l + 1], off[l]:off[l + 1]] += np.diag(diag[l])
    for (a, b), C in cross.items():
        H[off[a]:off[a + 1], off[b]:off[b + 1]] += C
        H[off[b]:off[b + 1], off[a]:off[a + 1]] += C.T
    return H


def flat_shift_space(axis_sets, ranks, traces, rel_tol: float = 1e-12):
    """Axis shifts c along which the NLL is constant: every modality's tuple sums
    unchanged (sum of c over its axes = 0, the null space of the modality-axis
    incidence matrix, Identifiability appendix) and the linear term unchanged
    (slope 1/2 sum_l c_l tr_l = 0).  The null space comes from the SVD; if every
    basis vector's slope vanishes (to rel_tol of sum_l |c_l| tr_l) the whole
    null space is flat, else the flat shifts are its subspace orthogonal to the
    slope vector.  Returned orthonormal in the metric <c, c'> = sum_l r_l c_l c'_l."""
    L = len(ranks)
    M = np.zeros((len(axis_sets), L))
    for t, m in enumerate(axis_sets):
        M[t, list(m)] = 1.0
    _, sv, Vt = np.linalg.svd(M)
    rank = int(np.sum(sv > 1e-12))
    N = Vt[rank:].T                                        # L x d, orthonormal columns
    if N.shape[1] == 0:
        return []
    tr = np.asarray(traces, dtype=np.float64)
    slope = N.T @ tr
    if np.any(np.abs(slope) > rel_tol * (np.abs(N).T @ tr)):
        # the coefficient vectors orthogonal to the slope vector
        _, _, Wt = np.linalg.svd(slope[None, :])
        N = N @ Wt[1:].T
    r = np.asarray(ranks, dtype=np.float64)
    out = []
    for c in N.T:
        for q in out:
            c = c - (np.sum(r * c * q)) * q
        nrm = math.sqrt(np.sum(r * c * c))
        if nrm > 1e-12:
            out.append(c / nrm)
    return out


def flat_directions(prob: Problem, rel_tol: float = 1e-12):
    """Axis shifts c (sum over each modality's axes = 0) along which the NLL is constant."""
    return flat_shift_space(prob.modalities, prob.ranks, [e.sum() for e in prob.E], rel_tol)


def _gauge_value(lam, c):
    return float(sum(c[l] * lam[l].sum() for l in range(len(lam))))


def cold_start(prob: Problem):
    """Algorithm 1's start: lambda^0 = 1/E, projected onto the box."""
    return [np.maximum(1.0 / e, eps) for e, eps in zip(prob.E, prob.eps)]


def nearest_feasible_shift(t_star, flats, lam, eps, max_iter: int = 10_000):
    """The gauge rule inside the box.  Moving lam by sum_q t_q c_q (c_q the flat
    directions, orthonormal in the gauge metric) changes the q-th gauge value by
    t_q and keeps every tuple sum, so the NLL and its gradient; it stays in the
    box while min_i lam_l,i + u_l >= eps_l for every axis, u_l = sum_q t_q c_q,l.
    Returns the t nearest to t_star (Euclidean) under those constraints.

    The primal active-set method for a strictly convex quadratic program
    (Nocedal and Wright, Numerical Optimization, Algorithm 16.3) from the
    feasible point t = 0 (no move) with an empty working set: the step to the
    minimiser on the working set's constraints taken as equalities, cut short
    by the first constraint it would violate (which joins the set), and, at a
    minimiser of the working set, the constraint with the most negative
    multiplier leaves; it stops when every multiplier is non-negative."""
    C = np.array(flats, dtype=np.float64)                  # q x L: column l is the normal of axis l
    q, L = C.shape
    m = np.array([float(x.min()) for x in lam])
    b = np.array(eps, dtype=np.float64) - m                # need C^T t >= b
    t_star = np.asarray(t_star, dtype=np.float64)
    t = np.zeros(q)
    W = []
    for _ in range(max_iter):
        g = t_star - t                                     # minus the objective's gradient
        tol = 1e-12 * (float(np.linalg.norm(g)) + float(np.linalg.norm(t_star)) + 1e-300)
        if W:
            A = C[:, W]
            mu = np.linalg.solve(A.T @ A, A.T @ g)         # g's component in the span of the normals
            p = g - A @ mu if len(W) < q else np.zeros(q)  # q independent normals span everything
        else:
            mu, p = np.zeros(0), g
        if np.linalg.norm(p) <= tol:
            # minimiser on the working set; the multipliers of t - t_star = A lambda are -mu
            size = mu * np.linalg.norm(C[:, W], axis=0) if W else mu
            if not W or np.all(size <= tol):
                return t
            W.pop(int(np.argmax(size)))
            continue
        alpha, block = 1.0, -1
        pn = float(np.linalg.norm(p))
        for l in range(L):
            if l in W:
                continue
            ap = float(C[:, l] @ p)
            # a normal in the span of the working set's (two axes whose
            # coefficients are proportional in every flat direction) is
            # orthogonal to p up to rounding: it cannot block
            if ap < -1e-12 * float(np.linalg.norm(C[:, l])) * pn:
                a_l = max(0.0, float(C[:, l] @ t - b[l])) / -ap     # slack / rate of its decrease
                if a_l < alpha:
                    alpha, block = a_l, l
        t = t + alpha * p
        if block >= 0:
            W.append(block)
    raise RuntimeError("gauge projection did not terminate")


def snap_to_bound(lam, u, eps):
    """lam_l + u_l per axis; a value the shift leaves within the rounding of the
    addition above its bound is put on the bound (the exact shift puts it
    there: the gauge projection is tight on that axis)."""
    out = []
    for l, x in enumerate(lam):
        y = x + u[l]
        tiny = 4 * np.finfo(float).eps * (np.abs(x) + abs(u[l]) + eps[l])
        out.append(np.where(y - eps[l] <= tiny, eps[l], y))
    return out


def _fix_gauge(lam, prob, flats):
    """Back to the gauge of the start 1/E along the flat directions, as near as the
    box allows (nearest_feasible_shift)."""
    if not flats:
        return lam
    target = cold_start(prob)
    t_star = [_gauge_value(target, c) - _gauge_value(lam, c) for c in flats]
    t = nearest_feasible_shift(t_star, flats, lam, prob.eps)
    u = np.array(flats).T @ t
    return snap_to_bound(lam, u, prob.eps)


def kkt_residual(lam, g, prob: Problem) -> float:
    res = 0.0
    for l in range(prob.n_axes):
        at = lam[l] <= prob.eps[l] * (1.0 + 1e-12)
        r = np.where(at, np.maximum(0.0, -g[l]), np.abs(g[l])) / (0.5 * prob.E[l])
        res = max(res, float(r.max()))
    return res


@dataclass
class SolveResult:
    lam: list
    iters: int
    kkt: float
    converged: bool
    n_pinned: list


def split_axes(prob: Problem):
    """(outer, inner): inner is the independent set of the modality graph with the
    largest total rank (enumerated; at most a few axes), outer the rest."""
    L = prob.n_axes
    best = None
    for mask in range(1 << L):
        inner = [l for l in range(L) if mask >> l & 1]
        if any(a in inner and b in inner for a, b in prob.modalities):
            continue
        w = sum(prob.ranks[l] for l in inner)
        if best is None or w > best[0]:
            best = (w, inner)
    inner = best[1]
    return [l for l in range(L) if l not in inner], inner


def _partners(prob: Problem, m):
    return [a if b == m else b for a, b in prob.modalities if m in (a, b)]


def inner_solve(lam_partners, E, eps, x0=None):
    """Minimisers x_j >= eps of 1/2 [E_j x - sum_i log(p_i + x)] for every j:
    the root of phi_j(x) = sum_i 1/(p_i + x) - E_j (convex and decreasing in x),
    or eps where phi_j(eps) <= 0.  Newton's method from a point left of the
    root converges monotonically from the left; a start x0 right of the root
    lands left of it after one step (the tangent of a convex function lies
    below it), and a step below eps restarts at eps."""
    p = np.asarray(lam_partners, dtype=np.longdouble)[:, None]
    E = np.asarray(E, dtype=np.longdouble)
    x = np.full(E.shape, eps, dtype=np.longdouble) if x0 is None else np.maximum(
        np.asarray(x0, dtype=np.longdouble), eps)

    def phi(x, sel):
        t = 1.0 / (p + x[None, :])
        return t.sum(axis=0) - E[sel], (t * t).sum(axis=0)

    allj = np.ones(E.shape, dtype=bool)
    v, dv = phi(np.full(E.shape, eps, dtype=np.longdouble), allj)
    pinned = v <= 0
    x[pinned] = eps
    # the iterations in FP64 (the same monotone Newton), then in extended
    # precision until the step is below its rounding
    p64, E64 = np.asarray(p, np.float64), np.asarray(E, np.float64)
    x64 = np.asarray(x, np.float64)
    todo = ~pinned
    for _ in range(400):
        if not todo.any():
            break
        t = 1.0 / (p64 + x64[todo][None, :])
        xn = x64[todo] + (t.sum(axis=0) - E64[todo]) / (t * t).sum(axis=0)
        xn = np.where(xn < eps, eps, xn)
        done = np.abs(xn - x64[todo]) <= 1e-13 * xn
        x64[todo] = xn
        idx = np.flatnonzero(todo)
        todo[idx[done]] = False
    x = np.asarray(x64, dtype=np.longdouble)
    todo = ~pinned
    for _ in range(50):
        if not todo.any():
            break
        v, dv = phi(x[todo], todo)
        step = v / dv                       # Newton: x - phi / phi' with phi' = -dv
        xn = x[todo] + step
        xn = np.where(xn < eps, eps, xn)
        done = np.abs(xn - x[todo]) <= 4 * np.finfo(np.longdouble).eps * xn
        x[todo] = xn
        idx = np.flatnonzero(todo)
        todo[idx[done]] = False
    return np.asarray(x, dtype=np.float64), pinned


def _sum_inv(lam_a, lam_b, axis):
    """sum over the other axis of 1/(lam_a,i + lam_b,j), in extended precision."""
    t = 1.0 / (np.asarray(lam_a, np.longdouble)[:, None] + np.asarray(lam_b, np.longdouble)[None, :])
    return np.asarray(t.sum(axis=axis), dtype=np.float64)


def grad_precise(lam, prob: Problem):
    """The gradient of the NLL with the pair sums in extended precision."""
    g = [0.5 * e.copy() for e in prob.E]
    for a, b in prob.modalities:
        g[a] -= 0.5 * _sum_inv(lam[a], lam[b], 1)
        g[b] -= 0.5 * _sum_inv(lam[a], lam[b], 0)
    return g


def _profile(prob: Problem, outer, inner):
    """evaluate(x, need_derivs) of the profiled NLL over the outer eigenvalues
    (concatenated), for oracle.newton.minimize_box; the last inner solution is
    kept in state["lam"] and reused as the next start."""
    off = np.concatenate([[0], np.cumsum([prob.ranks[l] for l in outer])])
    state = {"inner": {m: None for m in inner}, "lam": None}

    def full(x):
        lam = [None] * prob.n_axes
        for t, l in enumerate(outer):
            lam[l] = x[off[t]:off[t + 1]]
        pins = {}
        for m in inner:
            parts = np.concatenate([lam[l] for l in _partners(prob, m)])
            lam[m], pins[m] = inner_solve(parts, prob.E[m], prob.eps[m], state["inner"][m])
            state["inner"][m] = lam[m]
        return lam, pins

    def evaluate(x, need):
        lam, pins = full(x)
        state["lam"] = lam
        f = nll(lam, prob)
        if not need:
            return f
        g = grad_precise(lam, prob)
        gx = np.concatenate([g[l] for l in outer])
        diag, cross = hess_parts(lam, prob)
        n = int(off[-1])
        H = np.zeros((n, n))
        pos = {l: t for t, l in enumerate(outer)}
        for t, l in enumerate(outer):
            H[off[t]:off[t + 1], off[t]:off[t + 1]] += np.diag(diag[l])
        for (a, b), C in cross.items():
            if a in pos and b in pos:
                H[off[pos[a]]:off[pos[a] + 1], off[pos[b]]:off[pos[b] + 1]] += C
                H[off[pos[b]]:off[pos[b] + 1], off[pos[a]]:off[pos[a] + 1]] += C.T
        # Schur complement of the free inner coordinates (their Hessian block is diagonal)
        for m in inner:
            free = ~pins[m]
            B = np.zeros((n, int(free.sum())))
            for (a, b), C in cross.items():
                if b == m and a in pos:
                    B[off[pos[a]]:off[pos[a] + 1]] += C[:, free]
                elif a == m and b in pos:
                    B[off[pos[b]]:off[pos[b] + 1]] += C[free, :].T
            H -= (B / diag[m][free][None, :]) @ B.T
        return f, gx, H

    return evaluate, off, state


def solve_eigs(prob: Problem, warm=None, tol: float = 1e-15, max_iter: int = 500) -> SolveResult:
    """The minimiser over the box (profile likelihood, see the module header),
    started from Algorithm 1's 1/E or from ``warm`` (moved to the gauge and
    clipped to the box), then moved to the start's gauge."""
    flats = flat_directions(prob)
    lam0 = cold_start(prob)
    if warm is not None:
        w = _fix_gauge([np.asarray(x, dtype=np.float64).copy() for x in warm], prob, flats)
        lam0 = [np.maximum(l, eps) for l, eps in zip(w, prob.eps)]
    outer, inner = split_axes(prob)
    evaluate, off, state = _profile(prob, outer, inner)
    x0 = np.concatenate([lam0[l] for l in outer])
    lo = np.concatenate([np.full(prob.ranks[l], prob.eps[l]) for l in outer])
    scale = np.concatenate([0.5 * prob.E[l] for l in outer])
    x = x0
    it = 0
    for _round in range(4):
        # minimise, then move to the start's gauge along the flat directions; the
        # projection's own rounding can lift an eigenvalue off its bound by a
        # few ulps of the shift, so the solve resumes until the point is stable
        x, k_it, _, _ = minimize_box(evaluate, x, lo, scale, tol, max_iter)
        it += k_it
        evaluate(x, False)
        lam = [np.array(l, dtype=np.float64) for l in state["lam"]]
        lam = [np.maximum(l, e) for l, e in zip(_fix_gauge(lam, prob, flats), prob.eps)]
        kkt = kkt_residual(lam, grad_precise(lam, prob), prob)
        x = np.concatenate([lam[l] for l in outer])
        if kkt <= max(tol, 1e-14) or not flats:
            break
    pinned = [int(np.sum(l <= e * (1 + 1e-12))) for l, e in zip(lam, prob.eps)]
    return SolveResult(lam, it, kkt, kkt <= max(tol, 1e-14), pinned)


def projected_gradient(prob: Problem, tol: float = 1e-9, max_iter: int = 200_000):
    """Projected gradient descent of the NLL over the box from Algorithm 1's start
    1/E: lambda <- max(lambda - t g, eps), the step t grown by 2 after an accepted
    step and cut by 4 until the NLL decreases by at least a tenth of the
    first-order prediction along the projected move.  Slow; small cross-checks."""
    lam = cold_start(prob)
    t = 1.0
    it = 0
    while it < max_iter:
        g = grad(lam, prob)
        if kkt_residual(lam, g, prob) <= tol:
            break
        f0 = nll(lam, prob)
        while True:
            trial = [np.maximum(l - t * gl, e) for l, gl, e in zip(lam, g, prob.eps)]
            move = sum(float(np.dot(gl, tl - l)) for gl, tl, l in zip(g, trial, lam))
            if nll(trial, prob) <= f0 + 0.1 * move:
                break
            t *= 0.25
            if t < 1e-300:
                return lam, it
        lam = trial
        t *= 2.0
        it += 1
    return lam, it
