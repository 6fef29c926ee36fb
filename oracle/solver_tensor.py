"""Eigenvalue maximum-likelihood estimate for modalities of any number of
axes (tensor-variate data).  Test infrastructure only.

The model equation for a modality gamma with axes l_1..l_K: with the
eigenvectors fixed to those of the S_l (Theorem 1), the Kronecker sum of the
axes' precisions has eigenvalues lambda_{l_1,i_1} + ... + lambda_{l_K,i_K} over
all index tuples (the derivation appendix: r_forall = prod r_l), so

    NLL = 1/2 [ sum_l sum_i E_l,i lambda_l,i
                - sum_gamma sum_{tuples of gamma} log(sum_{l in gamma} lambda_l,i_l) ]

and the eigenvalue-gradient Proposition gives

    dNLL/dlambda_l,i = 1/2 ( E_l,i - sum_{gamma containing l} sum_{tuples with i_l = i} 1/s ),

with s the tuple's sum.  The Hessian has a diagonal block per axis and, for
every two axes of a modality, the cross block sum over the remaining axes of
1/2 s^-2.  Two-axis modalities reduce this to the pair model of
``oracle.solver``.

Readings and stopping rule as ``oracle.solver`` (box lambda >= eps, scaled
KKT, the start's gauge restored along flat directions).  Method: the whole
problem as one dense projected Newton (``oracle.newton.minimize_box``:
Bertsekas' active set and projection-arc search, a Levenberg-Marquardt term
proportional to the gradient), with the gradient's tuple sums taken in
extended precision so that the scaled KKT residual reaches ~1e-15.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .newton import minimize_box
from .solver import default_eps, flat_shift_space, nearest_feasible_shift, snap_to_bound


@dataclass
class TensorProblem:
    E: list                      # per axis: float64 array, descending, positive
    modalities: list             # list of tuples of distinct axes (length >= 2)
    eps: list = field(default=None)

    def __post_init__(self):
        self.E = [np.asarray(e, dtype=np.float64) for e in self.E]
        if self.eps is None:
            self.eps = default_eps(self.E)
        self.eps = [float(x) for x in self.eps]
        for e in self.E:
            if e.ndim != 1 or e.size == 0 or not np.all(e > 0) or not np.all(np.isfinite(e)):
                raise ValueError("every E_l must be a nonempty positive finite vector")
        self.modalities = [tuple(int(a) for a in m) for m in self.modalities]
        for m in self.modalities:
            if len(m) < 2 or len(set(m)) != len(m) or not all(0 <= a < len(self.E) for a in m):
                raise ValueError("bad modality")

    @property
    def n_axes(self):
        return len(self.E)

    @property
    def ranks(self):
        return [e.size for e in self.E]


def _sums(lam, m):
    """The tuple sums of modality m as an array of shape (r_{m_0}, ..., r_{m_K-1})."""
    K = len(m)
    s = 0.0
    for t, a in enumerate(m):
        shape = [1] * K
        shape[t] = -1
        s = s + lam[a].reshape(shape)
    return s


def nll(lam, prob: TensorProblem) -> float:
    lin = sum(float(np.dot(e, l)) for e, l in zip(prob.E, lam))
    logs = sum(float(np.sum(np.log(_sums(lam, m)))) for m in prob.modalities)
    return 0.5 * (lin - logs)


def grad(lam, prob: TensorProblem):
    g = [0.5 * e.copy() for e in prob.E]
    for m in prob.modalities:
        inv = 1.0 / _sums(lam, m)
        for t, a in enumerate(m):
            g[a] -= 0.5 * inv.sum(axis=tuple(u for u in range(len(m)) if u != t))
    return g


def hess_dense(lam, prob: TensorProblem):
    off = np.concatenate([[0], np.cumsum(prob.ranks)])
    H = np.zeros((off[-1], off[-1]))
    for m in prob.modalities:
        inv2 = 0.5 / _sums(lam, m) ** 2
        K = len(m)
        for t, a in enumerate(m):
            d = inv2.sum(axis=tuple(u for u in range(K) if u != t))
            H[off[a]:off[a + 1], off[a]:off[a + 1]] += np.diag(d)
            for t2 in range(t + 1, K):
                b = m[t2]
                C = inv2.sum(axis=tuple(u for u in range(K) if u not in (t, t2)))
                H[off[a]:off[a + 1], off[b]:off[b + 1]] += C
                H[off[b]:off[b + 1], off[a]:off[a + 1]] += C.T
    return H


def flat_directions(prob: TensorProblem, rel_tol: float = 1e-12):
    """Axis shifts c (sum over each modality's axes = 0) along which the NLL is
    constant (oracle.solver.flat_shift_space)."""
    return flat_shift_space(prob.modalities, prob.ranks, [e.sum() for e in prob.E], rel_tol)


def cold_start(prob: TensorProblem):
    return [np.maximum(1.0 / e, eps) for e, eps in zip(prob.E, prob.eps)]


def _fix_gauge(lam, prob, flats):
    """Back to the gauge of the start 1/E along the flat directions, as near as the
    box allows (oracle.solver.nearest_feasible_shift)."""
    if not flats:
        return lam
    target = cold_start(prob)
    t_star = [sum(c[l] * (target[l].sum() - lam[l].sum()) for l in range(len(lam))) for c in flats]
    t = nearest_feasible_shift(t_star, flats, lam, prob.eps)
    u = np.array(flats).T @ t
    return snap_to_bound(lam, u, prob.eps)


def kkt_residual(lam, g, prob: TensorProblem) -> float:
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


def grad_precise(lam, prob: TensorProblem):
    """The gradient with the tuple sums in extended precision."""
    g = [0.5 * e.copy() for e in prob.E]
    for m in prob.modalities:
        inv = 1.0 / _sums([np.asarray(x, np.longdouble) for x in lam], m)
        for t, a in enumerate(m):
            g[a] -= np.asarray(0.5 * inv.sum(axis=tuple(u for u in range(len(m)) if u != t)), np.float64)
    return g


def solve_eigs(prob: TensorProblem, warm=None, tol: float = 1e-15, max_iter: int = 500) -> SolveResult:
    """The minimiser over the box by one dense projected Newton (see the module
    header) from the cold start 1/E or ``warm`` (moved to the gauge and clipped),
    then moved to the start's gauge."""
    flats = flat_directions(prob)
    lam0 = cold_start(prob)
    if warm is not None:
        w = _fix_gauge([np.asarray(x, dtype=np.float64).copy() for x in warm], prob, flats)
        lam0 = [np.maximum(l, e) for l, e in zip(w, prob.eps)]
    off = np.concatenate([[0], np.cumsum(prob.ranks)])
    L = prob.n_axes

    def split(x):
        return [x[off[l]:off[l + 1]] for l in range(L)]

    def evaluate(x, need):
        lam = split(x)
        f = nll(lam, prob)
        if not need:
            return f
        return f, np.concatenate(grad_precise(lam, prob)), hess_dense(lam, prob)

    lo = np.concatenate([np.full(prob.ranks[l], prob.eps[l]) for l in range(L)])
    scale = np.concatenate([0.5 * e for e in prob.E])
    x = np.concatenate(lam0)
    it = 0
    for _round in range(4):
        # minimise, then move to the start's gauge along the flat directions; the
        # projection's own rounding can lift an eigenvalue off its bound by a
        # few ulps of the shift, so the solve resumes until the point is stable
        x, k_it, _, _ = minimize_box(evaluate, x, lo, scale, tol, max_iter)
        it += k_it
        lam = [np.maximum(l, e) for l, e in zip(_fix_gauge([v.copy() for v in split(x)], prob, flats), prob.eps)]
        kkt = kkt_residual(lam, grad_precise(lam, prob), prob)
        x = np.concatenate(lam)
        if kkt <= max(tol, 1e-14) or not flats:
            break
    pinned = [int(np.sum(l <= e * (1 + 1e-12))) for l, e in zip(lam, prob.eps)]
    return SolveResult(lam, it, kkt, kkt <= max(tol, 1e-14), pinned)
