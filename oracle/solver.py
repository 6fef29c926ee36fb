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

Method: projected Newton for bound constraints (Bertsekas 1982) with a
Levenberg-Marquardt damping that vanishes at the solution, an Armijo search
along the projection arc, Newton systems solved by a Schur complement that
eliminates an independent set of axes (whose Hessian blocks are diagonal).
``alg1_gradient_descent`` is the literal gradient descent of Algorithm 1 for
small cross-checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


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


def _hub_axes(prob: Problem):
    """Minimum-size vertex cover of the modality graph; the rest is an independent set."""
    L = prob.n_axes
    best = None
    for mask in range(1 << L):
        K = [l for l in range(L) if mask >> l & 1]
        if all(a in K or b in K for a, b in prob.modalities):
            w = sum(prob.ranks[l] for l in K)
            if best is None or w < best[0]:
                best = (w, K)
    return best[1]


def newton_direction(lam, g, free, prob: Problem, rho: float):
    """Solve (H_FF + rho diag(H_FF)) d_F = -g_F by a Schur complement on the hub axes."""
    diag, cross = hess_parts(lam, prob)
    K = _hub_axes(prob)
    leaves = [l for l in range(prob.n_axes) if l not in K]
    fidx = [np.nonzero(f)[0] for f in free]
    dd = [d * (1.0 + rho) for d in diag]
    # hub system over free hub coordinates
    koff = np.concatenate([[0], np.cumsum([fidx[l].size for l in K])])
    nk = int(koff[-1])
    S = np.zeros((nk, nk))
    rhs = np.zeros(nk)
    pos = {l: t for t, l in enumerate(K)}
    for t, l in enumerate(K):
        sl = slice(koff[t], koff[t + 1])
        S[sl, sl] += np.diag(dd[l][fidx[l]])
        rhs[sl] = -g[l][fidx[l]]

    def block(a, b):  # cross block rows of axis a, cols of axis b (free coords only)
        if (a, b) in cross:
            C = cross[(a, b)]
        else:
            C = cross[(b, a)].T
        return C[np.ix_(fidx[a], fidx[b])]

    for (a, b) in cross:
        if a in pos and b in pos:
            C = block(a, b)
            S[koff[pos[a]]:koff[pos[a] + 1], koff[pos[b]]:koff[pos[b] + 1]] += C
            S[koff[pos[b]]:koff[pos[b] + 1], koff[pos[a]]:koff[pos[a] + 1]] += C.T
    for m in leaves:
        Dm = dd[m][fidx[m]]
        gm = -g[m][fidx[m]]
        partners = [l for l in K if (l, m) in cross or (m, l) in cross]
        Bs = {l: block(l, m) for l in partners}
        for l in partners:
            sl = slice(koff[pos[l]], koff[pos[l] + 1])
            rhs[sl] -= Bs[l] @ (gm / Dm)
            for l2 in partners:
                sl2 = slice(koff[pos[l2]], koff[pos[l2] + 1])
                S[sl, sl2] -= (Bs[l] / Dm[None, :]) @ Bs[l2].T
    dK = np.linalg.solve(S, rhs) if nk else np.zeros(0)
    d = [np.zeros_like(e) for e in prob.E]
    for t, l in enumerate(K):
        d[l][fidx[l]] = dK[koff[t]:koff[t + 1]]
    for m in leaves:
        Dm = dd[m][fidx[m]]
        acc = -g[m][fidx[m]].copy()
        for l in K:
            if (l, m) in cross or (m, l) in cross:
                acc -= block(l, m).T @ d[l][fidx[l]]
        d[m][fidx[m]] = acc / Dm
    return d


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
        for l in range(L):
            if l in W:
                continue
            ap = float(C[:, l] @ p)
            if ap < 0.0:
                a_l = max(0.0, float(C[:, l] @ t - b[l])) / -ap     # slack / rate of its decrease
                if a_l < alpha:
                    alpha, block = a_l, l
        t = t + alpha * p
        if block >= 0:
            W.append(block)
    raise RuntimeError("gauge projection did not terminate")


def _fix_gauge(lam, prob, flats):
    """Back to the gauge of the start 1/E along the flat directions, as near as the
    box allows (nearest_feasible_shift)."""
    if not flats:
        return lam
    target = cold_start(prob)
    t_star = [_gauge_value(target, c) - _gauge_value(lam, c) for c in flats]
    t = nearest_feasible_shift(t_star, flats, lam, prob.eps)
    u = np.array(flats).T @ t
    return [l + u[i] for i, l in enumerate(lam)]


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


STEP_SHRINK = 64.0


def solve_eigs(prob: Problem, warm=None, tol: float = 1e-12, max_iter: int = 200) -> SolveResult:
    """Projected Newton from the cold start 1/E, or from a warm start (moved to the
    gauge and clipped to the box) when its NLL is not above the cold start's.

    The minimiser does not depend on the path.  Along flat directions the NLL is
    constant: steps may drift along them, and the result is moved back to the
    start's gauge at the end."""
    flats = flat_directions(prob)
    lam = cold_start(prob)
    if warm is not None:
        # a supplied start is used when it is at least as good as 1/E
        w = _fix_gauge([np.asarray(x, dtype=np.float64).copy() for x in warm], prob, flats)
        w = [np.maximum(l, eps) for l, eps in zip(w, prob.eps)]
        if nll(w, prob) <= nll(lam, prob):
            lam = w
    eps = prob.eps
    it = 0
    g = grad(lam, prob)
    kkt = kkt_residual(lam, g, prob)
    for _round in range(3):
        stalled = False
        while kkt > tol and it < max_iter:
            it += 1
            f0 = nll(lam, prob)
            diag, _ = hess_parts(lam, prob)
            # coordinates within a diagonal-Newton step of their bound that want to go down
            active = []
            for l in range(prob.n_axes):
                reach = np.minimum(1e-3 * lam[l], g[l] / diag[l])
                active.append((lam[l] - eps[l] <= reach) & (g[l] > 0))
            free = [~a for a in active]
            rho = min(1e-2, kkt)
            d = newton_direction(lam, g, free, prob, rho)
            for l in range(prob.n_axes):
                d[l][active[l]] = -g[l][active[l]] / diag[l][active[l]]
            # floor of the step: an active coordinate may go to its bound, a free one
            # may shrink by at most STEP_SHRINK per iteration (a coupled Newton step
            # can overshoot far below the optimum, and recovery from the bound
            # doubles the value per iteration at best)
            floor = [np.where(active[l], eps[l], np.maximum(eps[l], lam[l] / STEP_SHRINK))
                     for l in range(prob.n_axes)]
            alpha = 1.0
            accepted = False
            for _ in range(60):
                trial = [np.maximum(lam[l] + alpha * d[l], floor[l]) for l in range(prob.n_axes)]
                pred = 0.0
                for l in range(prob.n_axes):
                    pred += alpha * float(np.dot(g[l][free[l]], d[l][free[l]]))
                    pred += float(np.dot(g[l][active[l]], trial[l][active[l]] - lam[l][active[l]]))
                f1 = nll(trial, prob)
                if f1 <= f0 + 1e-4 * pred or abs(pred) <= 1e-13 * (abs(f0) + 1.0):
                    accepted = True
                    break
                alpha *= 0.5
            if not accepted:
                stalled = True
                break
            lam = trial
            g = grad(lam, prob)
            kkt = kkt_residual(lam, g, prob)
        # back to the start's gauge along the flat directions; resume if that
        # moved the point off the tolerance (rounding of the shift, the box)
        lam = [np.maximum(l, e) for l, e in zip(_fix_gauge(lam, prob, flats), eps)]
        g = grad(lam, prob)
        kkt = kkt_residual(lam, g, prob)
        if kkt <= tol or it >= max_iter or stalled or not flats:
            break
    pinned = [int(np.sum(l <= e * (1 + 1e-12))) for l, e in zip(lam, eps)]
    return SolveResult(lam, it, kkt, kkt <= tol, pinned)


def alg1_gradient_descent(prob: Problem, tol: float = 1e-9, max_iter: int = 200_000):
    """Algorithm 1 as printed: lambda^0 = 1/E, mu = 1, lambda <- lambda - mu * grad,
    with mu halved while some modality's sum of smallest eigenvalues is below the
    sum of its eps, or while the step would not lower the NLL ("decrease mu if
    needed").  For small cross-checks only."""
    lam = [1.0 / e for e in prob.E]
    mu = 1.0
    it = 0
    while it < max_iter:
        g = grad(lam, prob)
        if kkt_residual(lam, g, prob) <= tol:
            break
        f0 = nll(lam, prob)
        while True:
            trial = [l - mu * gl for l, gl in zip(lam, g)]
            ok = all(trial[a].min() + trial[b].min() >= prob.eps[a] + prob.eps[b]
                     for a, b in prob.modalities)
            if ok and nll(trial, prob) < f0:
                break
            mu *= 0.5
            if mu < 1e-300:
                return lam, it
        lam = trial
        it += 1
    return lam, it
