"""Pins of the tensor-variate eigenvalue MLE oracle: the NLL against the log
determinant of explicitly built Kronecker sums, the gradient and Hessian
against finite differences, reduction to the (pinned) pair solver for
two-axis modalities, and two closed forms of single three-axis modalities."""
import numpy as np
import pytest

from oracle import solver as S
from oracle import solver_tensor as T

from ._tensor_inputs import low_rank_tensor_spectra


def _kron_sum(diags):
    n = int(np.prod([d.size for d in diags]))
    out = np.zeros((n, n))
    for t, d in enumerate(diags):
        M = np.ones((1, 1))
        for u, e in enumerate(diags):
            M = np.kron(M, np.diag(d) if u == t else np.eye(e.size))
        out += M
    return out


def test_nll_is_the_kronecker_log_determinant():
    rng = np.random.default_rng(1)
    E = [rng.uniform(0.5, 3, 3), rng.uniform(0.5, 3, 2), rng.uniform(0.5, 3, 4), rng.uniform(0.5, 3, 2)]
    mods = [(0, 1, 2), (1, 3), (0, 2, 3)]
    prob = T.TensorProblem(E, mods)
    lam = [rng.uniform(0.2, 2, e.size) for e in E]
    lin = sum(float(e @ l) for e, l in zip(E, lam))
    logdet = sum(np.linalg.slogdet(_kron_sum([lam[a] for a in m]))[1] for m in mods)
    assert abs(T.nll(lam, prob) - 0.5 * (lin - logdet)) < 1e-11


def test_gradient_and_hessian_by_finite_differences():
    rng = np.random.default_rng(2)
    E = [rng.uniform(0.5, 3, 3), rng.uniform(0.5, 3, 2), rng.uniform(0.5, 3, 3)]
    prob = T.TensorProblem(E, [(0, 1, 2), (0, 2)])
    lam = [rng.uniform(0.3, 2, e.size) for e in E]
    flat = np.concatenate(lam)
    off = np.concatenate([[0], np.cumsum(prob.ranks)])
    split = lambda x: [x[off[l]:off[l + 1]] for l in range(3)]
    h = 1e-6
    g = np.concatenate(T.grad(lam, prob))
    gn = np.array([(T.nll(split(flat + h * np.eye(flat.size)[q]), prob) -
                    T.nll(split(flat - h * np.eye(flat.size)[q]), prob)) / (2 * h) for q in range(flat.size)])
    np.testing.assert_allclose(g, gn, rtol=1e-6, atol=1e-8)
    H = T.hess_dense(lam, prob)
    Hn = np.array([(np.concatenate(T.grad(split(flat + h * np.eye(flat.size)[q]), prob)) -
                    np.concatenate(T.grad(split(flat - h * np.eye(flat.size)[q]), prob))) / (2 * h)
                   for q in range(flat.size)])
    np.testing.assert_allclose(H, Hn, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("seed,ranks,mods", [
    (3, (5, 7), [(0, 1)]),
    (4, (6, 4, 5), [(0, 1), (0, 2)]),
    (5, (4, 4, 3, 5), [(0, 1), (1, 2), (2, 3), (0, 3)]),
])
def test_two_axis_modalities_reduce_to_the_pair_solver(seed, ranks, mods):
    rng = np.random.default_rng(seed)
    E = [np.sort(rng.uniform(0.2, 5.0, r))[::-1] for r in ranks]
    a = S.solve_eigs(S.Problem(E, mods))
    b = T.solve_eigs(T.TensorProblem(E, mods))
    assert a.converged and b.converged
    for x, y in zip(a.lam, b.lam):
        np.testing.assert_allclose(y, x, rtol=1e-9, atol=1e-12 * float(np.max(x)))


def test_closed_form_single_rank_one_triple():
    """One three-axis modality of rank-one axes, E_1 < E_2, E_3: the two larger
    pin at eps and lambda_1 = 1/E_1 - eps_2 - eps_3 (stationarity of the free one)."""
    E = [np.array([0.5]), np.array([2.0]), np.array([3.0])]
    prob = T.TensorProblem(E, [(0, 1, 2)])
    res = T.solve_eigs(prob)
    assert res.converged
    eps = prob.eps
    assert res.lam[1][0] == eps[1] and res.lam[2][0] == eps[2]
    assert abs(res.lam[0][0] - (1 / 0.5 - eps[1] - eps[2])) <= 1e-12 * 2.0


def test_closed_form_balanced_triple_keeps_the_start_gauge():
    """Equal rank-one spectra: the minimisers form the plane lambda_1 + lambda_2 +
    lambda_3 = 1/E; the start's gauge (equal shifts) picks 1/(3E) each."""
    E = [np.array([1.5])] * 3
    res = T.solve_eigs(T.TensorProblem(E, [(0, 1, 2)]))
    assert res.converged
    for l in res.lam:
        assert abs(l[0] - 1 / 4.5) < 1e-12


def test_kkt_and_shared_axes_three_axis_graph():
    rng = np.random.default_rng(6)
    ranks = (6, 5, 4, 7)
    E = [np.sort(rng.uniform(0.2, 5.0, r))[::-1] for r in ranks]
    prob = T.TensorProblem(E, [(0, 1, 2), (0, 3), (1, 2, 3)])
    res = T.solve_eigs(prob)
    assert res.converged and res.kkt <= 1e-12
    assert all(np.all(l >= e) for l, e in zip(res.lam, prob.eps))


def _spectra(shape, rank, seed):
    return low_rank_tensor_spectra(shape, rank, seed)


def _projection_by_enumeration(t_star, C, b):
    """Brute force: the feasible projection of t_star onto every affine set where
    a linearly independent choice of constraints holds with equality, nearest wins."""
    import itertools
    q, L = C.shape
    best, best_d = None, np.inf
    for k in range(0, min(q, L) + 1):
        for A in itertools.combinations(range(L), k):
            t = np.array(t_star, dtype=np.float64)
            if k:
                M = C[:, list(A)]
                if np.linalg.matrix_rank(M) < k:
                    continue
                t = t - M @ np.linalg.solve(M.T @ M, M.T @ t - b[list(A)])
            if np.all(C.T @ t - b >= -1e-10 * (1 + np.abs(b))):
                d = float(np.sum((t - t_star) ** 2))
                if d < best_d:
                    best, best_d = t, d
    return best


@pytest.mark.parametrize("seed", range(40))
def test_gauge_projection_against_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    L = int(rng.integers(2, 9))
    q = int(rng.integers(1, L))
    C = np.linalg.qr(rng.standard_normal((L, q)))[0].T
    lam = [rng.uniform(0.0, 2.0, 4) + 1e-3 for _ in range(L)]
    eps = [1e-3] * L
    for l in rng.choice(L, size=int(rng.integers(0, 3)), replace=False):
        lam[l][0] = eps[l]                                  # an axis already at its bound
    t_star = rng.standard_normal(q) * 10.0 ** rng.uniform(-2, 2)
    b = np.array(eps) - np.array([x.min() for x in lam])
    t = S.nearest_feasible_shift(t_star, list(C), lam, eps)
    ref = _projection_by_enumeration(t_star, C, b)
    np.testing.assert_allclose(t, ref, atol=1e-10 * (1 + np.abs(t_star).max()))


@pytest.mark.parametrize("seed", range(6))
def test_nearest_feasible_shift_is_the_qp_solution(seed):
    """The gauge rule's projection against a general constrained optimiser, up
    to the many-axis shape of a shared frame axis with 20 row/column pairs."""
    from scipy.optimize import LinearConstraint, minimize
    rng = np.random.default_rng(seed)
    L = int(rng.integers(2, 7)) if seed < 4 else 41
    q = int(rng.integers(1, L)) if seed < 4 else 21
    C = np.linalg.qr(rng.standard_normal((L, q)))[0].T            # q x L
    lam = [rng.uniform(0.1, 2.0, 5) for _ in range(L)]
    eps = [1e-3] * L
    t_star = rng.standard_normal(q) * 3.0
    t = S.nearest_feasible_shift(t_star, list(C), lam, eps)
    b = np.array(eps) - np.array([x.min() for x in lam])
    res = minimize(lambda x: np.sum((x - t_star) ** 2), np.zeros(q), jac=lambda x: 2 * (x - t_star),
                   hess=lambda x: 2 * np.eye(q), constraints=[LinearConstraint(C.T, b, np.inf)],
                   method="trust-constr", options={"gtol": 1e-12, "xtol": 1e-14, "maxiter": 5000})
    assert np.all(C.T @ t - b >= -1e-12)
    assert np.all(C.T @ res.x - b >= -1e-8)
    # strictly convex: a feasible point no worse than the reference is the optimum
    assert np.sum((t - t_star) ** 2) <= np.sum((res.x - t_star) ** 2) + 1e-9
    np.testing.assert_allclose(t, res.x, atol=1e-4)
    # KKT certificate: t - t_star = sum over active constraints of mu_l C_l, mu >= 0
    from scipy.optimize import nnls
    slack = C.T @ t - b
    A = np.flatnonzero(slack <= 1e-10 * (1 + np.abs(b)))
    if A.size == 0:
        np.testing.assert_allclose(t, t_star, atol=1e-14)
    else:
        mu, rnorm = nnls(C[:, A], t - t_star)
        assert rnorm <= 1e-10 * (1 + np.linalg.norm(t_star))


@pytest.mark.parametrize("shape,mods", [((6, 5, 4), [(0, 1, 2)]), ((5, 4, 3, 3), [(0, 1, 2, 3)]),
                                        ((6, 5, 4), [(0, 1, 2), (0, 2)])])
def test_minimum_matches_a_general_bounded_optimiser(shape, mods):
    """Balanced tensor spectra (the start's gauge leaves the box): the solve's NLL
    is the minimum L-BFGS-B finds over the same box, the solution is in the box,
    and its tuple sums are gauge-free (the same from a perturbed warm start)."""
    from scipy.optimize import minimize
    E = _spectra(shape, 2, 7)
    if len(mods) > 1:                       # a second modality over axes 0 and 2
        E = [E[0], E[1], E[2]]
    prob = T.TensorProblem(E, mods)
    res = T.solve_eigs(prob)
    assert res.converged and res.kkt <= 1e-12
    assert all(np.all(l >= e) for l, e in zip(res.lam, prob.eps))
    off = np.concatenate([[0], np.cumsum(prob.ranks)])
    split = lambda x: [x[off[l]:off[l + 1]] for l in range(prob.n_axes)]
    f = lambda x: T.nll(split(x), prob)
    gfun = lambda x: np.concatenate(T.grad(split(x), prob))
    x0 = np.concatenate(T.cold_start(prob))
    bounds = [(e, None) for l, e in enumerate(prob.eps) for _ in range(prob.ranks[l])]
    ref = minimize(f, x0, jac=gfun, bounds=bounds, method="L-BFGS-B",
                   options={"ftol": 1e-16, "gtol": 1e-14, "maxiter": 50000, "maxcor": 50})
    f_ours = T.nll(res.lam, prob)
    assert f_ours <= ref.fun + 1e-9 * abs(ref.fun)
    assert abs(f_ours - ref.fun) <= 1e-7 * abs(ref.fun)
    rng = np.random.default_rng(1)
    for m in mods:
        s_ref = T._sums(res.lam, m)
        s_lb = T._sums(split(ref.x), m)
        np.testing.assert_allclose(s_lb, s_ref, rtol=2e-3)


def test_gauge_is_the_start_when_feasible_and_a_bound_otherwise():
    """Equal rank-one spectra: the start's gauge is inside the box and is kept
    exactly.  Balanced tensor spectra where it is not: the result's gauge is the
    nearest feasible one, so some axis' smallest eigenvalue sits at its bound."""
    E = _spectra((20, 32, 32), 4, 1)
    prob = T.TensorProblem(E, [(0, 1, 2)])
    res = T.solve_eigs(prob)
    assert res.converged
    flats = T.flat_directions(prob)
    assert len(flats) == 2
    target = T.cold_start(prob)
    gap = [sum(c[l] * (target[l].sum() - res.lam[l].sum()) for l in range(3)) for c in flats]
    if max(abs(x) for x in gap) > 1e-9 * sum(t.sum() for t in target):
        assert any(abs(l.min() - e) <= 1e-12 * l.max() for l, e in zip(res.lam, prob.eps))


@pytest.mark.parametrize("ranks,mods,balanced_pairs,want", [
    ((4, 3, 5), [(0, 1, 2)], False, 1),                       # one modality, K = 3, unequal traces: K - 2
    ((4, 3, 5, 2), [(0, 1, 2, 3)], False, 2),                 # K = 4: K - 2
    ((6, 6, 4, 5, 3), [(0, 1), (2, 3, 4)], True, 2),          # balanced pair (1) + unbalanced triple (1)
    ((6, 6, 4, 5, 3), [(0, 1), (2, 3, 4)], False, 2),         # both unbalanced: null space 3, less 1
    ((5, 7, 4), [(0, 1), (0, 2)], False, 0),                  # shared axis, one null direction, sloped
    ((4, 4, 3, 3), [(0, 1), (1, 2), (2, 3), (0, 3)], False, 0),  # even cycle, sloped
])
def test_flat_shift_space_dimension_and_constancy(ranks, mods, balanced_pairs, want):
    """The flat shifts: their number (by hand: the null space of the incidence
    matrix, less one when some null shift has a slope), and the NLL is constant
    along each of them, evaluated from its definition."""
    rng = np.random.default_rng(sum(ranks))
    E = [np.sort(rng.uniform(0.5, 4.0, r))[::-1].copy() for r in ranks]
    if balanced_pairs:                                        # equal traces on the pair modality's axes
        E[1] = E[0].copy()
    prob = T.TensorProblem(E, mods)
    flats = T.flat_directions(prob)
    assert len(flats) == want
    lam = [rng.uniform(1.0, 2.0, r) for r in ranks]
    f0 = T.nll(lam, prob)
    r = np.array(ranks, dtype=np.float64)
    for i, c in enumerate(flats):
        assert abs(np.sum(r * c * c) - 1.0) < 1e-12
        for j in range(i):
            assert abs(np.sum(r * c * flats[j])) < 1e-12
        for t in (-0.3, 0.2, 0.5):
            moved = [l + t * c[a] for a, l in enumerate(lam)]
            assert abs(T.nll(moved, prob) - f0) <= 1e-11 * abs(f0)


def test_flat_shift_space_does_not_depend_on_the_basis():
    """Same axis sets listed in another order (a different SVD basis): the same
    flat subspace (equal projectors in the gauge metric)."""
    rng = np.random.default_rng(4)
    ranks = (5, 4, 6, 3, 4)
    E = [np.sort(rng.uniform(0.5, 4.0, r))[::-1].copy() for r in ranks]
    a = T.flat_directions(T.TensorProblem(E, [(0, 1), (2, 3, 4)]))
    b = T.flat_directions(T.TensorProblem(E, [(4, 3, 2), (1, 0)]))
    P = lambda F: sum(np.outer(c, c) for c in F) @ np.diag(ranks)
    assert len(a) == len(b) == 2
    np.testing.assert_allclose(P(a), P(b), atol=1e-12)
