"""Pins of the tensor-variate eigenvalue MLE oracle: the NLL against the log
determinant of explicitly built Kronecker sums, the gradient and Hessian
against finite differences, reduction to the (pinned) pair solver for
two-axis modalities, and two closed forms of single three-axis modalities."""
import numpy as np
import pytest

from oracle import solver as S
from oracle import solver_tensor as T


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
