"""Parity of gmgm_solve_eigs_tensor (HIP, through the C ABI) with the CPU
oracle's dense projected-Newton solve for modalities of any number of axes.

Bar: every eigenvalue within 1e-10 relative plus 1e-12 of its axis' largest
(an eigenvalue that the gauge rule puts on its bound is there only up to the
rounding of the shift, so bound membership is compared through the values);
the GPU's own KKT residual <= 1e-12.  At the size of the paper's COIL-20 run
with every principal component (41 axes, 5192 unknowns), where the oracle's
dense solve takes minutes, the GPU result is checked by properties that hold
at any size, in FP64 on the CPU: the scaled KKT residual of the oracle's
gradient at the GPU's point, the box, and the gauge rule (the projection from
that point does not move it).
"""
import numpy as np
import pytest

from oracle import solver as S
from oracle import solver_tensor as T

from ._tensor_inputs import coil_like_spectra, low_rank_tensor_spectra

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _gpu_solve(lib, E, mods, eps=None, warm=None, **kw):
    r = lib.solve_eigs_tensor([_dev(e) for e in E], mods, eps=eps,
                              warm=None if warm is None else [_dev(w) for w in warm], **kw)
    return [x.cpu().numpy() for x in r.lam], r.info


def _compare(prob, ref_lam, lam, info, label):
    assert info["converged"] and info["kkt"] <= 1e-12, (label, info)
    for l in range(prob.n_axes):
        a, b = lam[l], ref_lam[l]
        err = np.abs(a - b) - (1e-10 * np.abs(b) + 1e-12 * np.max(b))
        assert np.all(err <= 0), (label, l, float(np.max(np.abs(a - b) / np.abs(b))))
        assert np.all(a >= prob.eps[l]), (label, l)
    for l in range(min(prob.n_axes, 8)):
        assert abs(info["eps"][l] - prob.eps[l]) <= 1e-15 * prob.eps[l]
        assert info["n_pinned"][l] == int(np.sum(lam[l] <= prob.eps[l] * (1 + 1e-12)))


def _check(lib, E, mods, label, eps=None):
    prob = T.TensorProblem(E, mods, eps=eps)
    ref = T.solve_eigs(prob)
    assert ref.converged, label
    lam, info = _gpu_solve(lib, E, mods, eps=eps)
    _compare(prob, ref.lam, lam, info, label)
    return prob, ref, lam, info


def test_closed_forms(lib):
    E = [np.array([0.5]), np.array([2.0]), np.array([3.0])]
    prob = T.TensorProblem(E, [(0, 1, 2)])
    lam, info = _gpu_solve(lib, E, [(0, 1, 2)])
    assert info["converged"] and info["n_pinned"] == [0, 1, 1]
    assert lam[1][0] == prob.eps[1] and lam[2][0] == prob.eps[2]
    assert abs(lam[0][0] - (2.0 - prob.eps[1] - prob.eps[2])) <= 1e-12 * 2.0
    lam, info = _gpu_solve(lib, [np.array([1.5])] * 3, [(0, 1, 2)])
    assert info["converged"] and info["n_flat"] == 2
    for x in lam:
        assert abs(x[0] - 1 / 4.5) < 1e-12


@pytest.mark.parametrize("seed,ranks,mods", [
    (3, (5, 7), [(0, 1)]),
    (4, (60, 400, 50), [(0, 1), (0, 2)]),
    (5, (4, 40, 3, 35), [(0, 1), (1, 2), (2, 3), (0, 3)]),
])
def test_two_axis_modalities_match_the_pair_solver(lib, seed, ranks, mods):
    rng = np.random.default_rng(seed)
    E = [np.sort(rng.uniform(0.2, 5.0, r))[::-1].copy() for r in ranks]
    prob = S.Problem(E, mods)
    ref = S.solve_eigs(prob)
    lam, info = _gpu_solve(lib, E, mods)
    _compare(prob, ref.lam, lam, info, f"pairs {ranks}")
    r = lib.solve_eigs([_dev(e) for e in E], mods)
    for a, b in zip(lam, r.lam):
        b = b.cpu().numpy()
        assert np.all(np.abs(a - b) <= 1e-10 * np.abs(b) + 1e-12 * np.max(b))


@pytest.mark.parametrize("shape,rank,mods", [
    ((20, 32, 32), 4, [(0, 1, 2)]),
    ((40, 24, 24), 4, [(0, 1, 2)]),
    ((12, 10, 8, 6), 4, [(0, 1, 2, 3)]),
    ((30, 16, 16), 3, [(0, 1, 2), (0, 1)]),
    ((9, 7, 5, 4, 3), 2, [(0, 1, 2, 3, 4)]),
])
def test_tensor_spectra(lib, shape, rank, mods):
    E = low_rank_tensor_spectra(shape, rank, seed=sum(shape))
    _check(lib, E, mods, f"tensor {shape} {mods}")


def test_larger_dense_system(lib):
    """580 unknowns over 5.8 million index tuples: parity and determinism."""
    E = low_rank_tensor_spectra((300, 160, 120), 4, seed=11)
    _check(lib, E, [(0, 1, 2)], "580 unknowns")
    a, _ = _gpu_solve(lib, E, [(0, 1, 2)])
    b, _ = _gpu_solve(lib, E, [(0, 1, 2)])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_flat_combinations_across_modalities(lib):
    """A balanced pair modality beside an unbalanced three-axis one: the null
    space of the incidence matrix is 3-dimensional, its zero-slope part 2."""
    rng = np.random.default_rng(0)
    e0 = np.sort(rng.uniform(1, 5, 6))[::-1].copy()
    E = [e0, e0.copy(), np.sort(rng.uniform(1, 5, 4))[::-1].copy(), np.sort(rng.uniform(1, 5, 5))[::-1].copy(),
         np.sort(rng.uniform(1, 5, 3))[::-1].copy()]
    prob, ref, lam, info = _check(lib, E, [(0, 1), (2, 3, 4)], "flat combinations")
    assert info["n_flat"] == 2 == len(T.flat_directions(prob))


def test_eight_axis_modality_and_sixty_four_axes(lib):
    """The limits: one modality of 8 axes (with a pair modality beside it), and
    64 axes in 21 modalities (frame, a_i, b_i, c_i) with private groups of
    equal size."""
    rng = np.random.default_rng(12)
    E8 = low_rank_tensor_spectra((3, 2, 2, 2, 3, 2, 2, 2), 1, seed=8)
    _check(lib, E8, [tuple(range(8)), (0, 4)], "8-axis modality")
    E64 = [np.sort(rng.uniform(0.5, 4.0, 3))[::-1].copy() for _ in range(64)]
    mods = [(0, 1 + 3 * i, 2 + 3 * i, 3 + 3 * i) for i in range(21)]
    prob, ref, lam, info = _check(lib, E64, mods, "64 axes")
    assert len(lam) == 64 and info["n_flat"] == len(T.flat_directions(prob))


def test_private_groups_of_different_sizes(lib):
    """Shared frame axis, private groups of 1, 2 and 2 axes with different
    ranks (the per-group factorisation path)."""
    E = low_rank_tensor_spectra((12, 9, 7), 3, seed=21)
    rng = np.random.default_rng(22)
    extra = [np.sort(rng.uniform(0.5, 30.0, r))[::-1].copy() for r in (5, 8, 6)]
    _check(lib, E + extra, [(0, 1, 2), (0, 3), (0, 4, 5)], "groups 16 / 5 / 14")


def test_tensor_spectra_truncated_and_explicit_eps(lib):
    """Retained ranks below the axis lengths (unbalanced: no flat direction) and
    bounds given by the caller."""
    E = low_rank_tensor_spectra((50, 40, 30), 5, seed=9)
    Er = [E[0][:20].copy(), E[1][:15].copy(), E[2][:30].copy()]
    _check(lib, Er, [(0, 1, 2)], "truncated")
    _check(lib, Er, [(0, 1, 2)], "eps", eps=[1e-6, 3e-7, 2e-6])


def test_coil_shape_top_ten_components(lib):
    """The paper's COIL-20 shape: 20 modalities (frame, row_i, col_i) sharing
    the frame axis, 10 principal components per axis (410 unknowns)."""
    E, mods = coil_like_spectra(seed=1)
    Er = [e[:10].copy() for e in E]
    _check(lib, Er, mods, "coil r=10")


def test_coil_shape_all_components(lib):
    """Every principal component (72 + 40 x 128 = 5192 unknowns, 21 flat
    directions): FP64 KKT of the oracle's gradient, the box and the gauge rule
    at the GPU's point."""
    E, mods = coil_like_spectra(seed=1)
    prob = T.TensorProblem(E, mods)
    lam, info = _gpu_solve(lib, E, mods)
    assert info["converged"] and info["kkt"] <= 1e-12 and info["n_flat"] == 21, info
    assert all(np.all(x >= e) for x, e in zip(lam, prob.eps))
    g = T.grad(lam, prob)
    assert T.kkt_residual(lam, g, prob) <= 1e-10
    flats = T.flat_directions(prob)
    target = T.cold_start(prob)
    t_star = [sum(c[l] * (target[l].sum() - lam[l].sum()) for l in range(prob.n_axes)) for c in flats]
    t = S.nearest_feasible_shift(t_star, flats, lam, prob.eps)
    u = np.array(flats).T @ t
    assert np.all(np.abs(u) <= 1e-9 * np.array([x.max() for x in lam])), float(np.max(np.abs(u)))
    print("coil all components:", info["iterations"], "iterations", flush=True)


@pytest.mark.parametrize("pert", [1e-10, pytest.param(1e-8, marks=pytest.mark.xfail(
    reason="the escape mode's line search stops at KKT 1.2e-8 after 34 iterations on this case (open; the "
           "library spectra of the COIL shape, imbalanced by ~5e-8, converge in 83)", strict=False))])
def test_nearly_balanced_modality_reaches_the_box(lib, pert):
    """A single modality whose axes' traces differ by `pert` relative (as
    spectra from FP32 Grams of a balanced tensor do): the 21st-like shift
    direction has a tiny slope and the minimiser sits on the box far along
    it.  The GPU must converge there (the escape mode after 30 iterations)
    and agree with the oracle, which pins one eigenvalue on two axes."""
    E = low_rank_tensor_spectra((20, 32, 32), 4, seed=2)
    E[1] = E[1] * (1 + pert)
    prob, ref, lam, info = _check(lib, E, [(0, 1, 2)], f"nearly balanced {pert}")
    assert info["iterations"] <= 120, info


def test_order_of_axes_and_modalities_does_not_matter(lib):
    """The coordinate layout follows the order of the modalities and of their
    axes; the solution must not (within the parity bar)."""
    E = low_rank_tensor_spectra((12, 9, 7), 3, seed=21)
    rng = np.random.default_rng(22)
    E = E + [np.sort(rng.uniform(0.5, 30.0, r))[::-1].copy() for r in (5, 8, 6)]
    mods = [(0, 1, 2), (0, 3), (0, 4, 5)]
    a, _ = _gpu_solve(lib, E, mods)
    perm = [4, 2, 0, 5, 1, 3]                              # new axis q is old axis perm[q]
    inv = {old: new for new, old in enumerate(perm)}
    mods_p = [tuple(inv[x] for x in reversed(m)) for m in reversed(mods)]
    b, _ = _gpu_solve(lib, [E[perm[q]] for q in range(6)], mods_p)
    for q in range(6):
        x, y = b[q], a[perm[q]]
        assert np.all(np.abs(x - y) <= 1e-10 * np.abs(y) + 1e-12 * np.max(y)), q


def test_warm_start_and_determinism(lib):
    E = low_rank_tensor_spectra((20, 32, 32), 4, seed=2)
    mods = [(0, 1, 2)]
    prob = T.TensorProblem(E, mods)
    ref = T.solve_eigs(prob)
    cold, cinfo = _gpu_solve(lib, E, mods)
    again, _ = _gpu_solve(lib, E, mods)
    for x, y in zip(cold, again):
        assert np.array_equal(x, y)
    rng = np.random.default_rng(3)
    warm = [x * np.exp(0.01 * rng.standard_normal(x.size)) for x in ref.lam]
    lam, info = _gpu_solve(lib, E, mods, warm=warm)
    assert info["warm_used"]
    _compare(prob, ref.lam, lam, info, "warm")


def test_errors(lib):
    E = [np.array([3.0, 2.0]), np.array([1.0, 0.5, 0.25]), np.array([2.0])]
    for bad_E in ([np.array([3.0, -1.0]), E[1], E[2]], [np.array([3.0, np.nan]), E[1], E[2]]):
        with pytest.raises(lib.GmgmError) as ei:
            _gpu_solve(lib, bad_E, [(0, 1, 2)])
        assert ei.value.status == 3
    for mods in ([(0,)], [(0, 0, 1)], [(0, 1, 2), (2, 1, 0)], [(0, 1)], [(0, 1, 3)]):
        with pytest.raises(lib.GmgmError) as ei:
            _gpu_solve(lib, E, mods)
        assert ei.value.status == 1, mods
    with pytest.raises(lib.GmgmError) as ei:        # more than 64 axes
        _gpu_solve(lib, [np.array([1.0])] * 65, [(0, l) for l in range(1, 65)])
    assert ei.value.status == 1
    with pytest.raises(lib.GmgmError) as ei:        # more than 8 axes in one modality
        _gpu_solve(lib, [np.array([1.0])] * 9, [tuple(range(9))])
    assert ei.value.status == 1
    with pytest.raises(lib.GmgmError) as ei:        # iteration limit
        _gpu_solve(lib, E, [(0, 1, 2)], max_iter=1)
    assert ei.value.status == 4
    lam, info = _gpu_solve(lib, E, [(0, 1, 2)], max_iter=1, raise_on_noconv=False)
    assert not info["converged"] and info["iterations"] == 1
    with pytest.raises(lib.GmgmError) as ei:        # one wave's share above 2^32 tuples
        _gpu_solve(lib, [np.ones(1)] + [np.linspace(2.0, 1.0, 2000)] * 3, [(0, 1, 2, 3)])
    assert ei.value.status == 2
    with pytest.raises(lib.GmgmError) as ei:        # dense system too large
        big = np.linspace(2.0, 1.0, 4100)
        _gpu_solve(lib, [big, big.copy(), np.array([1.0])], [(0, 1, 2)])
    assert ei.value.status == 2
    lam, info = _gpu_solve(lib, E, [(0, 1, 2)])      # the context stays usable
    assert info["converged"]


@pytest.mark.parametrize("which", ["coil10", "mixed"])
def test_from_perturbed_starts_against_the_independent_minimiser(lib, which):
    """Started 5% away from the oracle's minimiser (a dense projected Newton of
    its own, KKT ~1e-15), the GPU reaches it within the bar."""
    if which == "coil10":
        E, mods = coil_like_spectra(seed=1)
        E = [e[:10].copy() for e in E]
    else:
        E = low_rank_tensor_spectra((12, 9, 7), 3, seed=21)
        rng0 = np.random.default_rng(22)
        E = E + [np.sort(rng0.uniform(0.5, 30.0, r))[::-1].copy() for r in (5, 8, 6)]
        mods = [(0, 1, 2), (0, 3), (0, 4, 5)]
    prob = T.TensorProblem(E, mods)
    ref = T.solve_eigs(prob)
    assert ref.converged and ref.kkt <= 1e-14
    rng = np.random.default_rng(32)
    for t in range(2):
        warm = [x * np.exp(0.05 * rng.standard_normal(x.size)) for x in ref.lam]
        lam, info = _gpu_solve(lib, E, mods, warm=warm)
        assert info["warm_used"]
        _compare(prob, ref.lam, lam, info, f"{which} perturbed {t}")
