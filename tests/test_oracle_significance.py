"""Pins of the significance-thresholding oracle (Theorem 3 and the
Fisher-information appendix), checked against things other than its own
formulas:

* the edge entries of the Fisher information, recomputed by brute force: the
  second derivative of the paper's NLL (minus one half the sum over modalities
  of log det of the Kronecker-sum precision, the trace terms being linear) at
  the null, by central differences of numpy's slogdet on explicitly built
  Kronecker sums, for the appendix's worked example (axes of sizes 3, 2, 2;
  modalities (1, 2) and (1, 3));
* the block structure the corollary states (edges couple neither with each
  other nor with diagonal entries), by mixed differences;
* the normal quantile against the closed-form tail 0.5 erfc(z / sqrt 2);
* the thresholded CSR against its defining invariants.
"""
import math

import numpy as np
import pytest

from oracle import significance as SG

DIMS = (3, 2, 2)
MODALITIES = ((0, 1), (0, 2))
SIGMA2 = (1.7, 0.45)      # per modality


def _kron_sum_part(dims, axis, M):
    """The term I x ... x M x ... x I of a Kronecker sum (M on `axis`)."""
    out = np.ones((1, 1))
    for a, d in enumerate(dims):
        out = np.kron(out, M if a == axis else np.eye(d))
    return out


def _neg_half_logdet(h_by_param, params):
    """-1/2 sum_gamma log det(Omega_gamma) with Omega_gamma = sigma^-2 I plus
    h times each parameter's perturbation placed in the Kronecker sum."""
    tot = 0.0
    for g, axes in enumerate(MODALITIES):
        dims = [DIMS[a] for a in axes]
        om = np.eye(int(np.prod(dims))) / SIGMA2[g]
        for h, (axis, i, j) in zip(h_by_param, params):
            if axis not in axes:
                continue
            E = np.zeros((DIMS[axis], DIMS[axis]))
            if i == j:
                E[i, i] = 1.0
            else:
                E[i, j] = E[j, i] = 0.5      # the parameter enters as (E_ij + E_ji) / 2
            om = om + h * _kron_sum_part(dims, axes.index(axis), E)
        sign, ld = np.linalg.slogdet(om)
        assert sign > 0
        tot += -0.5 * ld
    return tot


def _hessian_entry(pa, pb, step=1e-3):
    f = lambda ha, hb: _neg_half_logdet((ha, hb), (pa, pb))
    return (f(step, step) - f(step, -step) - f(-step, step) + f(-step, -step)) / (4 * step * step)


def _d_all(axes):
    return int(np.prod([DIMS[a] for a in axes]))


@pytest.mark.parametrize("axis,i,j", [(0, 0, 1), (0, 1, 2), (0, 0, 2), (1, 0, 1), (2, 0, 1)])
def test_fisher_edge_entry_matches_brute_force_hessian(axis, i, j):
    num = _hessian_entry((axis, i, j), (axis, i, j))
    mods = [g for g, axes in enumerate(MODALITIES) if axis in axes]
    closed = SG.fisher_edge_entry(DIMS[axis], [_d_all(MODALITIES[g]) for g in mods], [SIGMA2[g] for g in mods])
    assert abs(num - closed) <= 1e-5 * closed, (num, closed)   # O(step^2) difference error


def test_fisher_edge_block_is_diagonal_and_uncoupled():
    edges = [(0, 0, 1), (0, 1, 2), (1, 0, 1), (2, 0, 1)]
    diags = [(0, 1, 1), (1, 0, 0), (2, 1, 1)]
    for a in range(len(edges)):
        for b in range(a + 1, len(edges)):
            assert abs(_hessian_entry(edges[a], edges[b])) < 1e-7
        for d in diags:
            assert abs(_hessian_entry(edges[a], d)) < 1e-7
    # a diagonal entry does couple to others (the A block is not diagonal)
    assert abs(_hessian_entry((0, 1, 1), (1, 0, 0))) > 1e-3


def test_edge_variance_is_the_theorem_statistic():
    """Theorem 3: sqrt(sum d_all sigma^4 / d_l) psi / 2 is standard normal, i.e.
    the variance is 4 d_l / sum d_all sigma^4, the inverse of the brute-force
    Fisher entry."""
    num = _hessian_entry((0, 0, 1), (0, 0, 1))
    var = SG.edge_variance(3, [6, 6], list(SIGMA2))
    assert abs(var * num - 1.0) < 1e-5
    assert abs(var - 4 * 3 / (6 * SIGMA2[0] ** 2 + 6 * SIGMA2[1] ** 2)) < 1e-12


@pytest.mark.parametrize("alpha,m", [(0.05, 1), (0.05, 190), (0.01, 4.95e11), (0.2, 3)])
def test_normal_quantile_tail(alpha, m):
    z = SG.z_two_sided(alpha, m)
    assert z > 0
    tail = 0.5 * math.erfc(z / math.sqrt(2.0))
    assert abs(tail - alpha / (2 * m)) <= 1e-10 * (alpha / (2 * m))


def test_threshold_monotone_and_default_tests():
    t1 = SG.significance_threshold(1000, [2e7], [3e7], 0.05)
    t2 = SG.significance_threshold(1000, [2e7], [3e7], 0.05, n_tests=1000 * 999 / 2)
    assert t1 == t2
    assert SG.significance_threshold(1000, [2e7], [3e7], 0.01) > t1       # stricter level
    assert SG.significance_threshold(1000, [2e7, 1e7], [3e7, 1e7], 0.05) < t1   # more data


def test_threshold_csr_invariants():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 6))
    P = A @ np.diag(rng.uniform(0.5, 2.0, 6)) @ A.T
    thr = float(np.quantile(np.abs(P), 0.8))
    rp, col, val = SG.threshold_csr(P, np.arange(40), thr)
    kept = set()
    for i in range(40):
        js = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(js) > 0)
        assert i not in js
        assert np.all(np.abs(P[i, js]) >= thr)
        np.testing.assert_array_equal(val[rp[i]:rp[i + 1]], P[i, js])
        others = np.setdiff1d(np.arange(40), np.append(js, i))
        assert np.all(np.abs(P[i, others]) < thr)
        kept |= {(i, int(j)) for j in js}
    assert all((j, i) in kept for (i, j) in kept)        # symmetric matrix, symmetric graph
    # an entry exactly at the threshold is kept
    rp2, col2, _ = SG.threshold_csr(P, [0], float(abs(P[0, 3])))
    assert 3 in col2
