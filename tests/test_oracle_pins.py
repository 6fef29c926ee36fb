"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute force
on tiny inputs (triple loops, np.kron, explicit inverses and partial traces
built from the stridewise-blockwise trace definition), closed forms derived
from the eigenvalue-gradient Proposition, invariants (KKT, Existence bound,
conservation under the identifiability shift), library routines on special
cases (SVD), and finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import solver as S
from oracle.solver import Problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(s):
    return np.random.default_rng(s)


# ---------------------------------------------------------------- Gram (Notation: S_l = mat mat^T)
def test_gram_matches_triple_loop():
    X = _rng(1).standard_normal((7, 5)).astype(np.float32)
    G = oracle.gram_dense(X)
    B = np.zeros((5, 5))
    for a in range(5):
        for b in range(5):
            s = 0.0
            for c in range(7):
                s += float(X[c, a]) * float(X[c, b])
            B[a, b] = s
    np.testing.assert_allclose(G, B, rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(G, G.T)


def test_gram_csr_equals_dense_and_diagonal():
    import synth
    X, _, _ = synth.nb_log1p(300, 40, 4, zipf=True, seed=7, beta0=-1.0)
    rp, ci, vv = synth.dense_to_csr(X)
    G1 = oracle.gram_csr(rp, ci, vv, 300, 40)
    G2 = oracle.gram_dense(X)
    np.testing.assert_allclose(G1, G2, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(np.diag(G2), (X.astype(np.float64) ** 2).sum(0), rtol=1e-13)


# ---------------------------------------------------------------- spectral (Alg. 1 first loop, Thm 1)
def test_eigh_residual_orthogonality_and_shared_spectrum():
    X = _rng(2).standard_normal((30, 12))
    G = oracle.gram_dense(X)
    e, V = oracle.eigh_desc(G)
    assert np.all(np.diff(e) <= 0)
    assert np.linalg.norm(G @ V - V * e) <= 50 * 12 * 2 ** -52 * np.linalg.norm(G)
    np.testing.assert_allclose(V.T @ V, np.eye(12), atol=1e-13)
    # nonzero spectra of X X^T and X^T X coincide (Algorithm section: singular vectors of mat_l)
    ec = np.sort(np.linalg.eigvalsh(X @ X.T))[::-1][:12]
    np.testing.assert_allclose(ec, e, rtol=1e-10)
    assert oracle.numerical_rank(e, 12) == 12
    assert oracle.numerical_rank(np.sort(np.linalg.eigvalsh(X @ X.T))[::-1], 30) == 12


def test_cell_factor_is_left_singular_vectors():
    X = _rng(3).standard_normal((40, 9))
    e, Vg = oracle.eigh_desc(oracle.gram_dense(X))
    U = oracle.cell_factor(X, Vg, e, 6)
    Us, s, _ = np.linalg.svd(X, full_matrices=False)
    np.testing.assert_allclose(s[:6] ** 2, e[:6], rtol=1e-12)
    for k in range(6):
        assert abs(abs(U[:, k] @ Us[:, k]) - 1.0) < 1e-10
    np.testing.assert_allclose(U.T @ U, np.eye(6), atol=1e-12)


# ---------------------------------------------------------------- Kronecker-sum identities (Intro, App. B)
def _kron_sum(Pg, Pc):
    """Psi_g (+) Psi_c = Psi_g (x) I + I (x) Psi_c (vec stacks cells fastest)."""
    return np.kron(Pg, np.eye(Pc.shape[0])) + np.kron(np.eye(Pg.shape[0]), Pc)


def _sb_trace(M, a, d, b):
    """tr^a_b[M]_{ij} = tr[M (I_a (x) J^{ij} (x) I_b)] from the Notation section's definition."""
    out = np.zeros((d, d))
    for i in range(d):
        for j in range(d):
            J = np.zeros((d, d))
            J[i, j] = 1.0
            out[i, j] = np.trace(M @ np.kron(np.kron(np.eye(a), J), np.eye(b)))
    return out


def _spd(n, rng):
    A = rng.standard_normal((n, n))
    return A @ A.T + n * np.eye(n)


def test_kronecker_sum_eigenvalues_are_pairwise_sums():
    rng = _rng(4)
    Pc, Pg = _spd(4, rng), _spd(3, rng)
    psi, phi = np.linalg.eigvalsh(Pc), np.linalg.eigvalsh(Pg)
    K = _kron_sum(Pg, Pc)
    ev = np.sort(np.linalg.eigvalsh(K))
    np.testing.assert_allclose(ev, np.sort((psi[:, None] + phi[None, :]).ravel()), rtol=1e-12)
    sign, logdet = np.linalg.slogdet(K)
    assert sign > 0
    assert abs(logdet - np.sum(np.log(psi[:, None] + phi[None, :]))) < 1e-11
    # trace relation of the Identifiability appendix: tr(Psi_g (+) Psi_c) = d_c tr Psi_g + d_g tr Psi_c
    assert abs(np.trace(K) - (4 * np.trace(Pg) + 3 * np.trace(Pc))) < 1e-10


def test_truncated_pseudo_determinant_and_nll():
    """Singular model: on span(V_g (x) V_c) the nonzero eigenvalues are psi_i + phi_j (i<=r_c, j<=r_g)."""
    rng = _rng(5)
    n, p, rc, rg = 6, 4, 3, 2
    Vc = np.linalg.qr(rng.standard_normal((n, rc)))[0]
    Vg = np.linalg.qr(rng.standard_normal((p, rg)))[0]
    psi, phi = rng.random(rc) + 0.5, rng.random(rg) + 0.5
    Pc, Pg = (Vc * psi) @ Vc.T, (Vg * phi) @ Vg.T
    Q = np.kron(Vg, Vc)                       # basis of the support
    Kr = Q.T @ _kron_sum(Pg, Pc) @ Q
    ev = np.sort(np.linalg.eigvalsh(Kr))
    np.testing.assert_allclose(ev, np.sort((psi[:, None] + phi[None, :]).ravel()), rtol=1e-12)
    # NLL with trace terms, data on the support: tr[S_c Psi_c] = sum E_c psi (Theorem 1 eigenvectors)
    Ec, Eg = np.array([5.0, 3.0, 1.0]), np.array([4.0, 2.0])
    Sc, Sg = (Vc * Ec) @ Vc.T, (Vg * Eg) @ Vg.T
    direct = 0.5 * (np.trace(Sc @ Pc) + np.trace(Sg @ Pg) - np.log(np.linalg.det(Kr)))
    got = S.nll([psi, phi], Problem([Ec, Eg], [(0, 1)]))
    assert abs(direct - got) < 1e-12


def test_sb_trace_extraction_property():
    """Extraction lemma: tr[(I_a (x) X (x) I_b) M] = tr[X tr^a_b[M]] for symmetric M
    (with the definition's index order the identity holds for M = M^T, the
    setting of the lemma: precision matrices and their pseudo-inverses)."""
    rng = _rng(6)
    a, d, b = 2, 3, 2
    M = rng.standard_normal((a * d * b, a * d * b))
    M = M + M.T
    X = rng.standard_normal((d, d))
    lhs = np.trace(np.kron(np.kron(np.eye(a), X), np.eye(b)) @ M)
    rhs = np.trace(X @ _sb_trace(M, a, d, b))
    assert abs(lhs - rhs) < 1e-12


# ---------------------------------------------------------------- eigenvalue MLE (Prop., Existence lemma)
def test_gradient_matches_finite_difference():
    rng = _rng(7)
    prob = Problem([np.sort(rng.random(5) * 5 + 1)[::-1], np.sort(rng.random(4) * 5 + 1)[::-1]], [(0, 1)])
    lam = [rng.random(5) + 0.3, rng.random(4) + 0.3]
    g = S.grad(lam, prob)
    H = S.hess_dense(lam, prob)
    flat = np.concatenate(lam)
    h = 1e-6
    for t in range(flat.size):
        e = np.zeros_like(flat)
        e[t] = h
        up = [(flat + e)[:5], (flat + e)[5:]]
        dn = [(flat - e)[:5], (flat - e)[5:]]
        fd = (S.nll(up, prob) - S.nll(dn, prob)) / (2 * h)
        assert abs(fd - np.concatenate(g)[t]) < 1e-7
        gfd = (np.concatenate(S.grad(up, prob)) - np.concatenate(S.grad(dn, prob))) / (2 * h)
        np.testing.assert_allclose(gfd, H[:, t], atol=1e-6)


def test_profile_gradient_and_hessian_by_finite_differences():
    """The profiled NLL over the outer axis (inner eigenvalues at their exact
    one-dimensional minimisers, some pinned at eps): its gradient is the partial
    gradient (envelope theorem) and its Hessian the Schur complement of the free
    inner coordinates -- both checked against central differences of the
    profiled function itself."""
    rng = _rng(8)
    Ec = np.sort(rng.random(5) * 3 + 1)[::-1]
    Eg = np.sort(rng.random(9) * 3 + 0.5)[::-1]
    Eg[:3] *= 6.0                       # a few gene eigenvalues pin at eps at this point
    prob = Problem([Ec, Eg], [(0, 1)])
    outer, inner = S.split_axes(prob)
    assert outer == [0] and inner == [1]
    evaluate, _, state = S._profile(prob, outer, inner)
    x = rng.random(5) + 1.0
    f, g, H = evaluate(x, True)
    pins = state["lam"][1] <= prob.eps[1] * (1 + 1e-12)
    assert 0 < pins.sum() < 9
    h = 1e-6
    for t in range(5):
        e = np.zeros(5)
        e[t] = h
        fp, gp, _ = evaluate(x + e, True)
        fm, gm, _ = evaluate(x - e, True)
        assert abs((fp - fm) / (2 * h) - g[t]) <= 1e-7 * max(1.0, abs(g[t]))
        np.testing.assert_allclose((gp - gm) / (2 * h), H[:, t], rtol=1e-5, atol=1e-7)


def test_inner_solve_is_the_one_dimensional_minimiser():
    rng = _rng(18)
    p = rng.random(7) + 0.1
    E = np.concatenate([rng.random(20) * 5 + 1, [1e4]])      # the last one pins at eps
    eps = 1e-9
    x, pinned = S.inner_solve(p, E, eps)
    assert pinned[-1] and x[-1] == eps and not pinned[:-1].any()
    # stationarity to the last bit, and a brute-force grid around each minimiser
    phi = (1.0 / (p[:, None] + x[None, :-1])).sum(axis=0) - E[:-1]
    assert np.all(np.abs(phi) <= 1e-14 * E[:-1])
    for j in range(20):
        grid = x[j] * (1 + np.linspace(-1e-3, 1e-3, 201))
        obj = E[j] * grid - np.log(p[:, None] + grid[None, :]).sum(axis=0)
        assert np.argmin(obj) == 100


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_closed_form_single_pair():
    """r_c = r_g = 1, E_c = E_g = E: psi + phi = 1/E, and the start's gauge gives psi = phi = 1/(2E)."""
    for case in _golden("solver_closed_forms.json")["single_pair"]:
        E = case["E"]
        r = S.solve_eigs(Problem([np.array([E]), np.array([E])], [(0, 1)]))
        assert r.converged
        assert abs(r.lam[0][0] - case["psi"]) <= 1e-14 * case["psi"]
        assert abs(r.lam[1][0] - case["phi"]) <= 1e-14 * case["phi"]


def test_closed_form_pinned_box():
    """r_c = 1, r_g = 2 with E_ga + E_gb > E_c >= 2 E_gb: phi_a pinned at eps (KKT), others closed form."""
    for case in _golden("solver_closed_forms.json")["box"]:
        Ec, Eg = np.array([case["Ec"]]), np.array(case["Eg"])
        prob = Problem([Ec, Eg], [(0, 1)])
        eps_g = prob.eps[1]
        r = S.solve_eigs(prob)
        assert r.converged and r.n_pinned == [0, 1]
        psi = 1.0 / (case["Ec"] - case["Eg"][1]) - eps_g
        assert abs(r.lam[0][0] - psi) <= 1e-12 * psi
        assert r.lam[1][0] == eps_g
        assert abs(r.lam[1][1] - (1.0 / case["Eg"][1] - psi)) <= 1e-12
        g = S.grad(r.lam, prob)
        assert g[1][0] >= 0          # pinned coordinate: KKT sign


def test_balanced_equal_spectra_give_equal_eigenvalues_and_conserve_gauge():
    rng = _rng(9)
    e = np.sort(rng.random(40) * 50 + 0.5)[::-1]
    r = S.solve_eigs(Problem([e, e.copy()], [(0, 1)]))
    assert r.converged
    np.testing.assert_allclose(r.lam[0], r.lam[1], rtol=1e-13)
    # sum psi - sum phi equals its value at the start 1/E (zero here)
    assert abs(r.lam[0].sum() - r.lam[1].sum()) < 1e-12 * r.lam[0].sum()


def test_kkt_and_existence_bound_on_generated_spectra():
    import synth
    X, _, _ = synth.nb_log1p(800, 60, 8, zipf=False, seed=11)
    e, _ = oracle.eigh_desc(oracle.gram_dense(X))
    for rc in (10, 30, 60):
        prob = Problem([e[:rc], e], [(0, 1)])
        r = S.solve_eigs(prob)
        assert r.converged and r.kkt <= 1e-12
        g = S.grad(r.lam, prob)
        for l, other in ((0, 60), (1, rc)):
            # 0 < lambda_i E_i <= (number of partner eigenvalues), the Existence lemma read with ranks
            prod = r.lam[l] * prob.E[l]
            assert np.all(prod > 0) and np.all(prod <= other * (1 + 1e-12))
            at = r.lam[l] <= prob.eps[l] * (1 + 1e-12)
            assert np.all(g[l][at] >= 0)
            assert np.all(np.abs(g[l][~at]) <= 1e-11 * prob.E[l][~at])
        if rc < 60:
            assert r.n_pinned[1] > 0      # unbalanced: the larger-trace axis pins


def test_stationarity_lemma_bruteforce_square():
    """Lemma S_l at full rank: S_c = tr_genes[Omega^-1], S_g = tr_cells[Omega^-1] at the MLE."""
    X = _rng(12).standard_normal((3, 3)) + 2.0 * np.eye(3)
    Sc, Sg = X @ X.T, X.T @ X
    ec, Vc = oracle.eigh_desc(Sc)
    eg, Vg = oracle.eigh_desc(Sg)
    r = S.solve_eigs(Problem([ec, eg], [(0, 1)]), tol=1e-14)
    psi, phi = r.lam
    Pc, Pg = (Vc * psi) @ Vc.T, (Vg * phi) @ Vg.T
    Oinv = np.linalg.inv(_kron_sum(Pg, Pc))        # vec: cells fastest -> kron order (genes, cells)
    np.testing.assert_allclose(_sb_trace(Oinv, 3, 3, 1), Sc, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(_sb_trace(Oinv, 1, 3, 3), Sg, rtol=1e-9, atol=1e-9)


def test_stationarity_lemma_bruteforce_truncated_support():
    """Same lemma on the singular model's support span(V_g (x) V_c) with n > p."""
    X = _rng(13).standard_normal((5, 3))
    Sc, Sg = X @ X.T, X.T @ X
    eg, Vg = oracle.eigh_desc(Sg)
    Vc = oracle.cell_factor(X, Vg, eg, 3)
    r = S.solve_eigs(Problem([eg.copy(), eg], [(0, 1)]), tol=1e-14)
    psi, phi = r.lam
    Q = np.kron(Vg, Vc)
    Kr = Q.T @ _kron_sum((Vg * phi) @ Vg.T, (Vc * psi) @ Vc.T) @ Q
    Pinv = Q @ np.linalg.inv(Kr) @ Q.T              # pseudo-inverse on the support
    np.testing.assert_allclose(_sb_trace(Pinv, 3, 5, 1), Sc, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(_sb_trace(Pinv, 1, 3, 5), Sg, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("E2", [[2.0, 1.0, 0.5], [3.0, 0.9, 0.5, 0.2]])
def test_projected_gradient_agrees_with_the_profile_solver(E2):
    """A plain projected gradient descent from Algorithm 1's start (balanced and
    unbalanced, the latter with eigenvalues at the bound) reaches the point the
    profile solver returns."""
    e = np.array([2.0, 1.0, 0.5])
    prob = Problem([e, np.array(E2)], [(0, 1)])
    lam, it = S.projected_gradient(prob, tol=1e-11)
    r = S.solve_eigs(prob)
    assert r.converged
    # gradient descent converges linearly; agreement to 1e-6 pins the same point
    for a, b in zip(lam, r.lam):
        np.testing.assert_allclose(a, b, rtol=1e-6, atol=1e-9 * np.max(b))


def test_warm_start_reaches_same_solution():
    rng = _rng(14)
    e = np.sort(rng.random(30) * 20 + 1)[::-1]
    for rc in (30, 12):
        prob = Problem([e[:rc].copy(), e], [(0, 1)])
        cold = S.solve_eigs(prob)
        warm = [cold.lam[0] * (1 + 0.05 * rng.standard_normal(rc)), cold.lam[1] * 1.1 + 0.01]
        w = S.solve_eigs(prob, warm=warm)
        assert w.converged
        for a, b in zip(cold.lam, w.lam):
            # the parity bar of the GPU solver: 1e-10 relative plus 1e-12 of the axis maximum
            assert np.all(np.abs(a - b) <= 1e-10 * np.abs(b) + 1e-12 * np.max(b))


def test_three_axis_shared_cells_solution_is_kkt_point():
    """Two modalities sharing the cell axis: gradient sums over both partner axes (Prop.)."""
    rng = _rng(15)
    Ec = np.sort(rng.random(8) * 40 + 5)[::-1]
    Eg = np.sort(rng.random(12) * 20 + 1)[::-1]
    Ep = np.sort(rng.random(6) * 20 + 1)[::-1]
    prob = Problem([Ec, Eg, Ep], [(0, 1), (0, 2)])
    r = S.solve_eigs(prob)
    assert r.converged
    g = S.grad(r.lam, prob)
    for l in range(3):
        at = r.lam[l] <= prob.eps[l] * (1 + 1e-12)
        assert np.all(g[l][at] >= 0)
        assert np.all(np.abs(g[l][~at]) <= 1e-11 * prob.E[l][~at])
    # gradient of the shared axis explicitly: both modalities contribute
    psi = r.lam[0]
    manual = 0.5 * (Ec - (1 / (psi[:, None] + r.lam[1][None])).sum(1) - (1 / (psi[:, None] + r.lam[2][None])).sum(1))
    np.testing.assert_allclose(manual, g[0], atol=1e-12 * Ec.max())


# ---------------------------------------------------------------- recomposition + top-k (Alg. 1 final loop)
def test_recompose_blockwise_and_rows_equal_dense():
    rng = _rng(16)
    V = rng.standard_normal((37, 5)).astype(np.float32)
    lam = rng.random(5) + 0.1
    D = oracle.psi_dense(V, lam)
    for b in (1, 4, 16, 37, 64):
        np.testing.assert_allclose(oracle.psi_blockwise(V, lam, b), D, rtol=1e-15, atol=1e-15)
    rows = [0, 5, 36]
    np.testing.assert_allclose(oracle.psi_rows(V, lam, rows), D[rows], rtol=1e-15, atol=1e-15)
    # explicit sum definition
    i, j = 3, 11
    s = sum(float(V[i, k]) * lam[k] * float(V[j, k]) for k in range(5))
    assert abs(D[i, j] - s) < 1e-14


def test_topk_bruteforce_and_rules():
    rng = _rng(17)
    vals = rng.standard_normal(50)
    i = 7
    vals[i] = 100.0                                   # the diagonal is excluded
    got = oracle.topk_row(vals, i, 5)
    cand = sorted([(-abs(vals[j]), j) for j in range(50) if j != i])[:5]
    assert list(got) == sorted(j for _, j in cand)
    # ties go to the smaller column
    t = np.zeros(20)
    t[[3, 9, 12, 15]] = 2.0
    t[[1, 18]] = -2.0
    assert list(oracle.topk_row(t, 0, 3)) == [1, 3, 9]
    assert list(oracle.topk_row(t, 3, 3)) == [1, 9, 12]
    t2 = np.concatenate([t, np.zeros(30)])
    rp, ci, vv = oracle.topk_csr(np.stack([vals, t2]), [i, 0], 3)
    assert list(rp) == [0, 3, 6]
    assert np.all(np.diff(ci[:3]) > 0) and np.all(np.diff(ci[3:]) > 0)
    np.testing.assert_array_equal(vv[3:], t[[1, 3, 9]])


def test_near_tie_flag():
    v = np.array([5.0, 4.0, 3.0, 3.0 * (1 - 1e-7), 1.0])
    assert oracle.near_tie_rows(v[None], [4], 3)[0]
    assert not oracle.near_tie_rows(v[None], [4], 2)[0]
