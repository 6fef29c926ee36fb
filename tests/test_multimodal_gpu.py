"""The shared-cell-axis path (RNA + ATAC peaks) on the GPU, through the C ABI:
CSR transpose, randomized subspace iteration for the axes too large for a
Gram, and the three-axis joint eigenvalue solve feeding the top-k.

Bars: the transpose is exact (same entries per row, order free); subspace
eigenvalues within 1e-9 relative of the FP64 oracle run on the same test
matrix, eigenvectors within 1e-6 (projector entries; FP32 output); the joint
solve as the two-axis solve (pinned sets identical, 1e-10 relative); top-k
rows identical to the oracle's on the GPU factors except flagged near ties.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import range_finder as RF
from oracle import solver as S

pytestmark = pytest.mark.gpu


def _d(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mat(lib, rp, col, val, n, p):
    return lib.CsrMatrix(_d(rp), _d(col), None if val is None else _d(val), n, p)


def _modalities(n, p_rna, p_pk, seed):
    X, _, _ = synth.nb_log1p(n, p_rna, 6, zipf=True, seed=seed)
    rna = synth.dense_to_csr(X)
    rp, col, _ = synth.csr_proxy(n, p_pk, 0.05, seed=seed + 1)
    return X, rna, (rp, col)


def test_csr_transpose_exact(lib):
    X, (rp, col, val), (prp, pcol) = _modalities(1500, 300, 700, 41)
    import scipy.sparse as sp
    for (r_, c_, v_, p) in ((rp, col, val, 300), (prp, pcol, None, 700)):
        M = _mat(lib, r_, c_, v_, 1500, p)
        T = M.transpose()
        ref = sp.csr_matrix((np.ones(c_.size, np.float32) if v_ is None else v_, c_, r_), shape=(1500, p)).T.tocsr()
        trp = T.row_ptr.cpu().numpy()
        assert np.array_equal(trp, ref.indptr.astype(np.int64))
        tc, tv = T.col.cpu().numpy(), T.val.cpu().numpy()
        for j in range(p):
            a, b = slice(trp[j], trp[j + 1]), slice(ref.indptr[j], ref.indptr[j + 1])
            o1, o2 = np.argsort(tc[a], kind="stable"), np.argsort(ref.indices[b], kind="stable")
            assert np.array_equal(tc[a][o1], ref.indices[b][o2])
            assert np.array_equal(tv[a][o1], ref.data[b][o2])


def _check_eig(E, V, E_ref, V_ref, label):
    E, V = E.cpu().numpy(), V.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(E, E_ref, rtol=1e-9, err_msg=label)
    P, P_ref = V @ V.T, V_ref @ V_ref.T
    assert np.max(np.abs(P - P_ref)) <= 1e-6, label
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) <= 1e-6, label


@pytest.mark.parametrize("k,q,r", [(40, 2, 20), (64, 0, 10), (128, 1, 100)])
def test_subspace_eig_cells_parity(lib, k, q, r):
    n = 2500
    X, (rp, col, val), (prp, pcol) = _modalities(n, 300, 700, 42)
    Om = np.random.default_rng(k + q).standard_normal((1000, k))
    E_ref, V_ref = RF.subspace_eig([(rp, col, val, n, 300), (prp, pcol, None, n, 700)], Om, q, r)
    E, V = lib.subspace_eig([_mat(lib, rp, col, val, n, 300), _mat(lib, prp, pcol, None, n, 700)], _d(Om), q, r)
    _check_eig(E, V, E_ref, V_ref, f"k={k} q={q}")


def test_subspace_eig_full_width_equals_gram_spectrum(lib):
    """One block, k = p: the subspace is the whole range, so the eigenvalues are
    the small Gram's (XX^T and X^T X share their nonzero spectrum)."""
    n, p = 1200, 90
    X, _, _ = synth.nb_log1p(n, p, 4, zipf=False, seed=43)
    rp, col, val = synth.dense_to_csr(X)
    Om = np.random.default_rng(1).standard_normal((p, p))
    E, V = lib.subspace_eig([_mat(lib, rp, col, val, n, p)], _d(Om), 0, 30)
    e_ref, _ = oracle.eigh_desc(oracle.gram_dense(X))
    np.testing.assert_allclose(E.cpu().numpy(), e_ref[:30], rtol=1e-10)


def test_peaks_axis_from_the_transpose(lib):
    """The peaks axis: leading eigenpairs of X_pk^T X_pk by subspace iteration on
    D = X_pk^T (blocks = the transpose, blocks_t = X_pk itself)."""
    n, p = 2500, 700
    rp, col, _ = synth.csr_proxy(n, p, 0.05, seed=44)
    M = _mat(lib, rp, col, None, n, p)
    Mt = M.transpose()
    Om = np.random.default_rng(2).standard_normal((n, 48))
    E, V = lib.subspace_eig([Mt], _d(Om), 2, 24, blocks_t=[M])
    Xd = np.zeros((n, p))
    Xd[np.repeat(np.arange(n), np.diff(rp)), col] = 1.0
    E_ref, V_ref = RF.subspace_eig([Xd.T], Om, 2, 24)
    _check_eig(E, V, E_ref, V_ref, "peaks")


def test_subspace_eig_errors(lib):
    n, p = 300, 50
    X, _, _ = synth.nb_log1p(n, p, 3, zipf=False, seed=45)
    rp, col, val = synth.dense_to_csr(X)
    M = _mat(lib, rp, col, val, n, p)
    with pytest.raises(lib.GmgmError) as ei:                # k > p
        lib.subspace_eig([M], _d(np.ones((p, 60))), 0, 10)
    assert ei.value.status == 2
    with pytest.raises(lib.GmgmError) as ei:                # rank-deficient test matrix
        lib.subspace_eig([M], _d(np.zeros((p, 8))), 0, 4)
    assert ei.value.status == 4
    with pytest.raises(lib.GmgmError) as ei:                # r > k
        lib.subspace_eig([M], _d(np.ones((p, 8))), 0, 9)
    assert ei.value.status == 1


def test_three_axis_chain_cells_genes_peaks(lib):
    """Cells shared by RNA (genes) and ATAC (peaks): GPU subspace iteration for
    cells and peaks, GPU Gram + eigh for genes, GPU joint solve (two
    modalities), GPU top-k on cells and peaks.  The solve is compared with the
    oracle's solve on the GPU's spectra (stage isolation), the top-k with the
    oracle's on the GPU's factors."""
    import torch
    n, p_g, p_p, r_c, r_p, k = 3000, 400, 900, 50, 40, 10
    X, (rp, col, val), (prp, pcol) = _modalities(n, p_g, p_p, 46)
    rna, pk = _mat(lib, rp, col, val, n, p_g), _mat(lib, prp, pcol, None, n, p_p)
    rng = np.random.default_rng(3)
    Ec, Vc = lib.subspace_eig([rna, pk], _d(rng.standard_normal((p_g + p_p, 64))), 2, r_c)
    Ep, Vp = lib.subspace_eig([pk.transpose()], _d(rng.standard_normal((n, 56))), 2, r_p, blocks_t=[pk])
    G = lib.gram(rna.row_ptr, rna.col, rna.val, n, p_g)
    Eg_all, _, rank = lib.eigh_small(G)
    Eg = Eg_all[:rank].contiguous()
    sol = lib.solve_eigs([Ec, Eg, Ep], [(0, 1), (0, 2)])
    E_np = [Ec.cpu().numpy(), Eg.cpu().numpy(), Ep.cpu().numpy()]
    prob = S.Problem(E_np, [(0, 1), (0, 2)])
    ref = S.solve_eigs(prob)
    assert sol.info["converged"] and ref.converged
    for l in range(3):
        a, b = sol.lam[l].cpu().numpy(), ref.lam[l]
        pa, pb = a <= prob.eps[l] * (1 + 1e-12), b <= prob.eps[l] * (1 + 1e-12)
        assert np.array_equal(pa, pb)
        assert np.all(np.abs(a - b)[~pb] <= 1e-10 * np.abs(b[~pb]) + 1e-12 * np.max(b))
    for V, lam, nrows in ((Vc, sol.lam[0], n), (Vp, sol.lam[2], p_p)):
        out = lib.recompose_topk(V, lam, k, prec="bf16")
        rows = np.arange(0, nrows, 11)
        Vn = V.cpu().numpy()
        P = oracle.psi_rows(Vn, lam.cpu().numpy(), rows)
        _, rcol, _ = oracle.topk_csr(P, rows, k)
        tie = oracle.near_tie_rows(P, rows, k)
        got = out.col.cpu().numpy().reshape(nrows, k)[rows]
        assert np.all((got == rcol.reshape(-1, k)).all(1) | tie)
