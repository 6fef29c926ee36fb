"""Pins of the randomized subspace-iteration oracle against dense
eigendecompositions and the Rayleigh-Ritz / interlacing properties -- no GPU."""
import numpy as np

import oracle
import synth
from oracle import range_finder as RF


def _blocks(seed):
    X1, _, _ = synth.nb_log1p(300, 40, 4, zipf=False, seed=seed)
    rng = np.random.default_rng(seed)
    X2 = (rng.random((300, 25)) < 0.1).astype(np.float32)
    return X1, X2


def test_full_width_subspace_equals_dense_eigendecomposition():
    """k = number of columns: the subspace is the whole range, so the result is
    the exact leading eigenpairs of D D^T."""
    X1, X2 = _blocks(1)
    D = np.concatenate([X1, X2], axis=1).astype(np.float64)
    Om = np.random.default_rng(2).standard_normal((65, 65))
    E, V = RF.subspace_eig([X1, X2], Om, q=0, r=20)
    e_ref, V_ref = oracle.eigh_desc(D @ D.T)
    np.testing.assert_allclose(E, e_ref[:20], rtol=1e-10)
    # eigenvectors up to sign (the leading spectrum is simple here)
    dots = np.abs(np.sum(V * V_ref[:, :20], axis=0))
    np.testing.assert_allclose(dots, 1.0, atol=1e-8)


def test_power_iterations_converge_and_ritz_values_interlace():
    X1, X2 = _blocks(3)
    D = np.concatenate([X1, X2], axis=1).astype(np.float64)
    e_ref, V_ref = oracle.eigh_desc(D @ D.T)
    Om = np.random.default_rng(4).standard_normal((65, 16))
    prev = None
    for q in (0, 1, 3, 8, 20):
        E, V = RF.subspace_eig([X1, X2], Om, q=q, r=6)
        assert np.all(E <= e_ref[:6] * (1 + 1e-12))           # Ritz values never exceed the eigenvalues
        if prev is not None:
            assert np.all(E >= prev * (1 - 1e-12))             # and grow with the iterations
        prev = E
    np.testing.assert_allclose(E, e_ref[:6], rtol=1e-8)
    np.testing.assert_allclose(np.abs(np.sum(V * V_ref[:, :6], axis=0)), 1.0, atol=1e-6)
    np.testing.assert_allclose(V.T @ V, np.eye(6), atol=1e-12)


def test_csr_blocks_equal_dense_blocks_and_orth_is_unique_qr():
    X1, X2 = _blocks(5)
    c1 = synth.dense_to_csr(X1) + (300, 40)
    rp, col, _ = synth.dense_to_csr(X2)
    c2 = (rp, col, None, 300, 25)                               # binary block: implicit ones
    Om = np.random.default_rng(6).standard_normal((65, 12))
    Ea, Va = RF.subspace_eig([X1, X2], Om, q=2, r=5)
    Eb, Vb = RF.subspace_eig([c1, c2], Om, q=2, r=5)
    np.testing.assert_allclose(Ea, Eb, rtol=1e-13)
    np.testing.assert_allclose(Va, Vb, atol=1e-12)
    Y = np.random.default_rng(7).standard_normal((50, 7))
    Q = RF.orth(Y)
    R = Q.T @ Y
    np.testing.assert_allclose(Q.T @ Q, np.eye(7), atol=1e-13)
    assert np.all(np.diag(R) > 0) and np.allclose(np.tril(R, -1), 0, atol=1e-12)


def test_single_block_is_the_gram_spectrum():
    """One modality: the leading eigenvalues of X X^T equal those of the small
    Gram X^T X (shared nonzero spectrum)."""
    X1, _ = _blocks(8)
    Om = np.random.default_rng(9).standard_normal((40, 40))
    E, _ = RF.subspace_eig([X1], Om, q=1, r=10)
    e_small, _ = oracle.eigh_desc(oracle.gram_dense(X1))
    np.testing.assert_allclose(E, e_small[:10], rtol=1e-10)
