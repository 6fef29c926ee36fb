"""Partial eigendecomposition and the cell-axis factor.  Test infrastructure only.

Algorithm 1, first loop: V_l = top r_l left singular vectors of D_l and
E_l = (top r_l singular values of D_l)^2.  Theorem 1 makes these the eigenvectors
of the estimate, so V is never iterated.  The Algorithm section notes that the
eigenvectors of S_l are the left singular vectors of mat_l, so S_l need not be
formed for the large axis.

For a cells x genes X with p << n we eigendecompose the small-axis Gram
G = X^T X = V_g diag(e) V_g^T (descending e) and take the cell factor from the
exact identity U_r = X V_g[:, :r] diag(e[:r])^(-1/2), with E_cells = e[:r]
(the nonzero spectra of X X^T and X^T X coincide).
"""
import numpy as np


def eigh_desc(G: np.ndarray):
    """All eigenpairs of the symmetric G, eigenvalues descending (LAPACK's eigh)."""
    w, V = np.linalg.eigh(np.asarray(G, dtype=np.float64))
    order = np.argsort(-w, kind="stable")
    return w[order], V[:, order]


def numerical_rank(e: np.ndarray, p: int) -> int:
    """Count of eigenvalues above p * 2^-52 * e_1 (e descending)."""
    if e.size == 0 or e[0] <= 0:
        return 0
    return int(np.sum(e > p * 2.0 ** -52 * e[0]))


def cell_factor(X: np.ndarray, Vg: np.ndarray, e: np.ndarray, r: int) -> np.ndarray:
    """U = X V_g[:, :r] diag(e[:r])^(-1/2): top-r left singular vectors of X."""
    X64 = np.asarray(X, dtype=np.float64)
    return (X64 @ Vg[:, :r]) / np.sqrt(e[:r])[None, :]
