"""Eigen-recomposition Psi_l = V_l diag(lambda_l) V_l^T.  Test infrastructure only.

Algorithm 1, final loop: Psi_l = thresh[V_l Lambda_l V_l^T], thresholded while
recomposing.  The oracle forms the matrix plainly: whole (tiny inputs) or one
row at a time, Psi_i. = (V_i * lambda) V^T (large inputs).
"""
import numpy as np


def psi_dense(V: np.ndarray, lam: np.ndarray) -> np.ndarray:
    V64 = np.asarray(V, dtype=np.float64)
    return (V64 * np.asarray(lam, dtype=np.float64)[None, :]) @ V64.T


def psi_rows(V: np.ndarray, lam: np.ndarray, rows) -> np.ndarray:
    """Rows ``rows`` of V diag(lam) V^T without forming the n x n matrix."""
    V64 = np.asarray(V, dtype=np.float64)
    W = V64[np.asarray(rows)] * np.asarray(lam, dtype=np.float64)[None, :]
    return W @ V64.T


def psi_blockwise(V: np.ndarray, lam: np.ndarray, block: int) -> np.ndarray:
    """The same matrix assembled from block x block tiles (for the block-invariance pin)."""
    V64 = np.asarray(V, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = V64.shape[0]
    out = np.empty((n, n))
    for i0 in range(0, n, block):
        for j0 in range(0, n, block):
            Wi = V64[i0:i0 + block] * lam[None, :]
            out[i0:i0 + block, j0:j0 + block] = Wi @ V64[j0:j0 + block].T
    return out
