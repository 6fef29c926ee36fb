"""Per-axis Gram ("covariance") matrices.  Test infrastructure only.

Notation section: S_l = mat_l[X] mat_l[X]^T with no centring or scaling.  For a
cells x genes matrix X the gene axis has S_genes = X^T X and the cell axis
S_cells = X X^T (the simplified-notation line writes mat_1[X] = X^T for the
first axis; we read the cell axis as the rows of X, so S_cells = X X^T).
"""
import numpy as np


def gram_dense(X: np.ndarray) -> np.ndarray:
    """X^T X in float64 from a dense X (values promoted exactly from float32)."""
    X64 = np.asarray(X, dtype=np.float64)
    return X64.T @ X64


def gram_csr(row_ptr, col, val, n: int, p: int) -> np.ndarray:
    """X^T X in float64 from CSR storage: sum over cells of outer products of rows."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    G = np.zeros((p, p), dtype=np.float64)
    for c in range(n):
        lo, hi = row_ptr[c], row_ptr[c + 1]
        if hi == lo:
            continue
        j = col[lo:hi]
        x = val[lo:hi]
        G[np.ix_(j, j)] += np.outer(x, x)
    return G
