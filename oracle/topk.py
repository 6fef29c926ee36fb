"""Per-row top-k thresholding into CSR.  Test infrastructure only.

Algorithm 1's thresh_{n_l} keeps n_l entries; the experiments keep "the top 5
strongest edges per gene/cell", and the complexity appendix keeps a heap of
n_l per pass.  Reading: per row i, rank j != i by |Psi_ij| descending, ties to
the smaller j, keep the first k; no symmetrisation; emit CSR with row_ptr = k*i,
columns ascending and the signed Psi_ij values.
"""
import numpy as np


def topk_row(values: np.ndarray, i: int, k: int) -> np.ndarray:
    """Indices of the k largest |values[j]|, j != i, ties to smaller j; returned ascending."""
    v = np.abs(np.asarray(values, dtype=np.float64))
    j = np.arange(v.size)
    keep = j != i
    v, j = v[keep], j[keep]
    order = np.lexsort((j, -v))          # primary: -|v| ascending, secondary: j ascending
    return np.sort(j[order[:k]])


def topk_csr(psi_rows: np.ndarray, row_ids, k: int):
    """CSR (row_ptr int64, col int32, val float64) of the top-k of each given row."""
    row_ids = np.asarray(row_ids)
    m = row_ids.size
    row_ptr = np.arange(m + 1, dtype=np.int64) * k
    col = np.empty(m * k, dtype=np.int32)
    val = np.empty(m * k, dtype=np.float64)
    for t in range(m):
        js = topk_row(psi_rows[t], int(row_ids[t]), k)
        col[t * k:(t + 1) * k] = js
        val[t * k:(t + 1) * k] = psi_rows[t][js]
    return row_ptr, col, val


def near_tie_rows(psi_rows: np.ndarray, row_ids, k: int, rel: float = 1e-6) -> np.ndarray:
    """True where the k-th and (k+1)-th largest |Psi_ij| (j != i) differ by under ``rel``."""
    row_ids = np.asarray(row_ids)
    out = np.zeros(row_ids.size, dtype=bool)
    for t in range(row_ids.size):
        v = np.abs(np.asarray(psi_rows[t], dtype=np.float64))
        v = np.delete(v, int(row_ids[t]))
        if v.size <= k:
            continue
        s = -np.sort(-v)
        out[t] = (s[k - 1] - s[k]) <= rel * s[k - 1]
    return out
