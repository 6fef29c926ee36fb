"""Significance thresholding of a recomposed precision matrix.
Test infrastructure only.

Theorem 3 and its proof in the Fisher-information appendix: under the null
hypothesis that every modality gamma has precision sigma_gamma^-2 I (no edges),
the Fisher information of the off-diagonal parameters is diagonal and does not
couple them to the diagonal or shift parameters (the block-structure
corollary).  The entry of an edge psi_lij of axis l is

    F_edge = sum over modalities gamma containing l of  A^gamma / (2 d_l),
             A^gamma = d^gamma_all sigma_gamma^4 / 2,

so that psi_lij is asymptotically N(0, 4 d_l / sum_gamma d^gamma_all sigma_gamma^4).
An edge is significant at level alpha, Bonferroni-corrected over m tests
(two-sided), when

    |psi_lij| >= t = 2 z sqrt(d_l / sum_gamma d^gamma_all sigma_gamma^4),
    z = Phi^-1(1 - alpha / (2 m)).

Readings (the paper does not fix these):
  * sigma_gamma^2 is the null model's maximum-likelihood variance,
    tr(S^gamma) / d^gamma_all (the mean squared entry of the modality's data).
  * m defaults to the number of edges of axis l, d_l (d_l - 1) / 2.
  * the sums run over the modalities that contain axis l (the proof's sum;
    the worked example's display writes the sum over all modalities in front
    of the whole matrix).
  * the statistic is the paper's: its variance is that of a parameter entering
    the precision as (E_ij + E_ji) / 2 (the worked example's edge entries),
    which is what this module computes.
  * an entry exactly at t is kept; the diagonal is not an edge.

The thresholded graph of one axis is then every (i, j), j != i, with
|Psi_ij| >= t, rows in ascending column order.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtri


def fisher_edge_entry(d_l: int, d_all, sigma2) -> float:
    """F_edge of axis l: sum over the modalities containing l of
    (d_all sigma^4 / 2) / (2 d_l)."""
    d_all = np.asarray(d_all, dtype=np.float64)
    s2 = np.asarray(sigma2, dtype=np.float64)
    return float(np.sum(d_all * s2 * s2 / 2.0) / (2.0 * d_l))


def edge_variance(d_l: int, d_all, sigma2) -> float:
    """Asymptotic null variance of an edge: the inverse of its (diagonal)
    Fisher-information entry."""
    return 1.0 / fisher_edge_entry(d_l, d_all, sigma2)


def null_sigma2(trace_s, d_all):
    """sigma_gamma^2 = tr(S^gamma) / d^gamma_all (the reading above)."""
    return np.asarray(trace_s, dtype=np.float64) / np.asarray(d_all, dtype=np.float64)


def z_two_sided(alpha: float, n_tests: float) -> float:
    """Phi^-1(1 - alpha / (2 m)): the upper quantile of the standard normal."""
    return float(-ndtri(alpha / (2.0 * n_tests)))


def significance_threshold(d_l: int, d_all, trace_s, alpha: float = 0.05, n_tests: float | None = None) -> float:
    """t = z * sqrt(edge variance) = 2 z sqrt(d_l / sum d_all sigma^4)."""
    if n_tests is None:
        n_tests = d_l * (d_l - 1) / 2.0
    s2 = null_sigma2(trace_s, d_all)
    return z_two_sided(alpha, n_tests) * math.sqrt(edge_variance(d_l, d_all, s2))


def threshold_row(psi_row: np.ndarray, i: int, thr: float) -> np.ndarray:
    """Columns j != i of one row with |Psi_ij| >= thr, ascending."""
    v = np.abs(np.asarray(psi_row, dtype=np.float64))
    keep = v >= thr
    keep[i] = False
    return np.nonzero(keep)[0].astype(np.int32)


def threshold_csr(psi_rows: np.ndarray, row_ids, thr: float):
    """CSR (row_ptr int64, col int32, val float64) of the thresholded rows."""
    row_ids = np.asarray(row_ids)
    cols, vals, ptr = [], [], [0]
    for t in range(row_ids.size):
        js = threshold_row(psi_rows[t], int(row_ids[t]), thr)
        cols.append(js)
        vals.append(np.asarray(psi_rows[t], dtype=np.float64)[js])
        ptr.append(ptr[-1] + js.size)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals) if vals else np.zeros(0)
    return np.asarray(ptr, dtype=np.int64), col.astype(np.int32), val


def near_threshold(psi_rows: np.ndarray, row_ids, thr: float, rel: float = 1e-9) -> np.ndarray:
    """Boolean mask (rows x n) of entries within rel of the threshold, whose
    side may depend on the summation order."""
    return np.abs(np.abs(np.asarray(psi_rows, dtype=np.float64)) - thr) <= rel * thr
