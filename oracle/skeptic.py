"""Nonparanormal Skeptic transform kept sparse ("Preserving input sparsity").
Test infrastructure only.

Each variable (here: each column of a samples x variables matrix) is ranked
across its samples, ties sharing the smallest rank, and mapped to the normal
scale: f(x) = Phi^-1(rank(x) / (n + 1)).  All zeros of a variable map to the
same value z, so the transformed matrix is S + 1 z^T with S zero wherever the
data are zero (the appendix's split into a sparse matrix and a rank-one term).
The transform is written out directly: scipy's rankdata ('min' ties) and
ndtri.  The Gram and the cell factor of S + 1 z^T are then those of a dense
matrix, computed by the other oracle functions on the dense transform.

Reading: the paper's example shares the smallest rank among ties (the zeros
of its first row both get rank 2); its text notes that tie handling is a
choice.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ndtri
from scipy.stats import rankdata


def skeptic_dense(X: np.ndarray) -> np.ndarray:
    """The transform of every column of the dense samples x variables X (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    R = np.apply_along_axis(lambda v: rankdata(v, method="min"), 0, X)
    return ndtri(R / (n + 1.0))


def skeptic_split(X: np.ndarray):
    """(S, z): S = transform - 1 z^T, zero where X is zero; z the zeros' value."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    F = skeptic_dense(X)
    rank0 = 1.0 + np.sum(X < 0.0, axis=0)
    z = ndtri(rank0 / (n + 1.0))
    S = F - z[None, :]
    S[X == 0.0] = 0.0
    return S, z
