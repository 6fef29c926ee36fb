"""Leading eigenpairs of a large axis by randomized subspace iteration.
Test infrastructure only.

For an axis shared by several modalities the axis' statistic is
S = D D^T with D = [X_1 | X_2 | ...] (the concatenation of the Notation
section; its eigenvectors are D's left singular vectors, Algorithm 1's first
loop), too large to form.  Its leading r eigenpairs come from randomized
subspace iteration (Halko, Martinsson and Tropp 2011, the subspace iteration
and the direct eigenvalue / SVD steps), in FP64:

    Y = D Omega            (Omega: sum_m p_m x k, passed in)
    Q = orth(Y)
    repeat q times:        Q' = orth(D^T Q);  Q = orth(D Q')
    Z = D^T Q;  T = Z^T Z  (= Q^T D D^T Q, k x k)
    T = W diag(theta) W^T, theta descending
    E = theta[:r],  V = Q W[:, :r]

orth(Y) is the Q factor of the thin QR decomposition with a positive R
diagonal (unique for full-rank Y).
"""
from __future__ import annotations

import numpy as np


def _dense(X):
    """(n x p) FP64 of a CSR triple or a dense array."""
    if isinstance(X, tuple):
        rp, col, val, n, p = X
        M = np.zeros((n, p))
        rows = np.repeat(np.arange(n), np.diff(rp))
        np.add.at(M, (rows, col), 1.0 if val is None else np.asarray(val, np.float64))
        return M
    return np.asarray(X, np.float64)


def orth(Y):
    Q, R = np.linalg.qr(Y)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def subspace_eig(blocks, Omega, q: int, r: int):
    """(E (r, descending), V (n x r)) of S = sum_m X_m X_m^T.

    blocks: list of X_m (dense arrays or (row_ptr, col, val, n, p_m) CSR
    triples) sharing their row axis; Omega: (sum_m p_m) x k."""
    Xs = [_dense(b) for b in blocks]
    D = np.concatenate(Xs, axis=1)
    Omega = np.asarray(Omega, np.float64)
    Q = orth(D @ Omega)
    for _ in range(q):
        Qp = orth(D.T @ Q)
        Q = orth(D @ Qp)
    Z = D.T @ Q
    T = Z.T @ Z
    theta, W = np.linalg.eigh((T + T.T) / 2)
    order = np.argsort(-theta, kind="stable")
    theta, W = theta[order], W[:, order]
    return theta[:r], Q @ W[:, :r]
