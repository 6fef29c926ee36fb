"""The reasoning behind the symmetric form's certificate, checked on the CPU
with BF16 operands emulated (no GPU).

In the symmetric form a row j receives the values Psi_ij of columns i in
earlier blocks from the sweep of row i: computed as bf16(W_i) . bf16(V_j),
with row i's W, not row j's.  Two facts make the certificate of row j sound:

1. that value is within row j's rounding bound beta_j = c ||W_j|| max ||V||
   (the products' magnitudes are psi_k |V_ik V_jk| either way, and
   sum_k psi_k |V_ik||V_jk| <= ||W_j|| ||V_i||);
2. with tau_j = e_k - beta_j (e_k: the smallest exact value among the k
   largest approximations of a column sample), every value dropped on either
   side (approximation <= tau_j) is exactly below the k-th exact value once
   tau_j + beta_j < that value, which the finalize requires.

The emulation sums products of rounded operands exactly (FP64), so it
measures the operand rounding the constant c covers.  The rows the symmetric
rules would certify must then have the oracle's top k; the rules follow the
library's (row side from the row's own 512-row block on, list of 32 started
from tau; column side above tau; the full-list and k-th - 2 beta terms).
"""

import numpy as np
import pytest

import oracle
import synth
from tests import _libs
from tests.test_rounding_bound import _bf16


@pytest.fixture(scope="module")
def g():
    _libs.ensure_built()
    import paper_2407_19892_amd as pkg
    pkg.load()
    return pkg


def _setup(n, r, seed):
    V = synth.cell_factor_proxy(n, r, 6, seed=seed).astype(np.float32)
    psi = 1.0 / synth.spectrum_proxy(max(r, 64), n, 6, seed=seed)[:r]
    W32 = (V.astype(np.float64) * psi).astype(np.float32)
    A = np.abs(_bf16(W32).astype(np.float64) @ _bf16(V).astype(np.float64).T)   # A[i, j]: row i's W
    E = V.astype(np.float64) * psi @ V.astype(np.float64).T
    return V, psi, W32, A, E


@pytest.mark.parametrize("seed", [1, 2])
def test_transposed_products_stay_within_the_owning_rows_bound(g, seed):
    n, r = 1200, 64
    V, psi, W32, A, E = _setup(n, r, seed)
    c, _ = g.rounding_bound("bf16", r)
    Wn = np.linalg.norm(V.astype(np.float64) * psi, axis=1)
    beta = c * Wn * np.linalg.norm(V.astype(np.float64), axis=1).max()
    err_own = np.abs(A - np.abs(E))          # row i's value from row i's W: within beta_i
    assert np.all(err_own <= beta[:, None])
    err_t = np.abs(A.T - np.abs(E))          # row j's value from row i's W: within beta_j
    assert np.all(err_t <= beta[:, None])


@pytest.mark.parametrize("k", [1, 10])
def test_rows_the_symmetric_rules_certify_have_the_exact_top_k(g, k):
    n, r, C, block, stride = 1500, 48, 32, 512, 8
    V, psi, W32, A, E = _setup(n, r, 3 + k)
    c, _ = g.rounding_bound("bf16", r)
    Wn = np.linalg.norm(V.astype(np.float64) * psi, axis=1)
    beta = c * Wn * np.linalg.norm(V.astype(np.float64), axis=1).max()
    absE = np.abs(E)
    np.fill_diagonal(absE, -1.0)
    nvt = -(-n // 32)
    samp = np.concatenate([np.arange(t * 32, min(n, t * 32 + 32)) for t in range(0, nvt, stride)])
    rows = np.arange(n)
    _, rcol, _ = oracle.topk_csr(E[rows], rows, k)
    rcol = rcol.reshape(n, k)
    tie = oracle.near_tie_rows(E[rows], rows, k)
    certified = 0
    for i in rows:
        # bound from the sample: exact values of the k largest approximations
        cols = samp[samp != i]
        top = cols[np.argsort(-A[i, cols], kind="stable")[:k]]
        tau = absE[i, top].min() - beta[i]
        if not tau > 0:
            continue                                   # no bound: re-swept in full
        b0 = (i // block) * block
        own = np.arange(b0, n)
        own = own[own != i]
        rv = A[i, own]
        keep = rv > tau
        lv = np.sort(rv[keep])[::-1]
        lj = own[keep][np.argsort(-rv[keep], kind="stable")]
        mout = -1.0
        if lv.size >= C:
            mout = lv[C - 1]
        if lv.size >= k:
            mout = max(mout, lv[k - 1] - 2 * beta[i])
        lv, lj = lv[:C], lj[:C]
        early = np.arange(0, b0)
        cv = A[early, i]                               # computed with row i' s W for i' < b0
        ck = cv > tau
        cand_v = np.concatenate([lv, cv[ck]])
        cand_j = np.concatenate([lj, early[ck]])
        if cand_v.size < k:
            continue
        ak = np.sort(cand_v)[::-1][k - 1]
        R = cand_j[cand_v >= ak - 2 * beta[i]]
        ex = absE[i, R]
        order = np.lexsort((R, -ex))
        tk = ex[order[k - 1]]
        if (mout >= 0 and not mout + beta[i] < tk) or not tau + beta[i] < tk:
            continue                                   # not certified: re-swept in full
        certified += 1
        got = np.sort(R[order[:k]])
        assert tie[i] or np.array_equal(got, np.sort(rcol[i])), (i, got, rcol[i])
    assert certified > 0.8 * n
