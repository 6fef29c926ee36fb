"""Parity of the sparse Nonparanormal Skeptic (gmgm_skeptic) and of the Gram
and cell factor of the transformed matrix S + 1 z^T (gmgm_gram_shifted,
gmgm_sketch_shifted) with the CPU oracle, through the C ABI.

Bars: S within 1e-6 (1 + |f|) of the FP64 transform (FP32 output); z within
1e-12; column sums within 1e-9 of sum |S|; the Gram within 1e-5 sqrt(G_aa G_bb)
of the dense transform's Gram (R12); the factor within 1e-5 sum_t |x~_t B_tj|.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import skeptic as SK

pytestmark = pytest.mark.gpu


def _d(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _csr(X):
    rp, col, val = synth.dense_to_csr(np.asarray(X, dtype=np.float32))
    return rp, col, val


def _check_transform(lib, X, label, binary=False):
    X = np.asarray(X, dtype=np.float32).astype(np.float64)   # the values the library sees
    n, p = X.shape
    rp, col, val = _csr(X)
    res = lib.skeptic(_d(rp), _d(col), None if binary else _d(val), n, p)
    S_ref, z_ref = SK.skeptic_split(X)
    rows = np.repeat(np.arange(n), np.diff(rp))
    want = S_ref[rows, col]
    got = res.val.cpu().numpy()
    F = want + z_ref[col]
    assert np.all(np.abs(got - want) <= 1e-6 * (1.0 + np.abs(F))), label
    np.testing.assert_allclose(res.z.cpu().numpy(), z_ref, rtol=0, atol=1e-12, err_msg=label)
    cs = res.csum.cpu().numpy()
    assert np.all(np.abs(cs - S_ref.sum(0)) <= 1e-9 * (np.abs(S_ref).sum(0) + 1.0)), label
    return rp, col, res


def test_paper_worked_example(lib):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "skeptic_worked_example.json")))
    X = np.asarray(g["data"], dtype=np.float64).T           # variables are the example's rows
    rp, col, res = _check_transform(lib, X, "worked example")
    n = X.shape[0]
    S = np.zeros_like(X)
    S[np.repeat(np.arange(n), np.diff(rp)), col] = res.val.cpu().numpy()
    np.testing.assert_allclose(S.T, np.asarray(g["split_sparse_2dp"]), atol=0.011)
    np.testing.assert_allclose(res.z.cpu().numpy(), np.asarray(g["split_z_2dp"]), atol=0.006)


@pytest.mark.parametrize("n,p,density,seed", [(97, 13, 0.3, 1), (2000, 300, 0.05, 2), (5000, 64, 0.6, 3)])
def test_transform_integer_ties(lib, n, p, density, seed):
    rng = np.random.default_rng(seed)
    X = rng.integers(-4, 9, size=(n, p)).astype(np.float64)
    X[rng.random((n, p)) > density] = 0.0
    X[:, 0] = 0.0                                             # an all-zero column
    X[: n // 2, 1] = 3.0                                      # a long run of ties
    _check_transform(lib, X, f"ties n={n} p={p}")


def test_transform_continuous_and_binary(lib):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((3000, 40))
    X[rng.random(X.shape) < 0.8] = 0.0
    _check_transform(lib, X, "continuous")
    B = (rng.random((1500, 30)) < 0.1).astype(np.float64)
    _check_transform(lib, B, "binary", binary=True)


def test_transform_of_count_data(lib):
    X, _, _ = synth.nb_log1p(4000, 200, 6, zipf=True, seed=11)
    _check_transform(lib, X, "nb counts")


def test_shifted_gram_and_factor(lib):
    n, p, r = 3000, 250, 40
    X, _, _ = synth.nb_log1p(n, p, 6, zipf=True, seed=12)
    rp, col, val = _csr(X)
    rpd, cold, vald = _d(rp), _d(col), _d(val)
    res = lib.skeptic(rpd, cold, vald, n, p)
    G = lib.gram(rpd, cold, res.val, n, p, shift=(res.z, res.csum)).cpu().numpy().astype(np.float64)
    F = SK.skeptic_dense(X)
    G_ref = oracle.gram_dense(F)
    d = np.sqrt(np.outer(np.diag(G_ref), np.diag(G_ref)))
    assert np.all(np.abs(G - G_ref) <= 1e-5 * d)
    # factor of the transformed matrix from the GPU eigenpairs of that Gram
    w, Vt, rank = lib.eigh_small(lib.gram(rpd, cold, res.val, n, p, shift=(res.z, res.csum)))
    U = lib.sketch(rpd, cold, res.val, n, p, Vt, w, r, z=res.z).cpu().numpy().astype(np.float64)
    V = Vt.cpu().numpy().T[:, :r]
    e = w.cpu().numpy()[:r]
    B = V / np.sqrt(e)[None, :]
    U_ref = F @ B
    scale = np.abs(F) @ np.abs(B)
    assert np.all(np.abs(U - U_ref) <= 1e-5 * scale)


def test_errors(lib):
    import torch
    X = np.zeros((10, 4))
    X[2, 1] = np.nan
    X[3, 2] = 1.0
    rp, col, val = synth.dense_to_csr(np.where(np.isnan(X), 0.0, X).astype(np.float32))
    val_bad = val.copy()
    val_bad[0] = np.nan
    with pytest.raises(lib.GmgmError) as ei:
        lib.skeptic(_d(rp), _d(col), _d(val_bad), 10, 4)
    assert ei.value.status == 3
    lib.sync()
    col_bad = col.copy()
    col_bad[0] = 7
    with pytest.raises(lib.GmgmError) as ei:
        lib.skeptic(_d(rp), _d(col_bad), _d(val), 10, 4)
    assert ei.value.status == 2
    lib.sync()
    res = lib.skeptic(_d(rp), _d(col), _d(val), 10, 4)      # the context stays usable
    assert res.z.numel() == 4
