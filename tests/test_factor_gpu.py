"""Parity of the factor steps (HIP, through the C ABI) with the CPU oracle:
gmgm_gram (small-axis Gram), gmgm_eigh_small (FP64 eigendecomposition) and
gmgm_sketch (cell-axis factor U = X V diag(e)^-1/2).

Bars (each stage fed the oracle's own inputs):
* Gram: |G - G_ref| <= 1e-5 sqrt(G_aa G_bb) (FP32 result, FP64 reference),
  G exactly symmetric.
* eigh: |e - e_ref| <= 64 p 2^-52 e_1; residual |G v - e v| and
  orthogonality at the same scale; eigenvectors of well-separated eigenvalues
  equal the oracle's up to sign; numerical rank identical.
* sketch: |U - U_ref| <= 1e-5 sum_t |x_t B_tj| per entry (B the scaled
  eigenvector panel).
Inputs: the NB-log1p generator (cells x genes, clustered) at small and
medium sizes, a 40k x 20k 5%-dense CSR stand-in at the full gene width.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

_CACHE = {}


def _nb(n, p, clusters, zipf, seed):
    key = ("nb", n, p, clusters, zipf, seed)
    if key not in _CACHE:
        X, _, _ = synth.nb_log1p(n, p, clusters, zipf=zipf, seed=seed)
        _CACHE[key] = X
    return _CACHE[key]


def _dev(*arrs):
    import torch
    return [None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _gram_gpu(lib, rp, col, val, n, p, path=None):
    """path: None (the library's choice), "dense" (FP32 MFMA panels) or
    "sparse" (products of the nonzeros into FP64 LDS tiles)."""
    import os
    rpd, cd, vd = _dev(rp, col, val)
    old = os.environ.get("GMGM_GRAM_PATH")
    if path is not None:
        os.environ["GMGM_GRAM_PATH"] = path
    try:
        return lib.gram(rpd, cd, vd, n, p).cpu().numpy()
    finally:
        if path is not None:
            if old is None:
                del os.environ["GMGM_GRAM_PATH"]
            else:
                os.environ["GMGM_GRAM_PATH"] = old


def _check_gram(G, Gref, label):
    assert G.dtype == np.float32
    assert np.array_equal(G, G.T), label
    d = np.sqrt(np.maximum(np.diag(Gref), 0))
    tol = 1e-5 * np.outer(d, d) + 1e-30
    err = np.abs(G.astype(np.float64) - Gref)
    assert np.all(err <= tol), (label, float(np.max(err / tol)))


@pytest.mark.parametrize("path", ["dense", "sparse"])
@pytest.mark.parametrize("n,p,clusters,zipf,seed", [(2000, 500, 8, False, 1000), (3001, 700, 5, True, 7),
                                                    (257, 31, 3, False, 8)])
def test_gram_parity_generator(lib, n, p, clusters, zipf, seed, path):
    X = _nb(n, p, clusters, zipf, seed)
    rp, col, val = synth.dense_to_csr(X)
    G = _gram_gpu(lib, rp, col, val, n, p, path)
    _check_gram(G, oracle.gram_csr(rp, col, val, n, p), f"{n}x{p} {path}")


def test_gram_sparse_path_unsorted_duplicate_and_block_edges(lib):
    """Sparse path: rows whose columns are not strictly increasing (shuffled,
    duplicated) mixed with sorted rows, columns on both sides of the 128-column
    block edges, p not a multiple of 128, empty rows, 5%-dense rows."""
    rng = np.random.default_rng(11)
    n, p = 3000, 777
    rows = []
    for r in range(n):
        m = int(rng.binomial(p, 0.05))
        c = np.sort(rng.choice(p, m, replace=False))
        if r % 7 == 0 and m > 1:
            rng.shuffle(c)
        if r % 11 == 0 and m > 0:
            c = np.concatenate([c, c[:2]])
        if r % 13 == 0:
            c = np.array([127, 128, 255, 256, 767, 768, 776], dtype=np.int64)
        if r % 17 == 0:
            c = np.zeros(0, np.int64)
        rows.append(c.astype(np.int32))
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([c.size for c in rows])
    col = np.concatenate(rows)
    val = rng.standard_normal(col.size).astype(np.float32)
    X = np.zeros((n, p))
    np.add.at(X, (np.repeat(np.arange(n), np.diff(rp)), col), val.astype(np.float64))
    Gref = X.T @ X
    for path in ("sparse", "dense"):
        _check_gram(_gram_gpu(lib, rp, col, val, n, p, path), Gref, path)
    _check_gram(_gram_gpu(lib, rp, col, None, n, p, "sparse"), _ones_gram(rp, col, n, p), "sparse binary")


def _ones_gram(rp, col, n, p):
    X = np.zeros((n, p))
    np.add.at(X, (np.repeat(np.arange(n), np.diff(rp)), col), 1.0)
    return X.T @ X


def test_gram_parity_workload_100k_by_2000(lib):
    """The 100k cells x 2000 genes workload (20 Zipf clusters)."""
    X = _nb(100_000, 2000, 20, True, 2000)
    rp, col, val = synth.dense_to_csr(X)
    G = _gram_gpu(lib, rp, col, val, 100_000, 2000)
    _check_gram(G, oracle.gram_dense(X), "100k x 2000")


@pytest.mark.parametrize("path", ["dense", "sparse"])
def test_gram_binary_values_duplicates_empty_rows_and_tiny(lib, path):
    rng = np.random.default_rng(3)
    X = (rng.random((300, 45)) < 0.1).astype(np.float32)
    X[17] = 0
    X[299] = 0
    rp, col, _ = synth.dense_to_csr(X)
    G = _gram_gpu(lib, rp, col, None, 300, 45, path)      # implicit ones
    _check_gram(G, oracle.gram_dense(X), "binary")
    # duplicate column entries add up (row 0 holds column 3 twice)
    rp2 = np.array([0, 3, 4], dtype=np.int64)
    col2 = np.array([3, 3, 1, 0], dtype=np.int32)
    val2 = np.array([1.5, 2.0, -1.0, 4.0], dtype=np.float32)
    Xd = np.zeros((2, 5), np.float32)
    Xd[0, 3] = 3.5
    Xd[0, 1] = -1.0
    Xd[1, 0] = 4.0
    _check_gram(_gram_gpu(lib, rp2, col2, val2, 2, 5, path), oracle.gram_dense(Xd), "duplicates")
    # one cell, one gene; all-zero matrix
    G1 = _gram_gpu(lib, np.array([0, 1], np.int64), np.array([0], np.int32), np.array([3.0], np.float32), 1, 1,
                   path)
    assert G1[0, 0] == np.float32(9.0)
    Gz = _gram_gpu(lib, np.zeros(11, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32), 10, 300, path)
    assert not Gz.any()


@pytest.mark.parametrize("path", ["dense", "sparse"])
def test_gram_full_gene_width_sampled(lib, path):
    """20k genes (dense: 79 x 79 output tiles, two densified panels; sparse:
    157 x 158 / 2 tile pairs): every diagonal entry exact-checked, a 96 x 96
    sample of entries against FP64."""
    import scipy.sparse as sp
    n, p = 40_000, 20_000
    rp, col, val = synth.csr_proxy(n, p, 0.05, seed=3000, workers=4)
    G = _gram_gpu(lib, rp, col, val, n, p, path)
    assert np.array_equal(G, G.T)
    diag = np.bincount(col, weights=val.astype(np.float64) ** 2, minlength=p)
    assert np.all(np.abs(np.diag(G) - diag) <= 1e-5 * diag + 1e-30)
    idx = np.unique(np.concatenate([np.arange(40), np.arange(p - 40, p),
                                    np.random.default_rng(1).integers(0, p, 16)]))
    X = sp.csr_matrix((val, col, rp), shape=(n, p))
    Xs = X[:, idx].toarray().astype(np.float64)
    Gref = Xs.T @ Xs
    _check_gram(np.ascontiguousarray(G[np.ix_(idx, idx)]), Gref, "20k sample")


@pytest.mark.parametrize("path", ["dense", "sparse"])
def test_gram_errors(lib, path, monkeypatch):
    monkeypatch.setenv("GMGM_GRAM_PATH", path)
    rp, col, val = _dev(np.array([0, 2, 1], np.int64), np.array([0, 1], np.int32), np.array([1, 2], np.float32))
    with pytest.raises(lib.GmgmError) as ei:                # row_ptr decreasing
        lib.gram(rp, col, val, 2, 3)
    assert ei.value.status == 2
    rp, col, val = _dev(np.array([0, 2], np.int64), np.array([0, 5], np.int32), np.array([1, 2], np.float32))
    with pytest.raises(lib.GmgmError) as ei:                # column out of range
        lib.gram(rp, col, val, 1, 3)
    assert ei.value.status == 2
    rp, col, val = _dev(np.array([0, 2], np.int64), np.array([0, 1], np.int32), np.array([1, np.nan], np.float32))
    with pytest.raises(lib.GmgmError) as ei:
        lib.gram(rp, col, val, 1, 3)
    assert ei.value.status == 3
    with pytest.raises(lib.GmgmError) as ei:
        lib.gram(rp, col, val, 1, 70_000)
    assert ei.value.status == 2
    G = lib.gram(*_dev(np.array([0, 1], np.int64), np.array([0], np.int32), np.array([2.0], np.float32)), 1, 1)
    assert float(G[0, 0]) == 4.0                             # usable after errors


def _sym32(G):
    G = np.asarray(G, np.float64)
    return ((G + G.T) / 2).astype(np.float32)


def _eigh_gpu(lib, G32):
    (Gd,) = _dev(np.ascontiguousarray(G32, dtype=np.float32))
    w, Vt, rank = lib.eigh_small(Gd)
    return w.cpu().numpy(), Vt.cpu().numpy().T, rank         # V: columns are eigenvectors


def _check_eigh(G32, w, V, rank, label):
    G = G32.astype(np.float64)
    p = G.shape[0]
    e_ref, V_ref = oracle.eigh_desc(G)
    scale = 64 * p * 2.0 ** -52 * max(abs(e_ref[0]), 1e-300)
    assert np.all(np.diff(w) <= 0), label
    assert np.all(np.abs(w - e_ref) <= scale), (label, float(np.max(np.abs(w - e_ref)) / scale))
    assert np.linalg.norm(G @ V - V * w[None, :], axis=0).max() <= scale, label
    assert np.abs(V.T @ V - np.eye(p)).max() <= 128 * p * 2.0 ** -52, label
    gap = np.minimum(np.abs(np.diff(e_ref, prepend=np.inf)), np.abs(np.diff(e_ref, append=-np.inf)))
    sep = gap > 1e-6 * e_ref[0]
    dots = np.abs(np.sum(V[:, sep] * V_ref[:, sep], axis=0))
    assert np.all(np.abs(dots - 1) <= 1e-6), label
    assert rank == oracle.numerical_rank(e_ref, p), label


@pytest.mark.parametrize("n,p,clusters,zipf,seed", [(2000, 500, 8, False, 1000), (3001, 700, 5, True, 7)])
def test_eigh_parity_generator_grams(lib, n, p, clusters, zipf, seed):
    X = _nb(n, p, clusters, zipf, seed)
    G32 = _sym32(oracle.gram_dense(X))
    w, V, rank = _eigh_gpu(lib, G32)
    _check_eigh(G32, w, V, rank, f"{p}")
    (Gd,) = _dev(G32)                                        # eigenvalues only
    w2, Vt2, rank2 = lib.eigh_small(Gd, vectors=False)
    assert Vt2 is None and rank2 == rank
    e_ref = oracle.eigh_desc(G32.astype(np.float64))[0]
    assert np.all(np.abs(w2.cpu().numpy() - e_ref) <= 64 * p * 2.0 ** -52 * abs(e_ref[0]))


def test_eigh_workload_2000_rank_deficient_and_tiny(lib):
    X = _nb(100_000, 2000, 20, True, 2000)
    G32 = _sym32(oracle.gram_dense(X))
    _check_eigh(G32, *_eigh_gpu(lib, G32), "2000")
    Y = np.random.default_rng(4).standard_normal((50, 200))
    Gd = _sym32(Y.T @ Y)                                     # rank 50
    w, V, rank = _eigh_gpu(lib, Gd)
    _check_eigh(Gd, w, V, rank, "rank-deficient")
    assert rank == oracle.numerical_rank(oracle.eigh_desc(Gd.astype(np.float64))[0], 200)
    for G in (np.array([[2.5]], np.float32), np.diag(np.arange(7, 0, -1)).astype(np.float32)):
        _check_eigh(G, *_eigh_gpu(lib, G), "tiny")


def test_eigh_errors(lib):
    import torch
    G = np.eye(4, dtype=np.float32)
    G[1, 2] = G[2, 1] = np.inf
    with pytest.raises(lib.GmgmError) as ei:
        _eigh_gpu(lib, G)
    assert ei.value.status == 3
    w, V, rank = _eigh_gpu(lib, np.eye(3, dtype=np.float32))
    assert rank == 3


def _sketch_gpu(lib, rp, col, val, n, p, V, e, r):
    rpd, cd, vd = _dev(rp, col, val)
    Vt, ed = _dev(np.ascontiguousarray(V.T), e)               # column-major storage of V
    return lib.sketch(rpd, cd, vd, n, p, Vt, ed, r).cpu().numpy()


def _check_sketch(X, V, e, r, U, label):
    Uref = oracle.cell_factor(X, V, e, r)
    B = np.abs(V[:, :r]) / np.sqrt(e[:r])[None, :]
    scale = np.abs(X.astype(np.float64)) @ B
    assert np.all(np.abs(U - Uref) <= 1e-5 * scale + 1e-30), (label, float(np.max(np.abs(U - Uref) / (scale + 1e-300))))


@pytest.mark.parametrize("r", [1, 50, 64, 100, 128, 200])
def test_sketch_parity(lib, r):
    n, p = 3001, 700
    X = _nb(n, p, 5, True, 7)
    e, V = oracle.eigh_desc(oracle.gram_dense(X))
    rp, col, val = synth.dense_to_csr(X)
    U = _sketch_gpu(lib, rp, col, val, n, p, V, e, r)
    _check_sketch(X, V, e, r, U, f"r={r}")


def test_sketch_workload_100k_by_2000_r50(lib):
    X = _nb(100_000, 2000, 20, True, 2000)
    e, V = oracle.eigh_desc(oracle.gram_dense(X))
    rp, col, val = synth.dense_to_csr(X)
    U = _sketch_gpu(lib, rp, col, val, 100_000, 2000, V, e, 50)
    _check_sketch(X, V, e, 50, U, "100k")
    # the identity's consequence: orthonormal columns (up to the FP32 result)
    assert np.abs(U.astype(np.float64).T @ U - np.eye(50)).max() < 1e-4


def test_sketch_errors_and_binary(lib):
    rng = np.random.default_rng(5)
    X = (rng.random((80, 30)) < 0.2).astype(np.float32)
    e, V = oracle.eigh_desc(oracle.gram_dense(X))
    rp, col, _ = synth.dense_to_csr(X)
    U = _sketch_gpu(lib, rp, col, None, 80, 30, V, e, 10)
    _check_sketch(X, V, e, 10, U, "binary")
    with pytest.raises(lib.GmgmError) as ei:                # eigenvalue <= 0
        _sketch_gpu(lib, rp, col, None, 80, 30, V, np.concatenate([[-1.0], e[1:]]), 10)
    assert ei.value.status == 3
    with pytest.raises(lib.GmgmError) as ei:                # r > p (storage large enough)
        _sketch_gpu(lib, rp, col, None, 80, 30, np.hstack([V, V[:, :1]]), np.append(e, 1.0), 31)
    assert ei.value.status == 2
    bad = col.copy()
    bad[3] = 30
    with pytest.raises(lib.GmgmError) as ei:
        _sketch_gpu(lib, rp, bad, None, 80, 30, V, e, 10)
    assert ei.value.status == 2


def test_pipeline_gram_eigh_sketch_recompose(lib):
    """End to end on the 2000 x 500 workload: GPU Gram -> GPU eigh -> GPU sketch
    -> GPU top-k; the cell factor spans the oracle's (projector difference)
    and the top-k agrees with the oracle's on the GPU factor."""
    import torch
    n, p, r, k = 2000, 500, 100, 10
    X = _nb(n, p, 8, False, 1000)
    rp, col, val = synth.dense_to_csr(X)
    rpd, cd, vd = _dev(rp, col, val)
    G = lib.gram(rpd, cd, vd, n, p)
    w, Vt, rank = lib.eigh_small(G)
    assert rank == p
    U = lib.sketch(rpd, cd, vd, n, p, Vt, w, r)
    e_ref, V_ref = oracle.eigh_desc(oracle.gram_dense(X))
    Uref = oracle.cell_factor(X, V_ref, e_ref, r)
    Un = U.cpu().numpy().astype(np.float64)
    assert np.abs(Un @ Un.T - Uref @ Uref.T).max() < 1e-3
    psi = torch.from_numpy(1.0 / e_ref[:r]).cuda()
    out = lib.recompose_topk(U, psi, k, prec="bf16")
    rows = np.arange(0, n, 7)
    P = oracle.psi_rows(Un.astype(np.float32), 1.0 / e_ref[:r], rows)
    _, rcol, _ = oracle.topk_csr(P, rows, k)
    tie = oracle.near_tie_rows(P, rows, k)
    got = out.col.cpu().numpy().reshape(n, k)[rows]
    assert np.all((got == rcol.reshape(-1, k)).all(1) | tie)
