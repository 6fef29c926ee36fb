"""Parity of gmgm_recompose_topk with ranks above 128 and k up to 64 (the
K-loop sweep) with the CPU oracle, through the C ABI.

Algorithm 1's final loop recomposes every axis, the gene axis at its full
rank.  Bar as for the register-resident path: index sets identical to the
oracle's except on near-tie rows (k-th and (k+1)-th |Psi| within 1e-6
relative); values within 1e-5 of the FP64 value (scale sum_t |W_it V_jt|).

Inputs: the 2000 cells x 500 genes workload end to end through the oracle
(NB/log1p data, Gram, eigendecomposition, cell factor, eigenvalue MLE), both
axes at full rank (r = 500); the gene axis of the 100k x 2000 workload at its
shape (2000 x 2000, r = 2000: an orthogonal factor and eigenvalues from the
eigenvalue MLE of Marchenko-Pastur + spike spectra at r_c = 50); the gene axis
of the 1M x 20k workload at its shape (20k x 20k, r = 20k, Gaussian factor,
sampled rows); ragged sizes, row ranges, k up to 64, and rows that need the
FP32 re-sweep and the exact panels.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import solver as S
from tests import _adversarial

pytestmark = pytest.mark.gpu


def _run(lib, V, psi, k, prec, **kw):
    import torch
    Vd = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float32)).cuda()
    pd = torch.from_numpy(np.ascontiguousarray(psi, dtype=np.float64)).cuda()
    out = lib.recompose_topk(Vd, pd, k, prec=prec, stats=True, **kw)
    return out.row_ptr.cpu().numpy(), out.col.cpu().numpy(), out.val.cpu().numpy(), out.stats


def _check(V, psi, k, rows, col, val, label, all_rows=None):
    """col / val hold the CSR of `all_rows` (default: rows); compare `rows`."""
    rows = np.asarray(rows)
    all_rows = rows if all_rows is None else np.asarray(all_rows)
    pos = np.searchsorted(all_rows, rows)
    col = col.reshape(-1, k)[pos]
    val = val.reshape(-1, k)[pos]
    P = oracle.psi_rows(V, psi, rows)
    _, rcol, _ = oracle.topk_csr(P, rows, k)
    tie = oracle.near_tie_rows(P, rows, k)
    rcol = rcol.reshape(-1, k)
    bad = ~np.all(col == rcol, axis=1) & ~tie
    assert not bad.any(), f"{label}: rows {rows[bad][:6]} got {col[bad][:1]} want {rcol[bad][:1]}"
    W = np.asarray(V, np.float64)[rows] * psi[None, :]
    for t in range(rows.size):
        Vj = np.asarray(V[col[t]], np.float64)
        exact = Vj @ W[t]
        scale = np.abs(Vj) @ np.abs(W[t])
        assert np.all(np.abs(val[t] - exact) <= 1e-5 * scale + 1e-30), label
    assert np.all(np.diff(col, axis=1) > 0) and np.all(col != rows[:, None]), label
    return int(tie.sum())


_CFG0 = {}


def _config0():
    """2000 cells x 500 genes (8 equal clusters): oracle Gram, eigenpairs, cell
    factor and the eigenvalue MLE with both axes at full rank."""
    if not _CFG0:
        X, _, _ = synth.nb_log1p(2000, 500, 8, zipf=False, seed=1000)
        eg, Vg = oracle.eigh_desc(oracle.gram_dense(X))
        Vc = oracle.cell_factor(X, Vg, eg, 500)
        sol = S.solve_eigs(S.Problem([eg.copy(), eg.copy()], [(0, 1)]))
        _CFG0.update(Vc=Vc.astype(np.float32), Vg=Vg.astype(np.float32), psi=sol.lam[0], phi=sol.lam[1])
    return _CFG0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("axis", ["cells", "genes"])
def test_workload_2000x500_both_axes_full_rank(lib, prec, axis):
    c = _config0()
    V, lam = (c["Vc"], c["psi"]) if axis == "cells" else (c["Vg"], c["phi"])
    n = V.shape[0]
    rp, col, val, st = _run(lib, V, lam, 10, prec)
    assert np.array_equal(rp, np.arange(n + 1) * 10)
    _check(V, lam, 10, np.arange(n), col, val, f"{axis} {prec}")


def test_gene_axis_at_2000_by_2000(lib):
    rng = np.random.default_rng(2000)
    Q, _ = np.linalg.qr(rng.standard_normal((2000, 2000)))
    e = synth.spectrum_proxy(2000, 100_000, 20, seed=2000)
    phi = S.solve_eigs(S.Problem([e[:50].copy(), e.copy()], [(0, 1)])).lam[1]
    V = Q.astype(np.float32)
    for prec in ("fp32", "bf16"):
        _, col, val, st = _run(lib, V, phi, 10, prec)
        _check(V, phi, 10, np.arange(2000), col, val, f"2000x2000 {prec}")
        print(prec, st, flush=True)


def test_gene_axis_at_20k_by_20k_sampled_rows(lib):
    import torch
    n = r = 20_000
    rng = np.random.default_rng(3000)
    V = (rng.standard_normal((n, r), dtype=np.float32) / np.float32(np.sqrt(r)))
    phi = 1.0 / synth.spectrum_proxy(20_000, 1_000_000, 40, seed=3000)
    rows = np.unique(np.concatenate([np.arange(8), np.arange(n - 8, n), rng.integers(0, n, 8)]))
    for prec in ("fp32", "bf16"):
        _, col, val, st = _run(lib, V, phi, 10, prec)
        _check(V, phi, 10, rows, col, val, f"20k {prec}", all_rows=np.arange(n))
        c2 = col.reshape(n, 10)
        assert np.all(np.diff(c2, axis=1) > 0) and np.all(c2 != np.arange(n)[:, None])
        print(prec, st, flush=True)
        del col, val
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("n,r,k", [(3001, 300, 10), (1000, 777, 25), (2500, 200, 64), (4096, 129, 1),
                                   (700, 64, 40), (33, 150, 32)])
def test_ragged_sizes_and_large_k(lib, prec, n, r, k):
    if n > r:
        V = synth.cell_factor_proxy(n, r, 6, seed=n + r)
    else:                                   # fewer rows than the rank: a Gaussian factor
        V = (np.random.default_rng(n + r).standard_normal((n, r)) / np.sqrt(r)).astype(np.float32)
    psi = 1.0 / synth.spectrum_proxy(max(r, 64) * 3, 4 * max(r, 64), 6, seed=r)[:r]
    _, col, val, _ = _run(lib, V, psi, k, prec)
    _check(V, psi, k, np.arange(n), col, val, f"{prec} n={n} r={r} k={k}")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_row_ranges(lib, prec):
    V = synth.cell_factor_proxy(2600, 260, 6, seed=9)
    psi = 1.0 / synth.spectrum_proxy(800, 2600, 6, seed=9)[:260]
    for b, e in ((0, 2600), (31, 97), (2500, 2600), (1234, 1235)):
        rp, col, val, _ = _run(lib, V, psi, 12, prec, row_begin=b, row_end=e)
        assert np.array_equal(rp, np.arange(e - b + 1) * 12)
        _check(V, psi, 12, np.arange(b, e), col, val, f"{prec} rows [{b},{e})")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fallbacks_at_large_rank(lib, prec):
    """Aligned-rounding rows and a block of 72 exact ties at r = 300: the BF16
    certificate sends rows on, and the tie row reaches the exact panels."""
    A = _adversarial.aligned_rounding_rows("bf16", k=10, r=300)
    V, psi = A["V"], A["psi"]
    n = V.shape[0]
    _, col, val, st = _run(lib, V, psi, 10, prec)
    _check(V, psi, 10, np.arange(n), col, val, f"{prec} adversarial r=300")
    c2 = col.reshape(n, 10)
    assert A["hidden"] in c2[A["row"]]
    assert list(c2[A["tie_row"]]) == A["tie_cols"][:10]
    assert st["rows_fallback"] >= 1 and st["rows_exact"] >= 1, st


def test_k_limit_and_errors(lib):
    import torch
    V = torch.ones(100, 200, dtype=torch.float32, device="cuda")
    psi = torch.ones(200, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.GmgmError) as ei:
        lib.recompose_topk(V, psi, 65)
    assert ei.value.status == 1
    with pytest.raises(lib.GmgmError) as ei:
        lib.recompose_topk(V, psi, 10, cand_cap=16)          # the K-loop lists are 32, 64 or 128
    assert ei.value.status == 1
    big = torch.ones(4, 40000, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.GmgmError) as ei:
        lib.recompose_topk(big, torch.ones(40000, dtype=torch.float64, device="cuda"), 2)
    assert ei.value.status == 2
