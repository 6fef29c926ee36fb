"""Parity of gmgm_recompose_threshold (HIP, through the C ABI) with the CPU
oracle's thresholded graph: every j != i with |Psi_ij| >= thr, ascending.

Bar: the kept (i, j) sets identical to the oracle's except for entries within
1e-9 relative of the threshold (their side depends on the FP64 summation
order); values within 1e-5 relative of the FP64 value (scale: sum_k
|W_ik V_jk|); the output identical across precisions.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import significance as SG

pytestmark = pytest.mark.gpu

PRECS = ("fp32", "bf16", "fp8")


def _dev(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()


def _run(lib, V, psi, thr, prec, **kw):
    out = lib.recompose_threshold(_dev(V, np.float32), _dev(psi, np.float64), thr, prec=prec, **kw)
    return out.row_ptr.cpu().numpy(), out.col.cpu().numpy(), out.val.cpu().numpy(), out.nnz


def _check(V, psi, thr, rows, rp, col, val, label):
    rows = np.asarray(rows)
    P = oracle.psi_rows(V, psi, rows)
    near = SG.near_threshold(P, rows, thr)
    rrp, rcol, _ = SG.threshold_csr(P, rows, thr)
    assert rp.shape == (rows.size + 1,) and rp[0] == 0 and np.all(np.diff(rp) >= 0), label
    for t, i in enumerate(rows):
        got = col[rp[t]:rp[t + 1]]
        want = rcol[rrp[t]:rrp[t + 1]]
        assert np.all(np.diff(got) > 0), label
        diff = np.setxor1d(got, want)
        assert np.all(near[t, diff]), f"{label}: row {i} differs at {diff[:8]}"
    # values against FP64
    ri = np.repeat(rows, np.diff(rp))
    W = np.asarray(V, np.float64)[ri] * psi[None, :]
    Vj = np.asarray(V, np.float64)[col]
    exact = np.sum(W * Vj, axis=1)
    scale = np.sum(np.abs(W) * np.abs(Vj), axis=1)
    assert np.all(np.abs(val - exact) <= 1e-5 * scale + 1e-30), label
    assert np.all(col != ri), label
    return rp[-1]


def _psi(r, seed):
    return 1.0 / synth.spectrum_proxy(max(r, 64), 4000, 6, seed=seed)[:r]


def _quantile_thr(V, psi, frac, seed=0):
    """A threshold that keeps about `frac` of a row's entries."""
    rng = np.random.default_rng(seed)
    rows = rng.choice(V.shape[0], size=min(64, V.shape[0]), replace=False)
    P = np.abs(oracle.psi_rows(V, psi, rows))
    return float(np.quantile(P, 1.0 - frac))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,r,frac,seed", [(70, 5, 0.1, 1), (2053, 100, 0.004, 3), (4096, 128, 0.002, 4),
                                           (1500, 1, 0.01, 5), (3001, 33, 0.003, 6)])
def test_threshold_parity_structured(lib, prec, n, r, frac, seed):
    V = synth.cell_factor_proxy(n, r, 6, seed=seed)
    psi = _psi(r, seed)
    thr = _quantile_thr(V, psi, frac, seed)
    rp, col, val, nnz = _run(lib, V, psi, thr, prec)
    assert nnz == col.size
    _check(V, psi, thr, np.arange(n), rp, col, val, f"{prec} n={n} r={r}")


def test_threshold_same_output_every_precision(lib):
    V = synth.cell_factor_proxy(3000, 100, 8, seed=21)
    psi = _psi(100, 21)
    thr = _quantile_thr(V, psi, 0.003, 21)
    outs = [_run(lib, V, psi, thr, p) for p in PRECS]
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        np.testing.assert_array_equal(o[1], outs[0][1])
        np.testing.assert_array_equal(o[2], outs[0][2])


@pytest.mark.parametrize("prec", PRECS)
def test_threshold_row_ranges(lib, prec):
    rng = np.random.default_rng(11)
    n, r = 5000, 64
    V = rng.standard_normal((n, r)).astype(np.float32)
    psi = rng.random(r) + 0.05
    thr = _quantile_thr(V, psi, 0.002, 11)
    for b, e in ((0, n), (31, 97), (4090, 5000), (1234, 1235)):
        rp, col, val, _ = _run(lib, V, psi, thr, prec, row_begin=b, row_end=e)
        _check(V, psi, thr, np.arange(b, e), rp, col, val, f"{prec} rows [{b},{e})")


@pytest.mark.parametrize("prec", PRECS)
def test_candidate_overflow_goes_to_exact_scan(lib, prec):
    """Row 0 is a multiple s > 1 of 1100 identical rows u, and the threshold
    sits just above s |u|^2: every Psi_0j (j <= 1100) is a candidate within the
    rounding bound but none is kept; the sweep's room (1024 per row) overflows
    and the row is decided by the exact scan."""
    rng = np.random.default_rng(14)
    r = 40
    u = rng.standard_normal(r).astype(np.float32)
    rest = rng.standard_normal((900, r)).astype(np.float32) * 0.05
    V = np.concatenate([(1.5 * u)[None, :], np.repeat(u[None, :], 1100, axis=0), rest], axis=0)
    psi = np.ones(r)
    P0 = oracle.psi_rows(V, psi, [0])[0]
    hi, lo = float(np.abs(P0[1]) * (1.0 + 1e-5)), float(np.abs(P0[1]) * (1.0 - 1e-5))
    rp, col, val, nnz = _run(lib, V, psi, hi, prec)
    _check(V, psi, hi, np.arange(V.shape[0]), rp, col, val, f"{prec} overflow, none kept")
    assert rp[1] == 0
    # just below s |u|^2: row 0 keeps the 1100 copies (each copy keeps column 0)
    with pytest.raises(lib.GmgmError) as ei:
        _run(lib, V, psi, lo, prec, max_per_row=8)
    assert ei.value.status == 5
    rp, col, val, nnz = _run(lib, V, psi, lo, prec)
    assert rp[1] == 1100 and nnz == 2200
    _check(V, psi, lo, np.arange(V.shape[0]), rp, col, val, f"{prec} overflow, 1100 kept")


def test_capacity_retry_and_errors(lib):
    V = synth.cell_factor_proxy(1000, 50, 6, seed=7)
    psi = _psi(50, 7)
    thr = _quantile_thr(V, psi, 0.01, 7)
    full = _run(lib, V, psi, thr, "bf16", capacity=100_000)
    for cap in (0, 1, 100):                      # too small: the binding resizes once
        small = _run(lib, V, psi, thr, "bf16", capacity=cap)
        for a, b in zip(full, small):
            np.testing.assert_array_equal(a, b)
    Vd, pd = _dev(V, np.float32), _dev(psi, np.float64)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(lib.GmgmError) as ei:
            lib.recompose_threshold(Vd, pd, bad)
        assert ei.value.status == 3
    Vn = V.copy()
    Vn[3, 1] = np.nan
    with pytest.raises(lib.GmgmError) as ei:
        lib.recompose_threshold(_dev(Vn, np.float32), pd, thr)
    assert ei.value.status == 3
    lib.sync()
    assert lib.recompose_threshold(Vd, pd, thr).nnz == full[3]


def test_significance_threshold_end_to_end(lib):
    """Theorem 3's threshold from a synthetic count matrix's trace, applied to
    the cell axis recomposed from the oracle's eigenvalue MLE.  (At this size
    no edge is significant, as the paper notes the test is weak; the same
    factor is therefore also thresholded at a level that keeps a few edges.)"""
    from oracle import solver as S
    n, p, r = 3000, 300, 40
    X, _, _ = synth.nb_log1p(n, p, 6, zipf=True, seed=31)
    e, Vg = oracle.eigh_desc(oracle.gram_dense(X))
    U = oracle.cell_factor(X, Vg, e, r).astype(np.float32)
    psi = S.solve_eigs(S.Problem([e[:r].copy(), e.copy()], [(0, 1)])).lam[0]
    trace = float(np.sum(np.asarray(X, np.float64) ** 2))
    thr = lib.significance_threshold(n, [n * p], [trace], 0.05)
    assert abs(thr - SG.significance_threshold(n, [n * p], [trace], 0.05)) <= 1e-12 * thr
    for t in (thr, _quantile_thr(U, psi, 0.003, 31)):
        rp, col, val, nnz = _run(lib, U, psi, t, "bf16")
        _check(U, psi, t, np.arange(n), rp, col, val, f"significance thr={t}")


def test_full_size_one_million_cells_sampled(lib):
    """The benchmark's workload (1M cells, r = 100) at a threshold that keeps
    about ten entries per row: sampled rows against the oracle, every emitted
    value against FP64, CSR invariants on all rows."""
    import torch
    n, r = 1_000_000, 100
    V = synth.cell_factor_proxy(n, r, 40, seed=3000)
    psi = np.ascontiguousarray(1.0 / synth.spectrum_proxy(20_000, n, 48, seed=3000)[:r])
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.arange(16), np.arange(n - 16, n), rng.integers(0, n, 16)]))
    P = oracle.psi_rows(V, psi, rows)
    A = np.abs(P)
    A[np.arange(rows.size), rows] = 0.0
    thr = float(np.median(-np.sort(-A, axis=1)[:, 9]))          # the median 10th largest |Psi|
    out = lib.recompose_threshold(torch.from_numpy(V).cuda(), torch.from_numpy(psi).cuda(), thr, prec="bf16")
    rp, col, val = out.row_ptr.cpu().numpy(), out.col.cpu().numpy(), out.val.cpu().numpy()
    assert rp[0] == 0 and rp[-1] == out.nnz and np.all(np.diff(rp) >= 0)
    near = SG.near_threshold(P, rows, thr)
    rrp, rcol, _ = SG.threshold_csr(P, rows, thr)
    for t, i in enumerate(rows):
        got = col[rp[i]:rp[i + 1]]
        diff = np.setxor1d(got, rcol[rrp[t]:rrp[t + 1]])
        assert np.all(near[t, diff]), f"row {i} differs at {diff[:8]}"
    ri = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(col != ri) and col.min() >= 0 and col.max() < n
    for lo in range(0, out.nnz, 2_000_000):
        hi = min(out.nnz, lo + 2_000_000)
        W = V[ri[lo:hi]].astype(np.float64) * psi[None, :]
        Vj = V[col[lo:hi]].astype(np.float64)
        exact = np.sum(W * Vj, axis=1)
        scale = np.sum(np.abs(W) * np.abs(Vj), axis=1)
        assert np.all(np.abs(val[lo:hi] - exact) <= 1e-5 * scale)
        assert np.all(np.abs(exact) >= thr * (1 - 1e-9))
    same_row = ri[1:] == ri[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])          # ascending within rows
    print("threshold", thr, "nnz", out.nnz, flush=True)


@pytest.mark.parametrize("prec", PRECS)
def test_aligned_rounding_rows_keep_the_hidden_entry(lib, prec):
    """A threshold between a row's true largest |Psi_ij| and everything else,
    on inputs whose operand rounding pulls that entry furthest below it
    (tests/_adversarial.py): the entry must still be kept, as in the oracle."""
    from tests import _adversarial
    A = _adversarial.aligned_rounding_rows("fp8" if prec == "fp8" else "bf16", k=1)
    V, psi, thr = A["V"], A["psi"], A["thr"]
    n = V.shape[0]
    rp, col, val, nnz = _run(lib, V, psi, thr, prec)
    _check(V, psi, thr, np.arange(n), rp, col, val, f"{prec} adversarial")
    i, h = A["row"], A["hidden"]
    assert list(col[rp[i]:rp[i + 1]]) == [h]
    assert list(col[rp[h]:rp[h + 1]]) == [i]
    assert nnz == 2
