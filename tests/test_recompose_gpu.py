"""Parity of gmgm_recompose_topk (HIP, through the C ABI) with the CPU oracle.

Bar: top-k index sets identical to the oracle's except on rows the oracle flags
as near ties (k-th and (k+1)-th |Psi| within 1e-6 relative); values within
1e-5 relative of the FP64 value (scale: sum_k |W_ik V_jk|).  Inputs are
seeded synthetic cell factors; psi comes from a synthetic spectrum.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import _libs

pytestmark = pytest.mark.gpu

PRECS = ("fp32", "bf16", "fp8")


def _psi(r, seed, n=4000):
    return 1.0 / synth.spectrum_proxy(max(r, 64), n, 6, seed=seed)[:r]


def _run(lib, V, psi, k, prec, row_begin=0, row_end=None, cand_cap=0, stats=True):
    import torch
    Vd = torch.from_numpy(np.ascontiguousarray(V, dtype=np.float32)).cuda()
    pd = torch.from_numpy(np.ascontiguousarray(psi, dtype=np.float64)).cuda()
    out = lib.recompose_topk(Vd, pd, k, prec=prec, row_begin=row_begin, row_end=row_end,
                             cand_cap=cand_cap, stats=stats)
    return out.row_ptr.cpu().numpy(), out.col.cpu().numpy(), out.val.cpu().numpy(), out.stats


def _check(V, psi, k, rows, rp, col, val, label):
    rows = np.asarray(rows)
    m = rows.size
    assert rp.shape == (m + 1,) and np.array_equal(rp, np.arange(m + 1) * k), label
    P = oracle.psi_rows(V, psi, rows)
    _, rcol, rval = oracle.topk_csr(P, rows, k)
    tie = oracle.near_tie_rows(P, rows, k)
    col = col.reshape(m, k)
    val = val.reshape(m, k)
    rcol = rcol.reshape(m, k)
    same = np.all(col == rcol, axis=1)
    bad = ~same & ~tie
    assert not bad.any(), f"{label}: index mismatch on rows {rows[bad][:8]} (got {col[bad][:2]}, want {rcol[bad][:2]})"
    # values: the emitted value of each emitted (i, j) against FP64
    W = np.asarray(V, np.float64)[rows] * psi[None, :]
    Vj = np.asarray(V, np.float64)[col.ravel()].reshape(m, k, -1)
    exact = np.einsum("mr,mkr->mk", W, Vj)
    scale = np.einsum("mr,mkr->mk", np.abs(W), np.abs(Vj))
    assert np.all(np.abs(val - exact) <= 1e-5 * scale + 1e-30), label
    assert np.all(np.diff(col, axis=1) > 0), label
    assert np.all(col != rows[:, None]), label
    return tie.sum()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,r,k,seed", [(70, 5, 3, 1), (1000, 50, 10, 2), (2053, 100, 10, 3),
                                        (4096, 128, 16, 4), (1500, 1, 5, 5), (3001, 33, 24, 6)])
def test_parity_structured(lib, prec, n, r, k, seed):
    V = synth.cell_factor_proxy(n, r, 6, seed=seed)
    psi = _psi(r, seed)
    rp, col, val, st = _run(lib, V, psi, k, prec, cand_cap=32 if k > 12 else 0)
    _check(V, psi, k, np.arange(n), rp, col, val, f"{prec} n={n} r={r} k={k}")
    assert st["rows_fallback"] <= n


@pytest.mark.parametrize("prec", PRECS)
def test_parity_gaussian_and_row_range(lib, prec):
    rng = np.random.default_rng(11)
    n, r, k = 5000, 64, 10
    V = rng.standard_normal((n, r)).astype(np.float32)
    psi = rng.random(r) + 0.05
    for b, e in ((0, n), (31, 97), (4090, 5000), (1234, 1235)):
        rp, col, val, _ = _run(lib, V, psi, k, prec, row_begin=b, row_end=e)
        _check(V, psi, k, np.arange(b, e), rp, col, val, f"{prec} rows [{b},{e})")


@pytest.mark.parametrize("prec", PRECS)
def test_edge_k_equals_n_minus_1_and_tiny_n(lib, prec):
    rng = np.random.default_rng(12)
    for n, k in ((2, 1), (3, 2), (25, 24), (33, 20)):
        V = rng.standard_normal((n, 7)).astype(np.float32)
        psi = rng.random(7) + 0.1
        rp, col, val, _ = _run(lib, V, psi, k, prec, cand_cap=32)
        _check(V, psi, k, np.arange(n), rp, col, val, f"{prec} n={n} k={k}")


@pytest.mark.parametrize("prec", PRECS)
def test_exact_ties_go_to_smaller_column(lib, prec):
    """Duplicate rows with small-integer entries give exactly equal Psi values."""
    rng = np.random.default_rng(13)
    base = rng.integers(-3, 4, size=(40, 8)).astype(np.float32)
    V = np.concatenate([base, base, base[:17]], axis=0)          # 97 rows, many exact duplicates
    psi = rng.integers(1, 5, size=8).astype(np.float64)
    k = 6
    rp, col, val, _ = _run(lib, V, psi, k, prec)
    rows = np.arange(V.shape[0])
    P = oracle.psi_rows(V, psi, rows)
    _, rcol, _ = oracle.topk_csr(P, rows, k)
    np.testing.assert_array_equal(col, rcol)


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_input_reports_domain_error(lib, bad):
    """A row whose values are all NaN reaches the exact fallback with fewer than
    k comparable columns; the call must stay memory-safe and report E_DOMAIN."""
    import torch
    V = torch.ones(64, 4, dtype=torch.float32, device="cuda")
    V[5, 2] = bad
    psi = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.GmgmError) as ei:
        lib.recompose_topk(V, psi, 3, prec="bf16")
    assert ei.value.status == 3
    lib.sync()                                   # the fault is reported once
    # the context stays usable
    out = lib.recompose_topk(torch.ones(64, 4, dtype=torch.float32, device="cuda") * 0.5, psi, 3)
    assert out.col.shape[0] == 64 * 3


def test_argument_errors(lib):
    import torch
    V = torch.ones(64, 4, dtype=torch.float32, device="cuda")
    psi = torch.ones(4, dtype=torch.float64, device="cuda")
    for kw, status in (({"k": 0}, 1), ({"k": 64}, 1), ({"k": 3, "row_begin": 10, "row_end": 5}, 2),
                       ({"k": 3, "cand_cap": 7}, 1), ({"k": 20, "cand_cap": 16}, 1)):
        k = kw.pop("k")
        with pytest.raises(lib.GmgmError) as ei:
            lib.recompose_topk(V, psi, k, **kw)
        assert ei.value.status == status
    W = torch.ones(4, 40000, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.GmgmError):
        lib.recompose_topk(W, torch.ones(40000, dtype=torch.float64, device="cuda"), 3)


def test_repeat_calls_are_deterministic(lib):
    V = synth.cell_factor_proxy(3000, 100, 8, seed=21)
    psi = _psi(100, 21)
    a = _run(lib, V, psi, 10, "bf16")
    b = _run(lib, V, psi, 10, "bf16")
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("prec", ("bf16", "fp32"))
def test_full_size_one_million_cells_sampled(lib, prec):
    """The benchmark's workload (1M cells, r = 100, k = 10): sampled rows against
    the oracle, every emitted value against FP64, CSR invariants on all rows."""
    import torch
    n, r, k = 1_000_000, 100, 10
    V = _full_V()
    psi = _psi(r, 3000, n=n)
    Vd = torch.from_numpy(V).cuda()
    pd = torch.from_numpy(psi).cuda()
    out = lib.recompose_topk(Vd, pd, k, prec=prec, stats=True)
    col = out.col.cpu().numpy().reshape(n, k)
    val = out.val.cpu().numpy().reshape(n, k)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.arange(32), np.arange(n - 32, n), rng.integers(0, n, 24)]))
    _check(V, psi, k, rows, np.arange(rows.size + 1) * k, col[rows].ravel(), val[rows].ravel(), prec)
    assert np.all(np.diff(col, axis=1) > 0)
    assert np.all(col != np.arange(n)[:, None]) and col.min() >= 0 and col.max() < n
    # every value equals the FP64 dot product (computed on the CPU in chunks)
    for lo in range(0, n, 100_000):
        hi = min(n, lo + 100_000)
        W = V[lo:hi].astype(np.float64) * psi[None, :]
        Vj = V[col[lo:hi].ravel()].astype(np.float64).reshape(hi - lo, k, r)
        exact = np.einsum("mr,mkr->mk", W, Vj)
        scale = np.einsum("mr,mkr->mk", np.abs(W), np.abs(Vj))
        assert np.all(np.abs(val[lo:hi] - exact) <= 1e-5 * scale)
    print(prec, out.stats, flush=True)


_FULL = {}


def _full_V():
    if "V" not in _FULL:
        _FULL["V"] = synth.cell_factor_proxy(1_000_000, 100, 40, seed=3000)
    return _FULL["V"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("k", [1, 10])
def test_aligned_rounding_rows_reach_the_fallbacks(lib, prec, k):
    """Rows built so that operand rounding puts a true top-k column below 32
    decoys (tests/_adversarial.py): the result must still equal the oracle's,
    the low-precision certificate must send the row to the FP32 re-sweep, and a
    row whose top values are 72 exact ties must reach the exact scan."""
    from tests import _adversarial
    A = _adversarial.aligned_rounding_rows("fp8" if prec == "fp8" else "bf16", k=k)
    V, psi = A["V"], A["psi"]
    n = V.shape[0]
    rp, col, val, st = _run(lib, V, psi, k, prec, cand_cap=32)
    _check(V, psi, k, np.arange(n), rp, col, val, f"{prec} adversarial k={k}")
    col = col.reshape(n, k)
    assert A["hidden"] in col[A["row"]]
    # the tie row is a near tie by construction; the exact scan still resolves
    # ties to the smaller column, as the oracle does
    assert list(col[A["tie_row"]]) == A["tie_cols"][:k]
    assert st["rows_fallback"] >= 2, st
    assert st["rows_exact"] >= 1, st
