"""Parity of the symmetric form of gmgm_recompose_topk (BF16 operands, every
row of Psi; taken from 800,000 rows on, or forced with
GMGM_RECOMPOSE_PATH=symmetric) with the CPU oracle and with the full sweep of
the same library.

Bar: against the oracle as for the full sweep (index sets identical except on
near-tie rows, values within 1e-5 relative of FP64); against the full sweep:
identical CSR, since both emit the exact top k rounded once to float.  The
statistics say which form ran.
"""
import os

import numpy as np
import pytest

import synth
from tests import _adversarial
from tests.test_recompose_gpu import _check, _psi, _run

pytestmark = pytest.mark.gpu


class _path:
    def __init__(self, mode):
        self.mode = mode

    def __enter__(self):
        self.old = os.environ.get("GMGM_RECOMPOSE_PATH")
        os.environ["GMGM_RECOMPOSE_PATH"] = self.mode

    def __exit__(self, *exc):
        if self.old is None:
            os.environ.pop("GMGM_RECOMPOSE_PATH", None)
        else:
            os.environ["GMGM_RECOMPOSE_PATH"] = self.old


def _full_flops(n, kpad):
    return 2.0 * (32 * -(-n // 32)) * 32.0 * -(-n // 32) * kpad


def _kpad(r):
    return 32 if r <= 32 else 64 if r <= 64 else 112 if r <= 112 else 128


def _both(lib, V, psi, k, cand_cap=0):
    with _path("symmetric"):
        s = _run(lib, V, psi, k, "bf16", cand_cap=cand_cap)
    with _path("full"):
        f = _run(lib, V, psi, k, "bf16", cand_cap=cand_cap)
    return s, f


@pytest.mark.parametrize("n,r,k,seed", [(5000, 100, 10, 1), (4133, 64, 1, 2), (6000, 128, 24, 3),
                                        (3000, 32, 16, 4), (1100, 100, 10, 5), (2051, 7, 3, 6)])
def test_symmetric_matches_oracle_and_full_sweep(lib, n, r, k, seed):
    V = synth.cell_factor_proxy(n, r, 6, seed=seed)
    if seed == 1:
        V[[3, 700, 4999]] = 0.0       # rows without a bound: re-swept in full
    psi = _psi(r, seed)
    (rp, col, val, st), (rpf, colf, valf, stf) = _both(lib, V, psi, k, cand_cap=32 if k > 12 else 0)
    assert st["symmetric"] and not stf["symmetric"], (st, stf)
    assert stf["mfma_flops"] >= _full_flops(n, _kpad(r)), stf
    assert np.array_equal(rp, rpf) and np.array_equal(col, colf) and np.array_equal(val, valf)
    _check(V, psi, k, np.arange(n), rp, col, val, f"symmetric n={n} r={r} k={k}")
    if seed == 1:
        assert st["rows_fallback"] >= 3


def test_symmetric_at_200k_rows(lib):
    """Every row against the full sweep (the default), sampled rows (all
    clusters, the first and last tiles) against the oracle."""
    n, r, k = 200_000, 100, 10
    V = synth.cell_factor_proxy(n, r, 40, seed=21)
    psi = _psi(r, 21)
    with _path("symmetric"):
        rp, col, val, st = _run(lib, V, psi, k, "bf16")
    os.environ.pop("GMGM_RECOMPOSE_PATH", None)
    rpf, colf, valf, stf = _run(lib, V, psi, k, "bf16")
    # about half the column tiles plus a 1/8 sample, and the re-sweep of the
    # rows the first sweep cannot certify
    assert st["symmetric"] and not stf["symmetric"], (st, stf)
    assert st["mfma_flops"] < 0.75 * stf["mfma_flops"], (st, stf)
    assert np.array_equal(col, colf) and np.array_equal(val, valf)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([np.arange(40), np.arange(n - 40, n), rng.choice(n, 200, replace=False)]))
    sel = (rows[:, None] * k + np.arange(k)[None, :]).ravel()
    _check(V, psi, k, rows, np.arange(rows.size + 1) * k, col[sel], val[sel], "symmetric 200k sampled")


def test_symmetric_column_side_overflow_takes_the_full_sweep(lib):
    """Every |Psi_ij| equal (V of rank one): every value reaches its row's
    bound, the column side outgrows the per-wave buffers, and the call takes
    the full sweep; exact ties go to the smaller column."""
    n, r, k = 3000, 16, 5
    V = np.zeros((n, r), np.float32)
    V[:, 0] = 1.0
    psi = np.ones(r)
    with _path("symmetric"):
        rp, col, val, st = _run(lib, V, psi, k, "bf16")
    assert not st["symmetric"] and st["mfma_flops"] >= _full_flops(n, _kpad(r))
    col = col.reshape(n, k)
    want = np.array([[j for j in range(k + 1) if j != i][:k] for i in range(n)])
    assert np.array_equal(col, want)
    assert np.all(val == 1.0)


@pytest.mark.parametrize("k", [1, 10])
def test_symmetric_aligned_rounding_rows(lib, k):
    """The rows built so that BF16 rounding hides a true top-k column below 32
    decoys, and a row whose top values are 72 exact ties, among 16k rows of
    background: the symmetric form must still return the oracle's top k (the
    certificate sends these rows to the split-BF16 re-sweep, the tie row on to
    the exact scan)."""
    n = 16384
    A = _adversarial.aligned_rounding_rows("bf16", k=k, n=n)
    V, psi = A["V"].copy(), A["psi"]
    # background: clustered rows of norm 5 with zero mean over each half of
    # the coordinates, so nearly orthogonal to the special rows (constant on
    # each half up to a few entries): each side keeps its top k to itself,
    # and the background's rounding bound stays a few percent of its values
    special = np.zeros(n, bool)
    special[[A["row"], A["hidden"], A["tie_row"]] + list(A["d_cols"]) + list(A["s_cols"]) + list(A["tie_cols"])] = True
    B = synth.cell_factor_proxy(n, V.shape[1], 6, seed=30 + k).astype(np.float64)
    r1 = A["r1"]
    B[:, :r1] -= B[:, :r1].mean(axis=1, keepdims=True)
    B[:, r1:] -= B[:, r1:].mean(axis=1, keepdims=True)
    B *= 5.0 / np.linalg.norm(B, axis=1, keepdims=True)
    V[~special] = B[~special].astype(np.float32)
    with _path("symmetric"):
        rp, col, val, st = _run(lib, V, psi, k, "bf16", cand_cap=32)
    assert st["symmetric"], st
    rng = np.random.default_rng(k)
    rows = np.unique(np.concatenate([[A["row"], A["hidden"], A["tie_row"]], A["d_cols"], A["s_cols"],
                                     A["tie_cols"], np.arange(32), np.arange(n - 32, n),
                                     rng.choice(n, 200, replace=False)]))
    sel = (rows[:, None] * k + np.arange(k)[None, :]).ravel()
    _check(V, psi, k, rows, np.arange(rows.size + 1) * k, col[sel], val[sel], f"symmetric adversarial k={k}")
    col = col.reshape(n, k)
    assert A["hidden"] in col[A["row"]]
    assert list(col[A["tie_row"]]) == A["tie_cols"][:k]
    assert st["rows_fallback"] >= 2, st
    assert st["rows_exact"] >= 1, st


def test_size_rule_and_the_calls_that_stay_full(lib):
    """At 820,000 rows a BF16 call for every row takes the symmetric form by
    default; a row range, and GMGM_RECOMPOSE_PATH=full, take the full sweep.
    The rows they share are identical, and sampled rows match the oracle."""
    n, r, k = 820_000, 64, 10
    V = synth.cell_factor_proxy(n, r, 40, seed=41)
    psi = _psi(r, 41)
    os.environ.pop("GMGM_RECOMPOSE_PATH", None)
    rp, col, val, st = _run(lib, V, psi, k, "bf16")
    assert st["symmetric"], st
    b, e = 409_600, 411_203
    rpr, colr, valr, str_ = _run(lib, V, psi, k, "bf16", row_begin=b, row_end=e)
    assert not str_["symmetric"], str_
    assert np.array_equal(colr, col[b * k:e * k]) and np.array_equal(valr, val[b * k:e * k])
    with _path("full"):
        rpf, colf, valf, stf = _run(lib, V, psi, k, "bf16")
    assert not stf["symmetric"], stf
    assert np.array_equal(colf, col) and np.array_equal(valf, val)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.arange(16), np.arange(n - 16, n), rng.choice(n, 120, replace=False)]))
    sel = (rows[:, None] * k + np.arange(k)[None, :]).ravel()
    _check(V, psi, k, rows, np.arange(rows.size + 1) * k, col[sel], val[sel], "size rule 820k sampled")


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_symmetric_nonfinite_input_reports_domain_error(lib, bad):
    """A non-finite entry of V in the symmetric form: the call stays
    memory-safe and reports E_DOMAIN, and the context stays usable."""
    import torch
    V = torch.from_numpy(synth.cell_factor_proxy(2048, 16, 6, seed=50)).cuda()
    V[700, 3] = bad
    psi = torch.ones(16, dtype=torch.float64, device="cuda")
    with _path("symmetric"):
        with pytest.raises(lib.GmgmError) as ei:
            lib.recompose_topk(V, psi, 5, prec="bf16")
        assert ei.value.status == 3
        lib.sync()                                   # the fault is reported once
        V[700, 3] = 0.5
        out = lib.recompose_topk(V, psi, 5, prec="bf16", stats=True)
    assert out.col.shape[0] == 2048 * 5 and out.stats["symmetric"]


@pytest.mark.parametrize("n,r,k", [(5000, 100, 10), (3001, 128, 15), (2500, 40, 1)])
def test_symmetric_with_lists_of_16(lib, n, r, k):
    """cand_cap = 16 (the shorter lists: more rows go to the re-sweep) in the
    symmetric form: the same CSR as the full sweep and the oracle's top k."""
    V = synth.cell_factor_proxy(n, r, 6, seed=60 + k)
    psi = _psi(r, 60 + k)
    (rp, col, val, st), (rpf, colf, valf, stf) = _both(lib, V, psi, k, cand_cap=16)
    assert st["symmetric"] and not stf["symmetric"], (st, stf)
    assert np.array_equal(col, colf) and np.array_equal(val, valf)
    _check(V, psi, k, np.arange(n), rp, col, val, f"symmetric C=16 n={n} r={r} k={k}")
