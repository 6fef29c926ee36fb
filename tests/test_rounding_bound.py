"""The certificate's rounding constant (gmgm_rounding_bound, host arithmetic)
against independent emulations of the operand formats on the CPU.

The sweep's approximate value of Psi_ij = W_i . V_j uses W and V rounded to
the operand format; the certificate needs |Psi~ - Psi| <= c ||W_i|| ||V_j||.
Emulated here: IEEE bfloat16 and OCP FP8 e4m3 with round to nearest even (FP8
after a power-of-two scale that puts the row / tile maximum in (224, 448]);
products of rounded operands are summed exactly (FP64), so the emulation
measures the operand rounding that c must cover.  Inputs whose entries all
round the same way are the worst case for it.
"""

import numpy as np
import pytest

from tests import _adversarial, _libs


@pytest.fixture(scope="module")
def g():
    _libs.ensure_built()
    import paper_2407_19892_amd as pkg
    pkg.load()
    return pkg


def _bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even) and back."""
    x = np.asarray(x, np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    hi = b >> 16
    lo = b & 0xFFFF
    up = (lo > 0x8000) | ((lo == 0x8000) & ((hi & 1) == 1))
    hi = (hi + up.astype(np.uint64)) & 0xFFFF
    return (hi << 16).astype(np.uint32).view(np.float32)


def _e4m3_table():
    vals = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue                      # NaN
            vals.append(m / 8 * 2.0 ** -6 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7))
    vals = np.array(sorted(set(vals)))
    return vals


_E4M3 = _e4m3_table()


def _e4m3_round(y):
    """Nearest e4m3 value of |y| <= 448 (ties to the even code), sign kept."""
    y = np.asarray(y, np.float64)
    a = np.abs(y)
    idx = np.searchsorted(_E4M3, a)
    lo = _E4M3[np.clip(idx - 1, 0, _E4M3.size - 1)]
    hi = _E4M3[np.clip(idx, 0, _E4M3.size - 1)]
    dlo, dhi = a - lo, hi - a
    # codes are in value order, so the even code is the one at an even index
    lo_even = (np.clip(idx - 1, 0, _E4M3.size - 1) % 2) == 0
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ~lo_even)
    return np.sign(y) * np.where(pick_hi, hi, lo)


def _fp8_scale_exp(m):
    e = int(np.ceil(np.log2(m / 448.0)))
    while m > 448.0 * 2.0 ** e:
        e += 1
    while m <= 448.0 * 2.0 ** (e - 1):
        e -= 1
    return e


def _fp8(x, scale_max):
    e = _fp8_scale_exp(scale_max)
    return _e4m3_round(np.asarray(x, np.float64) * 2.0 ** -e) * 2.0 ** e


def _rounded_dot(prec, w, v, v_tile_max=None):
    w32 = np.asarray(w, np.float32)
    v32 = np.asarray(v, np.float32)
    if prec == "bf16":
        wr, vr = _bf16(w32), _bf16(v32)
    else:
        wr = _fp8(w32, np.abs(w32).max())
        vr = _fp8(v32, np.abs(v32).max() if v_tile_max is None else v_tile_max)
    return float(np.dot(np.asarray(wr, np.float64), np.asarray(vr, np.float64)))


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("r", [1, 7, 50, 100, 128])
def test_bound_covers_aligned_rounding(g, prec, r):
    c, kpad = g.rounding_bound(prec, r)
    assert kpad >= r
    u = _adversarial.U[prec]
    for a in (1 + u - u * u / 2, 1 - u / 2 + u * u / 2, 1 + u + u * u / 2):
        w = np.full(r, a, np.float32)
        exact = float(np.dot(w.astype(np.float64), w.astype(np.float64)))
        err = abs(_rounded_dot(prec, w, w) - exact)
        assert err <= c * exact, (prec, r, a, err / exact, c)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_bound_is_attained_up_to_accumulation_terms(g, prec):
    # both operands round down by ~u relative: the error reaches ~2u, which the
    # constant must cover and nearly equals (a bound of ~u, one unit roundoff
    # per product of two rounded operands, is not enough)
    r = 100
    c, _ = g.rounding_bound(prec, r)
    u = _adversarial.U[prec]
    w = np.full(r, 1 + u - u * u / 2, np.float32)
    exact = float(np.dot(w.astype(np.float64), w.astype(np.float64)))
    ratio = abs(_rounded_dot(prec, w, w) - exact) / exact
    assert ratio > 2 * u * (1 - 2 * u)
    assert ratio <= c < 1.2 * ratio + 1e-3 * u


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_bound_covers_random_operands(g, prec):
    rng = np.random.default_rng(3)
    for r in (5, 64, 100, 128):
        c, _ = g.rounding_bound(prec, r)
        for _ in range(200):
            w = rng.standard_normal(r).astype(np.float32) * np.float32(rng.uniform(0.01, 100))
            v = rng.standard_normal(r).astype(np.float32)
            exact = float(np.dot(w.astype(np.float64), v.astype(np.float64)))
            err = abs(_rounded_dot(prec, w, v) - exact)
            assert err <= c * np.linalg.norm(w.astype(np.float64)) * np.linalg.norm(v.astype(np.float64))


def test_fp32_bound_and_argument_checks(g):
    c, kpad = g.rounding_bound("fp32", 100)
    assert kpad == 104
    # FP32 rounding of W plus one FP32 ulp per accumulation step
    assert 2.0 ** -24 + 105 * 2.0 ** -23 <= c < 2.0 ** -24 + 2 * 106 * 2.0 ** -23
    with pytest.raises(g.GmgmError):
        g.rounding_bound("bf16", 0)


def _certify(approx, exact, k, cap, beta):
    """The finalize rule on one row: the sweep keeps the `cap` largest rounded
    values (ties to smaller j); candidates within 2 beta of the k-th are
    rescored exactly; the row is certified when the largest rounded value left
    out plus beta is below the exact k-th.  Returns (certified, chosen set)."""
    order = sorted(range(len(approx)), key=lambda j: (-approx[j], j))
    kept = order[:cap]
    ak = approx[kept[k - 1]]
    R = [j for j in kept if approx[j] >= ak - 2 * beta]
    top = sorted(R, key=lambda j: (-abs(exact[j]), j))[:k]
    T = abs(exact[top[-1]])
    m_out = max(approx[kept[cap - 1]] if len(order) > cap else -1.0, ak - 2 * beta)
    return m_out + beta < T, set(top)


@pytest.mark.parametrize("k", [1, 10])
def test_adversarial_rows_defeat_a_one_unit_bound_but_not_the_library_bound(g, k):
    """The GPU regression inputs, on the CPU: with a bound of one BF16 unit
    roundoff per rounded operand pair (2^-9 per operand) the certificate accepts
    a wrong top-k set; the library's constant rejects the row."""
    cap = 32
    A = _adversarial.aligned_rounding_rows("bf16", k=k, cap=cap)
    V, i = A["V"], A["row"]
    cols = [A["hidden"]] + A["d_cols"] + A["s_cols"]
    W = V[i].astype(np.float64)
    exact = [float(np.dot(W, V[j].astype(np.float64))) for j in cols]
    approx = [_rounded_dot("bf16", V[i], V[j]) for j in cols]
    true_top = set(sorted(range(len(cols)), key=lambda q: (-exact[q], q))[:k])
    assert 0 in true_top                                   # the hidden column belongs to the top k
    assert approx[0] < min(approx[1:])                     # ... but rounds below every decoy
    scale = np.linalg.norm(W) * max(np.linalg.norm(V[j].astype(np.float64)) for j in range(V.shape[0]))
    d = 2.0 ** -9
    c_one_unit = (1 + 2.0 ** -24) * (1 + d) * (1 + d) - 1
    ok_old, chosen_old = _certify(approx, exact, k, cap, c_one_unit * scale)
    assert ok_old and chosen_old != true_top               # the unsound bound certifies a wrong set
    c, _ = g.rounding_bound("bf16", V.shape[1])
    ok_new, _ = _certify(approx, exact, k, cap, c * scale)
    assert not ok_new                                      # the library's bound sends the row on


def test_large_rank_requests_report_the_precision_that_runs(g):
    """Above r = 4096 the streamed sweep runs every request with FP32 operands
    (the BF16 bound certifies no row there): the reported constant is FP32's."""
    c32, k32 = g.rounding_bound("fp32", 5000)
    for prec in ("bf16", "fp8"):
        c, kpad = g.rounding_bound(prec, 5000)
        assert (c, kpad) == (c32, k32)
    cb, _ = g.rounding_bound("bf16", 4096)
    assert cb > 4 * g.rounding_bound("fp32", 4096)[0]          # 4096 still runs BF16

