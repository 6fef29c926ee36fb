"""Number formats and layout tables of the library, checked on the CPU against
independent definitions (IEEE bfloat16 and OCP FP8 e4m3, round to nearest even)."""
import math
import struct

import numpy as np

from tests import _libs


def _bf16_ref(x):
    b = struct.unpack("<I", struct.pack("<f", x))[0]
    hi, lo = b >> 16, b & 0xFFFF
    if lo > 0x8000 or (lo == 0x8000 and hi & 1):
        hi += 1
    return hi & 0xFFFF


def _e4m3_values():
    """All finite non-negative e4m3 values by their definition (bias 7, 3 mantissa bits)."""
    vals = {}
    for e in range(16):
        for m in range(8):
            code = (e << 3) | m
            if code == 0x7F:
                continue                      # NaN
            v = m / 8 * 2.0 ** -6 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
            vals[code] = v
    return vals


def test_bf16_round_to_nearest_even():
    lib = _libs.probe_lib()
    rng = np.random.default_rng(0)
    xs = list(rng.standard_normal(2000).astype(np.float32)) + [1.0, -2.5, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 0.0]
    for x in xs:
        assert lib.probe_bf16_bits(float(x)) == _bf16_ref(float(x))


def test_e4m3_round_to_nearest_even_against_table():
    lib = _libs.probe_lib()
    table = _e4m3_values()
    codes = np.array(sorted(table))
    values = np.array([table[c] for c in codes])
    assert max(values) == 448.0
    for c, v in table.items():
        assert lib.probe_e4m3_decode(c) == v
        assert lib.probe_e4m3_bits(v) == c
        assert lib.probe_e4m3_bits(-v) == (c | 0x80 if v != 0 else lib.probe_e4m3_bits(-0.0))
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(0, 448, 3000), 2.0 ** rng.uniform(-12, 8.8, 3000)]).astype(np.float32)
    xs = xs[xs <= 448]
    for x in xs:
        x = float(x)
        d = np.abs(values - x)
        best = np.flatnonzero(d == d.min())
        if best.size > 1:                     # tie: even mantissa wins
            best = [b for b in best if codes[b] % 2 == 0]
        assert lib.probe_e4m3_bits(x) == codes[best[0]], x


def test_layout_tables_are_bijections():
    lib = _libs.probe_lib()
    # accumulator rows of the two lane halves cover 0..31 exactly once
    rows = sorted(lib.probe_acc_row(v, h) for v in range(16) for h in range(2))
    assert rows == list(range(32))
    # operand chunks cover each k of a padded tile exactly once
    for prec, ech, units in ((0, 4, 16), (1, 8, 8), (2, 16, 4)):
        ks = []
        for u in range(units):
            for h in range(2):
                k0 = lib.probe_chunk_k0(prec, u, h)
                ks.extend(range(k0, k0 + ech))
        assert sorted(ks) == list(range(units * 2 * ech))
