"""In-bounds check of the gfx950 MFMA builtins' lane layouts the kernels assume.

A and B are filled lane by lane from small integers (exact in every format),
following the library's operand mapping (lane l: row/column l % 32, k slot
chosen by l / 32 and the element); the accumulator is compared element by
element with the plain product under the library's accumulator mapping.
"""
import ctypes

import numpy as np
import pytest

from tests import _libs

pytestmark = pytest.mark.gpu


def _bf16(x):
    return np.array(x, np.float32).view(np.uint32) >> 16      # small integers: exact truncation


def _e4m3(x):
    lib = _libs.probe_lib()
    return np.array([lib.probe_e4m3_bits(float(v)) for v in np.ravel(x)], np.uint32).reshape(np.shape(x))


@pytest.mark.parametrize("prec,kdim", [(0, 2), (1, 16), (2, 64)])
def test_mfma_32x32_layout(prec, kdim):
    import torch
    lib = _libs.probe_lib()
    rng = np.random.default_rng(prec)
    A = rng.integers(-2, 3, size=(32, kdim)).astype(np.float32)     # rows i, k
    B = rng.integers(-2, 3, size=(kdim, 32)).astype(np.float32)     # k, cols j
    per = kdim // 2                                                # k values per lane
    Ab = np.zeros((64, 8), np.uint32)
    Bb = np.zeros((64, 8), np.uint32)
    for l in range(64):
        i, h = l % 32, l // 32
        ks = [h * per + e for e in range(per)]
        a, b = A[i, ks], B[ks, i]
        if prec == 0:
            Ab[l, 0] = a.view(np.uint32)[0]
            Bb[l, 0] = b.view(np.uint32)[0]
        elif prec == 1:
            pa, pb = _bf16(a), _bf16(b)
            for q in range(4):
                Ab[l, q] = pa[2 * q] | (pa[2 * q + 1] << 16)
                Bb[l, q] = pb[2 * q] | (pb[2 * q + 1] << 16)
        else:
            pa, pb = _e4m3(a), _e4m3(b)
            for q in range(8):
                Ab[l, q] = sum(int(pa[4 * q + z]) << (8 * z) for z in range(4))
                Bb[l, q] = sum(int(pb[4 * q + z]) << (8 * z) for z in range(4))
    Ad = torch.from_numpy(Ab.view(np.int32)).cuda()
    Bd = torch.from_numpy(Bb.view(np.int32)).cuda()
    Dd = torch.zeros(64 * 16, dtype=torch.float32, device="cuda")
    assert lib.probe_mfma(prec, ctypes.c_void_p(Ad.data_ptr()), ctypes.c_void_p(Bd.data_ptr()),
                          ctypes.c_void_p(Dd.data_ptr())) == 0
    D = Dd.cpu().numpy().reshape(64, 16)
    ref = A @ B
    got = np.zeros((32, 32), np.float32)
    for l in range(64):
        for v in range(16):
            got[lib.probe_acc_row(v, l // 32), l % 32] = D[l, v]
    if not np.array_equal(got, ref):
        print("lane 0 acc:", D[0], "\nlane 32 acc:", D[32])
        print("ref col 0:", ref[:, 0])
    np.testing.assert_array_equal(got, ref)
