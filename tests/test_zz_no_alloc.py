"""gmgm_recompose_topk_noalloc (the recomposition + top-k with its workspace in
a fixed device array) against gmgm_recompose_topk, through the C ABI.

Bar: identical CSR (both paths end in the same exact FP64 selection), and the
oracle's top-k on sampled rows as for gmgm_recompose_topk; two calls in a row,
the second smaller, so that the shared array holds the first call's contents;
rows that reach the FP32 re-sweep and the exact scan; a size beyond the array
rejected before launch; no device memory taken by the calls.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _dev(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()


def _own_context(lib):
    import torch
    h = ctypes.c_void_p()
    st = torch.cuda.current_stream().cuda_stream
    assert lib.load().gmgm_create(ctypes.byref(h), torch.cuda.current_device(), ctypes.c_void_p(st)) == 0
    return h


def _both(lib, ctx, V, psi, k, prec, **kw):
    Vd, pd = _dev(V, np.float32), _dev(psi, np.float64)
    a = lib.recompose_topk(Vd, pd, k, prec=prec, stats=True, noalloc=True, ctx=ctx, **kw)
    b = lib.recompose_topk(Vd, pd, k, prec=prec, stats=True, **kw)
    return a, b


def _same(a, b):
    for x, y in ((a.row_ptr, b.row_ptr), (a.col, b.col), (a.val, b.val)):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


def _oracle_rows(V, psi, k, rows, col, label):
    P = oracle.psi_rows(V, psi, rows)
    _, rcol, _ = oracle.topk_csr(P, rows, k)
    tie = oracle.near_tie_rows(P, rows, k)
    got = col.reshape(-1, k)[rows]
    ok = tie | np.all(got == rcol.reshape(-1, k), axis=1)
    assert ok.all(), f"{label}: rows {rows[~ok][:5]}"


def test_noalloc_matches_allocating_call_twice_in_a_row(lib):
    import torch
    ctx = _own_context(lib)
    try:
        # first call: 20000 cells, r = 100, BF16
        n1, r1, k1 = 20000, 100, 10
        V1 = synth.cell_factor_proxy(n1, r1, 12, seed=41)
        p1 = 1.0 / synth.spectrum_proxy(400, n1, 8, seed=41)[:r1]
        Vd, pd = _dev(V1, np.float32), _dev(p1, np.float64)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        a = lib.recompose_topk(Vd, pd, k1, prec="bf16", stats=True, noalloc=True, ctx=ctx)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        b = lib.recompose_topk(Vd, pd, k1, prec="bf16", stats=True)
        _same(a, b)
        rows = np.unique(np.concatenate([np.arange(40), np.arange(n1 - 40, n1),
                                         np.random.default_rng(1).integers(0, n1, 60)]))
        _oracle_rows(V1, p1, k1, rows, a.col.cpu().numpy(), "first call")
        # the allocating call's workspace here is tens of MiB; the fixed-array
        # call took none (allow for runtime-internal staging)
        assert free0 - free1 < 8 << 20, (free0, free1)
        # second, smaller call with rows that need the FP32 re-sweep and the exact scan
        from tests import _adversarial
        A = _adversarial.aligned_rounding_rows("bf16", k=10)
        a2, b2 = _both(lib, ctx, A["V"], A["psi"], 10, "bf16")
        _same(a2, b2)
        assert a2.stats["rows_fallback"] >= 2 and a2.stats["rows_exact"] >= 1, a2.stats
        n2 = A["V"].shape[0]
        _oracle_rows(A["V"], A["psi"], 10, np.arange(n2), a2.col.cpu().numpy(), "second call")
        # a row range of an FP32 call
        V3 = synth.cell_factor_proxy(3001, 33, 6, seed=42)
        p3 = 1.0 / synth.spectrum_proxy(64, 3001, 6, seed=42)[:33]
        a3, b3 = _both(lib, ctx, V3, p3, 7, "fp32", row_begin=17, row_end=2500)
        _same(a3, b3)
        # the streamed-contraction path (r = 300) with rows that need the exact panels
        A3 = _adversarial.aligned_rounding_rows("bf16", k=10, r=300)
        a4, b4 = _both(lib, ctx, A3["V"], A3["psi"], 10, "bf16")
        _same(a4, b4)
        assert a4.stats["rows_exact"] >= 1, a4.stats
        _oracle_rows(A3["V"], A3["psi"], 10, np.arange(A3["V"].shape[0]), a4.col.cpu().numpy(), "r=300")
    finally:
        lib.load().gmgm_destroy(ctx)


def test_noalloc_rejects_a_workspace_beyond_the_array(lib):
    import torch
    n, r = 1_000_000, 100
    V = torch.zeros(n, r, dtype=torch.float32, device="cuda")
    psi = torch.ones(r, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.GmgmError) as ei:
        lib.recompose_topk(V, psi, 10, prec="bf16", noalloc=True)
    assert ei.value.status == 2 and "exceeds the fixed" in str(ei.value)
    # the context stays usable
    out = lib.recompose_topk(V[:5000].contiguous(), psi, 10, prec="bf16", noalloc=True)
    assert out.col.numel() == 5000 * 10
