"""Python binding of libgmgm, the gfx950 HIP hot path of the multi-axis
Kronecker-sum Gaussian graphical model (arXiv 2407.19892).

Argument marshalling only: every step runs in the library's HIP kernels.
Torch provides device memory (output tensors) and the current HIP stream.
Loading fails loudly when the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmgm.so")

PREC = {"fp32": 0, "bf16": 1, "fp8": 2}
STATUS = {0: "OK", 1: "E_ARG", 2: "E_SHAPE", 3: "E_DOMAIN", 4: "E_NOCONV", 5: "E_OVERFLOW",
          6: "E_HIP", 7: "E_NOMEM"}

_lib = None
_ctx = {}


class GmgmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gmgm {STATUS.get(status, status)}: {msg}")
        self.status = status


class TopkStats(ctypes.Structure):
    _fields_ = [("cand_total", ctypes.c_int64), ("rows_fallback", ctypes.c_int64),
                ("rows_near_tie", ctypes.c_int64), ("rows_exact", ctypes.c_int64),
                ("mfma_flops", ctypes.c_double), ("symmetric", ctypes.c_int64)]


class Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_flat", ctypes.c_int32), ("warm_used", ctypes.c_int32), ("kkt", ctypes.c_double),
                ("n_pinned", ctypes.c_int64 * 8), ("eps", ctypes.c_double * 8)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32

# name -> (restype, argtypes)
SIGNATURES = {
    "gmgm_version": (ctypes.c_int, []),
    "gmgm_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    "gmgm_destroy": (None, [_P]),
    "gmgm_set_stream": (ctypes.c_int, [_P, _P]),
    "gmgm_last_error": (ctypes.c_char_p, [_P]),
    "gmgm_sync": (ctypes.c_int, [_P]),
    "gmgm_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "gmgm_kernel_times": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "gmgm_recompose_topk": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _I64, _I64, _I32, ctypes.c_int,
                                           _I32, _P, _P, _P, ctypes.POINTER(TopkStats)]),
    "gmgm_recompose_topk_noalloc": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _I64, _I64, _I32, ctypes.c_int,
                                                   _I32, _P, _P, _P, ctypes.POINTER(TopkStats)]),
    "gmgm_recompose_threshold": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _I64, _I64, ctypes.c_double, ctypes.c_int,
                                                _I32, _P, _P, _P, _I64, ctypes.POINTER(_I64)]),
    "gmgm_significance_threshold": (ctypes.c_int, [_P, _I64, _I32, ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                                   ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "gmgm_rounding_bound": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32)]),
    "gmgm_gram": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, _P, _P, _P]),
    "gmgm_gram_shifted": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "gmgm_sketch_shifted": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _I64, _P, _I64, _P, _P]),
    "gmgm_skeptic": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "gmgm_eigh_small": (ctypes.c_int, [_P, _I64, _P, _P, _P, ctypes.POINTER(_I64)]),
    "gmgm_sketch": (ctypes.c_int, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _I64, _P, _I64, _P]),
    "gmgm_ws_param_count": (_I64, []),
    "gmgm_ws_init": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "gmgm_ws_features": (ctypes.c_int, [_P, _P, _I64, _P, _I64, ctypes.c_double, ctypes.c_double, _P]),
    "gmgm_ws_targets": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, _I64, _P]),
    "gmgm_ws_forward": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "gmgm_ws_train_step": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I32, _P, _P, _P, ctypes.c_float,
                                          ctypes.c_float, ctypes.POINTER(ctypes.c_double), _P]),
    "gmgm_ws_apply": (ctypes.c_int, [_P, _P, _P, _I64, _P, _I64, _P, _P]),
    "gmgm_warmstart_state_bytes": (_I64, []),
    "gmgm_warmstart_state_init": (ctypes.c_int, [_P, _P, ctypes.c_float]),
    "gmgm_warmstart_infer": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "gmgm_warmstart_train_step": (ctypes.c_int, [_P, _P, _P, _I32, _P, _P, _P, ctypes.c_float,
                                                 ctypes.POINTER(ctypes.c_float)]),
    "gmgm_csr_transpose": (ctypes.c_int, [_P, Csr, _P, _P, _P]),
    "gmgm_subspace_eig": (ctypes.c_int, [_P, _I32, ctypes.POINTER(Csr), ctypes.POINTER(Csr), _P, _I64, _I32, _I64,
                                         _P, _P]),
    "gmgm_solve_eigs": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_P), _I32,
                                       ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(_P), ctypes.c_double, _I32, ctypes.POINTER(_P),
                                       ctypes.POINTER(SolveInfo)]),
    "gmgm_solve_eigs_tensor": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_P), _I32,
                                              ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_P),
                                              ctypes.c_double, _I32, ctypes.POINTER(_P),
                                              ctypes.POINTER(SolveInfo)]),
}


def load(path: str = LIB_PATH):
    """Load libgmgm.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _stream_handle(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def context(device=None):
    """The library context of `device`, re-pointed at torch's current stream."""
    import torch
    lib = load()
    dev = torch.cuda.current_device() if device is None else int(device)
    st = _stream_handle(dev)
    c = _ctx.get(dev)
    if c is None:
        h = _P()
        s = lib.gmgm_create(ctypes.byref(h), dev, _P(st))
        if s != 0:
            raise GmgmError(s, f"gmgm_create(device={dev}) failed")
        c = h
        _ctx[dev] = c
    else:
        _check(c, lib.gmgm_set_stream(c, _P(st)))
    return c


def _check(c, status):
    if status != 0:
        raise GmgmError(status, load().gmgm_last_error(c).decode())


def _ptr(t):
    return _P(t.data_ptr())


def sync(device=None):
    c = context(device)
    _check(c, load().gmgm_sync(c))


def set_timing(enable: bool, device=None):
    c = context(device)
    _check(c, load().gmgm_set_timing(c, 1 if enable else 0))


def kernel_times(device=None):
    """(total ms, count) of the timed dominant-kernel launches since the last query."""
    c = context(device)
    tot = ctypes.c_double()
    cnt = _I64()
    _check(c, load().gmgm_kernel_times(c, ctypes.byref(tot), ctypes.byref(cnt)))
    return tot.value, cnt.value


@dataclass
class TopkResult:
    row_ptr: "object"
    col: "object"
    val: "object"
    stats: dict | None = None


def recompose_topk(V, psi, k: int, prec: str = "bf16", row_begin: int = 0, row_end: int | None = None,
                   cand_cap: int = 0, stats: bool = False, check: bool = True, out=None,
                   noalloc: bool = False, ctx=None) -> TopkResult:
    """CSR of the per-row top-k of Psi = V diag(psi) V^T (see gmgm_recompose_topk;
    noalloc=True calls gmgm_recompose_topk_noalloc, which allocates nothing).
    ctx: a context handle to use instead of the device's shared one."""
    import torch
    if not (V.is_cuda and psi.is_cuda):
        raise ValueError("V and psi must be device tensors")
    if V.dtype != torch.float32 or psi.dtype != torch.float64:
        raise TypeError("V must be float32 and psi float64")
    if not V.is_contiguous() or not psi.is_contiguous() or V.dim() != 2:
        raise ValueError("V must be a contiguous 2-D tensor and psi contiguous")
    n, r = V.shape
    if psi.numel() != r:
        raise ValueError("psi must have r entries")
    row_end = n if row_end is None else row_end
    rows = max(0, row_end - row_begin)
    if out is None:
        rp = torch.empty(rows + 1, dtype=torch.int64, device=V.device)
        col = torch.empty(rows * k, dtype=torch.int32, device=V.device)
        val = torch.empty(rows * k, dtype=torch.float32, device=V.device)
    else:
        rp, col, val = out
    c = context(V.device.index) if ctx is None else ctx
    st = TopkStats() if stats else None
    fn = load().gmgm_recompose_topk_noalloc if noalloc else load().gmgm_recompose_topk
    _check(c, fn(c, n, r, _ptr(V), _ptr(psi), row_begin, row_end, k, PREC[prec], cand_cap, _ptr(rp), _ptr(col),
                 _ptr(val), ctypes.byref(st) if st is not None else None))
    if check:
        _check(c, load().gmgm_sync(c))
    sd = None
    if st is not None:
        sd = {"cand_total": st.cand_total, "rows_fallback": st.rows_fallback,
              "rows_near_tie": st.rows_near_tie, "rows_exact": st.rows_exact,
              "mfma_flops": st.mfma_flops, "symmetric": bool(st.symmetric)}
    return TopkResult(rp, col, val, sd)


@dataclass
class ThresholdResult:
    row_ptr: "object"
    col: "object"
    val: "object"
    nnz: int


def recompose_threshold(V, psi, thr: float, prec: str = "bf16", row_begin: int = 0, row_end: int | None = None,
                        max_per_row: int = 0, capacity: int | None = None) -> ThresholdResult:
    """CSR of every |Psi_ij| >= thr, j != i, of Psi = V diag(psi) V^T (see
    gmgm_recompose_threshold).  The output arrays first get `capacity` entries
    (default 16 per row); when the library reports more, they are resized to
    the reported count and the call is repeated once."""
    import torch
    if not (V.is_cuda and psi.is_cuda):
        raise ValueError("V and psi must be device tensors")
    if V.dtype != torch.float32 or psi.dtype != torch.float64:
        raise TypeError("V must be float32 and psi float64")
    if not V.is_contiguous() or not psi.is_contiguous() or V.dim() != 2:
        raise ValueError("V must be a contiguous 2-D tensor and psi contiguous")
    n, r = V.shape
    if psi.numel() != r:
        raise ValueError("psi must have r entries")
    row_end = n if row_end is None else row_end
    rows = max(0, row_end - row_begin)
    cap = rows * 16 if capacity is None else capacity
    c = context(V.device.index)
    rp = torch.empty(rows + 1, dtype=torch.int64, device=V.device)
    for attempt in range(2):
        col = torch.empty(max(cap, 1), dtype=torch.int32, device=V.device)
        val = torch.empty(max(cap, 1), dtype=torch.float32, device=V.device)
        nnz = _I64(0)
        st = load().gmgm_recompose_threshold(c, n, r, _ptr(V), _ptr(psi), row_begin, row_end, float(thr),
                                              PREC[prec], max_per_row, _ptr(rp), _ptr(col), _ptr(val), cap,
                                              ctypes.byref(nnz))
        if st == 5 and attempt == 0 and nnz.value > cap and "capacity" in load().gmgm_last_error(c).decode():
            cap = nnz.value
            continue
        _check(c, st)
        break
    return ThresholdResult(rp, col[:nnz.value], val[:nnz.value], nnz.value)


def significance_threshold(d_l: int, d_all, trace_s, alpha: float = 0.05, n_tests: float = 0.0) -> float:
    """Theorem 3's threshold for axis l (see gmgm_significance_threshold; host
    arithmetic, no device needed)."""
    d_all = [float(x) for x in d_all]
    trace_s = [float(x) for x in trace_s]
    if len(d_all) != len(trace_s):
        raise ValueError("d_all and trace_s must have one entry per modality")
    m = len(d_all)
    arr = ctypes.c_double * m
    out = ctypes.c_double(0.0)
    st = load().gmgm_significance_threshold(None, int(d_l), m, arr(*d_all), arr(*trace_s), float(alpha),
                                            float(n_tests), ctypes.byref(out))
    if st != 0:
        raise GmgmError(st, "gmgm_significance_threshold rejected its arguments")
    return out.value


def rounding_bound(prec: str, r: int):
    """(c, kpad): the certificate's rounding constant and padded MFMA depth
    (see gmgm_rounding_bound; host arithmetic, no device needed)."""
    c = ctypes.c_double(0.0)
    kp = _I32(0)
    st = load().gmgm_rounding_bound(PREC[prec], int(r), ctypes.byref(c), ctypes.byref(kp))
    if st != 0:
        raise GmgmError(st, "gmgm_rounding_bound rejected its arguments")
    return c.value, kp.value


@dataclass
class SolveResult:
    lam: list
    info: dict


def solve_eigs(E, modalities, eps=None, warm=None, tol: float = 1e-12, max_iter: int = 200,
               raise_on_noconv: bool = True) -> SolveResult:
    """Eigenvalue MLE over the box lambda >= eps (see gmgm_solve_eigs).

    E: list of FP64 device tensors (one per axis); modalities: list of (a, b)
    axis pairs; warm: optional list of FP64 device tensors.  Returns the
    per-axis eigenvalues (new device tensors) and the solve record."""
    import torch
    L = len(E)
    for e in E:
        if not (e.is_cuda and e.dtype == torch.float64 and e.dim() == 1 and e.is_contiguous()):
            raise TypeError("every E must be a contiguous 1-D float64 device tensor")
    if warm is not None:
        if len(warm) != L:
            raise ValueError("warm needs one tensor per axis")
        for w, e in zip(warm, E):
            if not (w.is_cuda and w.dtype == torch.float64 and w.is_contiguous() and w.numel() == e.numel()):
                raise TypeError("warm tensors must be contiguous float64 device tensors shaped like E")
    out = [torch.empty_like(e) for e in E]
    ranks = (_I64 * L)(*[e.numel() for e in E])
    eptr = (_P * L)(*[e.data_ptr() for e in E])
    optr = (_P * L)(*[o.data_ptr() for o in out])
    flat = [int(x) for ab in modalities for x in ab]
    mods = (_I32 * len(flat))(*flat)
    epsa = (ctypes.c_double * L)(*eps) if eps is not None else None
    wptr = (_P * L)(*[w.data_ptr() for w in warm]) if warm is not None else None
    info = SolveInfo()
    c = context(E[0].device.index)
    st = load().gmgm_solve_eigs(c, L, ranks, eptr, len(modalities), mods, epsa, wptr, float(tol),
                                int(max_iter), optr, ctypes.byref(info))
    d = {"iterations": info.iterations, "converged": bool(info.converged), "n_flat": info.n_flat,
         "warm_used": bool(info.warm_used),
         "kkt": info.kkt, "n_pinned": list(info.n_pinned[:L]), "eps": list(info.eps[:L])}
    if st == 4 and not raise_on_noconv:
        return SolveResult(out, d)
    _check(c, st)
    return SolveResult(out, d)


def solve_eigs_tensor(E, modalities, eps=None, warm=None, tol: float = 1e-12, max_iter: int = 200,
                      raise_on_noconv: bool = True) -> SolveResult:
    """Eigenvalue MLE for modalities of any number of axes (see
    gmgm_solve_eigs_tensor).  E: list of FP64 device tensors (one per axis);
    modalities: list of axis tuples (each of two or more distinct axes)."""
    import torch
    L = len(E)
    for e in E:
        if not (e.is_cuda and e.dtype == torch.float64 and e.dim() == 1 and e.is_contiguous()):
            raise TypeError("every E must be a contiguous 1-D float64 device tensor")
    if warm is not None:
        if len(warm) != L:
            raise ValueError("warm needs one tensor per axis")
        for w, e in zip(warm, E):
            if not (w.is_cuda and w.dtype == torch.float64 and w.is_contiguous() and w.numel() == e.numel()):
                raise TypeError("warm tensors must be contiguous float64 device tensors shaped like E")
    out = [torch.empty_like(e) for e in E]
    ranks = (_I64 * L)(*[e.numel() for e in E])
    eptr = (_P * L)(*[e.data_ptr() for e in E])
    optr = (_P * L)(*[o.data_ptr() for o in out])
    lens = (_I32 * len(modalities))(*[len(m) for m in modalities])
    flat = [int(a) for m in modalities for a in m]
    axes = (_I32 * max(1, len(flat)))(*flat)
    epsa = (ctypes.c_double * L)(*eps) if eps is not None else None
    wptr = (_P * L)(*[w.data_ptr() for w in warm]) if warm is not None else None
    info = SolveInfo()
    c = context(E[0].device.index)
    st = load().gmgm_solve_eigs_tensor(c, L, ranks, eptr, len(modalities), lens, axes, epsa, wptr, float(tol),
                                       int(max_iter), optr, ctypes.byref(info))
    d = {"iterations": info.iterations, "converged": bool(info.converged), "n_flat": info.n_flat,
         "warm_used": bool(info.warm_used),
         "kkt": info.kkt, "n_pinned": list(info.n_pinned[:L]), "eps": list(info.eps[:L])}
    if st == 4 and not raise_on_noconv:
        return SolveResult(out, d)
    _check(c, st)
    return SolveResult(out, d)


def _csr_args(row_ptr, col, val, n):
    import torch
    if not (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.numel() == n + 1):
        raise TypeError("row_ptr must be an int64 device tensor of n + 1 entries")
    if not (col.is_cuda and col.dtype == torch.int32):
        raise TypeError("col must be an int32 device tensor")
    if val is not None and not (val.is_cuda and val.dtype == torch.float32 and val.numel() == col.numel()):
        raise TypeError("val must be a float32 device tensor like col (or None)")
    for t in (row_ptr, col) + ((val,) if val is not None else ()):
        if not t.is_contiguous():
            raise ValueError("CSR tensors must be contiguous")
    return _ptr(row_ptr), _ptr(col), (_ptr(val) if val is not None else None), col.numel()


@dataclass
class SkepticResult:
    val: "object"      # S's values at X's entries (FP32)
    z: "object"        # per-column value of the zeros (FP64)
    csum: "object"     # column sums of S (FP64)


def skeptic(row_ptr, col, val, n: int, p: int) -> SkepticResult:
    """Nonparanormal Skeptic of the CSR matrix X kept sparse: X~ = S + 1 z^T
    (see gmgm_skeptic).  S shares X's row_ptr and col."""
    import torch
    rp, cp, vp, nnz = _csr_args(row_ptr, col, val, n)
    dev = row_ptr.device
    out = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)
    z = torch.empty(p, dtype=torch.float64, device=dev)
    cs = torch.empty(p, dtype=torch.float64, device=dev)
    c = context(dev.index)
    _check(c, load().gmgm_skeptic(c, n, p, nnz, rp, cp, vp, _ptr(out), _ptr(z), _ptr(cs)))
    return SkepticResult(out[:nnz], z, cs)


def gram(row_ptr, col, val, n: int, p: int, out=None, check: bool = True, shift=None):
    """G = X^T X (p x p, FP32) of the CSR matrix X (n x p); see gmgm_gram.
    With shift = (z, csum) (e.g. from skeptic), the Gram of X + 1 z^T
    (gmgm_gram_shifted)."""
    import torch
    rp, cp, vp, nnz = _csr_args(row_ptr, col, val, n)
    G = torch.empty(p, p, dtype=torch.float32, device=row_ptr.device) if out is None else out
    c = context(row_ptr.device.index)
    if shift is None:
        _check(c, load().gmgm_gram(c, n, p, nnz, rp, cp, vp, _ptr(G)))
    else:
        z, cs = shift
        _check(c, load().gmgm_gram_shifted(c, n, p, nnz, rp, cp, vp, _ptr(z), _ptr(cs), _ptr(G)))
    if check:
        _check(c, load().gmgm_sync(c))
    return G


def eigh_small(G, vectors: bool = True):
    """(evals descending, evecs column-major as a (p, p) tensor whose ROW j is
    eigenvector j -- None with vectors=False --, numerical rank) of the
    symmetric FP32 Gram; see gmgm_eigh_small."""
    import torch
    if not (G.is_cuda and G.dtype == torch.float32 and G.dim() == 2 and G.shape[0] == G.shape[1]
            and G.is_contiguous()):
        raise TypeError("G must be a contiguous square float32 device tensor")
    p = G.shape[0]
    w = torch.empty(p, dtype=torch.float64, device=G.device)
    Vt = torch.empty(p, p, dtype=torch.float64, device=G.device) if vectors else None
    rank = _I64()
    c = context(G.device.index)
    _check(c, load().gmgm_eigh_small(c, p, _ptr(G), _ptr(w), _ptr(Vt) if vectors else None, ctypes.byref(rank)))
    return w, Vt, rank.value


def sketch(row_ptr, col, val, n: int, p: int, Vt, evals, r: int, out=None, check: bool = True, z=None):
    """U = X V[:, :r] diag(e[:r])^-1/2 (n x r FP32).  Vt is the column-major
    eigenvector storage returned by eigh_small (row j = eigenvector j).  With z,
    the factor of X + 1 z^T (gmgm_sketch_shifted)."""
    import torch
    rp, cp, vp, nnz = _csr_args(row_ptr, col, val, n)
    if not (Vt.is_cuda and Vt.dtype == torch.float64 and Vt.is_contiguous() and Vt.dim() == 2
            and Vt.shape[1] >= p and Vt.shape[0] >= r):
        raise TypeError("Vt must be a contiguous float64 device tensor of shape (>= r, >= p)")
    if not (evals.is_cuda and evals.dtype == torch.float64 and evals.numel() >= r):
        raise TypeError("evals must be a float64 device tensor with >= r entries")
    U = torch.empty(n, r, dtype=torch.float32, device=row_ptr.device) if out is None else out
    c = context(row_ptr.device.index)
    if z is None:
        _check(c, load().gmgm_sketch(c, n, p, nnz, rp, cp, vp, _ptr(Vt), Vt.shape[1], _ptr(evals), r, _ptr(U)))
    else:
        _check(c, load().gmgm_sketch_shifted(c, n, p, nnz, rp, cp, vp, _ptr(Vt), Vt.shape[1], _ptr(evals), r,
                                             _ptr(z), _ptr(U)))
    if check:
        _check(c, load().gmgm_sync(c))
    return U


# ---------------------------------------------------------------- learned warm start
WS_BINS = 512
WS_IN = 2 * WS_BINS + 4
WS_OUT = 2 * WS_BINS


def ws_param_count() -> int:
    return int(load().gmgm_ws_param_count())


def _f64_vec(t, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 1 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous 1-D float64 device tensor")


def _f32_dev(t, name, numel=None):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements")


def ws_init(params, seed: int):
    _f32_dev(params, "params", ws_param_count())
    c = context(params.device.index)
    _check(c, load().gmgm_ws_init(c, _ptr(params), int(seed) & 0xFFFFFFFFFFFFFFFF))


def ws_features(Ec, Eg, dc: float, dg: float, out=None):
    """The 1028 features of an axis pair (see gmgm_ws_features)."""
    import torch
    _f64_vec(Ec, "Ec")
    _f64_vec(Eg, "Eg")
    f = torch.empty(WS_IN, dtype=torch.float32, device=Ec.device) if out is None else out
    _f32_dev(f, "out", WS_IN)
    c = context(Ec.device.index)
    _check(c, load().gmgm_ws_features(c, _ptr(Ec), Ec.numel(), _ptr(Eg), Eg.numel(), float(dc), float(dg), _ptr(f)))
    return f


def ws_targets(Ec, lam_c, Eg, lam_g, out=None):
    import torch
    for t, nm in ((Ec, "Ec"), (lam_c, "lam_c"), (Eg, "Eg"), (lam_g, "lam_g")):
        _f64_vec(t, nm)
    if lam_c.numel() != Ec.numel() or lam_g.numel() != Eg.numel():
        raise ValueError("eigenvalue vectors must match their spectra")
    f = torch.empty(WS_OUT, dtype=torch.float32, device=Ec.device) if out is None else out
    _f32_dev(f, "out", WS_OUT)
    c = context(Ec.device.index)
    _check(c, load().gmgm_ws_targets(c, _ptr(Ec), _ptr(lam_c), Ec.numel(), _ptr(Eg), _ptr(lam_g), Eg.numel(),
                                     _ptr(f)))
    return f


def ws_forward(params, feats, out=None):
    import torch
    _f32_dev(params, "params", ws_param_count())
    _f32_dev(feats, "feats")
    B = feats.numel() // WS_IN
    if feats.numel() != B * WS_IN:
        raise ValueError("feats must be batch x 1028")
    y = torch.empty(B, WS_OUT, dtype=torch.float32, device=feats.device) if out is None else out
    c = context(feats.device.index)
    _check(c, load().gmgm_ws_forward(c, _ptr(params), B, _ptr(feats), _ptr(y)))
    return y


def ws_train_step(params, m, v, step: int, feats, target, mask=None, lr: float = 1e-3, weight_decay: float = 0.0,
                  want_loss: bool = True, grad_out=None):
    """One AdamW step; returns the loss before the update (None if not wanted)."""
    n = ws_param_count()
    for t, nm in ((params, "params"), (m, "adam_m"), (v, "adam_v")):
        _f32_dev(t, nm, n)
    _f32_dev(feats, "feats")
    B = feats.numel() // WS_IN
    _f32_dev(target, "target", B * WS_OUT)
    if mask is not None:
        _f32_dev(mask, "mask", B * WS_OUT)
    if grad_out is not None:
        _f32_dev(grad_out, "grad_out", n)
    loss = ctypes.c_double()
    c = context(feats.device.index)
    _check(c, load().gmgm_ws_train_step(c, _ptr(params), _ptr(m), _ptr(v), int(step), B, _ptr(feats), _ptr(target),
                                        _ptr(mask) if mask is not None else None, float(lr), float(weight_decay),
                                        ctypes.byref(loss) if want_loss else None,
                                        _ptr(grad_out) if grad_out is not None else None))
    return loss.value if want_loss else None


def ws_apply(curves, Ec, Eg):
    """Warm-start eigenvalues (lam_c, lam_g) from one 1024-long output row."""
    import torch
    _f32_dev(curves, "curves", WS_OUT)
    _f64_vec(Ec, "Ec")
    _f64_vec(Eg, "Eg")
    lc = torch.empty_like(Ec)
    lg = torch.empty_like(Eg)
    c = context(Ec.device.index)
    _check(c, load().gmgm_ws_apply(c, _ptr(curves), _ptr(Ec), Ec.numel(), _ptr(Eg), Eg.numel(), _ptr(lc), _ptr(lg)))
    return lc, lg



def warmstart_state(weight_decay: float = 0.0, device=None):
    """A zeroed AdamW state for warmstart_train_step (see gmgm_warmstart_state_init)."""
    import torch
    nbytes = int(load().gmgm_warmstart_state_bytes())
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else int(device))
    st = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    c = context(dev.index)
    _check(c, load().gmgm_warmstart_state_init(c, _ptr(st), float(weight_decay)))
    return st


def warmstart_infer(weights, feats, out=None):
    """out (batch x 1024) = the warm-start network of feats (see gmgm_warmstart_infer)."""
    import torch
    _f32_dev(weights, "weights", ws_param_count())
    _f32_dev(feats, "feats")
    B = feats.numel() // WS_IN
    if feats.numel() != B * WS_IN:
        raise ValueError("feats must be batch x 1028")
    y = torch.empty(B, WS_OUT, dtype=torch.float32, device=feats.device) if out is None else out
    c = context(feats.device.index)
    _check(c, load().gmgm_warmstart_infer(c, _ptr(weights), B, _ptr(feats), _ptr(y)))
    return y


def warmstart_train_step(weights, opt_state, feats, target, mask=None, lr: float = 1e-3, want_loss: bool = True):
    """One AdamW step with the update count kept in opt_state (see
    gmgm_warmstart_train_step); returns the loss before the update."""
    _f32_dev(weights, "weights", ws_param_count())
    _f32_dev(feats, "feats")
    B = feats.numel() // WS_IN
    _f32_dev(target, "target", B * WS_OUT)
    if mask is not None:
        _f32_dev(mask, "mask", B * WS_OUT)
    if opt_state.numel() != int(load().gmgm_warmstart_state_bytes()) or not opt_state.is_cuda:
        raise ValueError("opt_state must come from warmstart_state()")
    loss = ctypes.c_float()
    c = context(feats.device.index)
    _check(c, load().gmgm_warmstart_train_step(c, _ptr(weights), _ptr(opt_state), B, _ptr(feats), _ptr(target),
                                               _ptr(mask) if mask is not None else None, float(lr),
                                               ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


# ---------------------------------------------------------------- shared large axis
class CsrMatrix:
    """A device CSR matrix (row_ptr int64, col int32, val float32 or None)."""

    def __init__(self, row_ptr, col, val, n_rows: int, n_cols: int):
        _csr_args(row_ptr, col, val, n_rows)
        self.row_ptr, self.col, self.val = row_ptr, col, val
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)

    @property
    def nnz(self):
        return self.col.numel()

    def c_struct(self):
        return Csr(self.n_rows, self.n_cols, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                   self.val.data_ptr() if self.val is not None else None)

    def transpose(self):
        """X^T as a CsrMatrix (see gmgm_csr_transpose)."""
        import torch
        dev = self.row_ptr.device
        rp = torch.empty(self.n_cols + 1, dtype=torch.int64, device=dev)
        col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        val = torch.empty(self.nnz, dtype=torch.float32, device=dev)
        c = context(dev.index)
        _check(c, load().gmgm_csr_transpose(c, self.c_struct(), _ptr(rp), _ptr(col), _ptr(val)))
        _check(c, load().gmgm_sync(c))
        return CsrMatrix(rp, col, val, self.n_cols, self.n_rows)


def subspace_eig(blocks, omega, q: int, r: int, blocks_t=None):
    """(evals (r, FP64), vecs (n x r, FP32)) of D D^T, D = [X_1 | ...] (see
    gmgm_subspace_eig).  blocks: list of CsrMatrix sharing n_rows; omega:
    (sum p_m) x k FP64 device tensor; blocks_t: their transposes (built when None)."""
    import torch
    if blocks_t is None:
        blocks_t = [b.transpose() for b in blocks]
    if not (omega.is_cuda and omega.dtype == torch.float64 and omega.dim() == 2 and omega.is_contiguous()):
        raise TypeError("omega must be a contiguous 2-D float64 device tensor")
    P = sum(b.n_cols for b in blocks)
    if omega.shape[0] != P:
        raise ValueError(f"omega must have {P} rows")
    k = omega.shape[1]
    n = blocks[0].n_rows
    dev = omega.device
    evals = torch.empty(r, dtype=torch.float64, device=dev)
    vecs = torch.empty(n, r, dtype=torch.float32, device=dev)
    B = (Csr * len(blocks))(*[b.c_struct() for b in blocks])
    BT = (Csr * len(blocks))(*[b.c_struct() for b in blocks_t])
    c = context(dev.index)
    _check(c, load().gmgm_subspace_eig(c, len(blocks), B, BT, _ptr(omega), k, int(q), int(r), _ptr(evals),
                                       _ptr(vecs)))
    return evals, vecs
