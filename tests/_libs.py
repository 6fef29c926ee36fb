"""Locating (and, when absent, building) the compiled libraries for tests."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MAIN = os.path.join(ROOT, "paper_2407_19892_amd", "libgmgm.so")
PROBE = os.path.join(ROOT, "tests", "probe", "libgmgm_probe.so")
HEADER_DIR = os.path.join(ROOT, "include")


def ensure_built():
    if not (os.path.exists(MAIN) and os.path.exists(PROBE)):
        import __graft_entry__
        __graft_entry__.build()


def probe_lib():
    ensure_built()
    lib = ctypes.CDLL(PROBE)
    lib.probe_bf16_bits.restype = ctypes.c_uint
    lib.probe_bf16_bits.argtypes = [ctypes.c_float]
    lib.probe_e4m3_bits.restype = ctypes.c_uint
    lib.probe_e4m3_bits.argtypes = [ctypes.c_float]
    lib.probe_e4m3_decode.restype = ctypes.c_float
    lib.probe_e4m3_decode.argtypes = [ctypes.c_uint]
    lib.probe_acc_row.restype = ctypes.c_int
    lib.probe_acc_row.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.probe_chunk_k0.restype = ctypes.c_int
    lib.probe_chunk_k0.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.probe_mfma.restype = ctypes.c_int
    lib.probe_mfma.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def declared_functions():
    """Names of the functions declared in include/*.h."""
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(gmgm_[a-z0-9_]+)\s*\(", text):
            names.append(m.group(1))
    return sorted(set(names))
