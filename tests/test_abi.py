"""The C-ABI library loads without a GPU and exports every declared entry point."""
import ctypes
import subprocess

from tests import _libs


def test_library_exports_every_declared_symbol():
    _libs.ensure_built()
    lib = ctypes.CDLL(_libs.MAIN)
    declared = _libs.declared_functions()
    assert "gmgm_recompose_topk" in declared
    missing = [name for name in declared if not hasattr(lib, name)]
    assert not missing, f"declared but not exported: {missing}"
    out = subprocess.run(["nm", "-D", "--defined-only", _libs.MAIN], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared:
        assert name in exported


def test_binding_signatures_cover_header():
    import paper_2407_19892_amd as g
    assert set(_libs.declared_functions()) == set(g.SIGNATURES)


def test_version_callable_without_gpu():
    import paper_2407_19892_amd as g
    lib = g.load()
    assert lib.gmgm_version() >= 100


def test_null_context_is_rejected_without_gpu():
    import paper_2407_19892_amd as g
    lib = g.load()
    assert lib.gmgm_sync(None) == 1          # GMGM_E_ARG
    assert lib.gmgm_last_error(None) == b"null context"
