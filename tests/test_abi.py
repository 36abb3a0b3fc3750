"""The C-ABI library loads and exports every function include/spdhss.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spdhss.h")
LIB = os.path.join(ROOT, "paper_2011_07632_amd", "libspdhss.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:spd_status|void|const char\*)\s+([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("h2_build", "spdhss_build", "ulv_factor", "ulv_apply", "h2_matvec", "pcg_solve"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_rejects_bad_arguments_without_a_device():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2011_07632_amd import binding as B
    # null arguments are rejected before any device work
    out = ctypes.c_void_p()
    code = B.lib.spdhss_build(None, None, None, ctypes.byref(out))
    assert code == B.SPD_E_INVALID and out.value is None
    assert b"null" in B.lib.spd_last_error()
