"""The C ABI library loads and exports every entry point include/dp.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2004_11658_amd", "libdp.so")
HDR = os.path.join(ROOT, "include", "dp.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["dp_init", "dp_compute", "dp_free", "dp_status", "dp_workspace_size"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdp.so not built")
def test_error_strings_without_device():
    lib = ctypes.CDLL(LIB)
    lib.dp_strerror.restype = ctypes.c_char_p
    assert lib.dp_strerror(0) == b"ok"
    assert b"workspace" in lib.dp_strerror(-6)
