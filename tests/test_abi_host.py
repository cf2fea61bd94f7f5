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


def test_library_never_allocates_device_or_pinned_memory():
    """The caller owns every device buffer: no allocation call in the library sources."""
    csrc = os.path.join(ROOT, "paper_2004_11658_amd", "csrc")
    bad = []
    for f in sorted(os.listdir(csrc)):
        src = open(os.path.join(csrc, f)).read()
        for call in ("hipMalloc", "hipHostMalloc", "hipMallocManaged", "hipExtMallocWithFlags",
                     "hipFree", "hipHostFree", "hipHostRegister"):
            if re.search(r"\b%s\s*\(" % call, src):
                bad.append((f, call))
    assert not bad, bad


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdp.so not built")
def test_init_rejects_bad_model_files_and_options(tmp_path):
    """Host-side validation of dp_init (no device needed: the model is parsed first)."""
    lib = ctypes.CDLL(LIB)
    lib.dp_init.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.dp_last_error.restype = ctypes.c_char_p
    lib.dp_last_error.argtypes = [ctypes.c_void_p]
    h = ctypes.c_void_p()
    p = tmp_path / "corrupt.bin"
    p.write_bytes(b"DPSEMDL1" + b"\x07" * 120)
    assert lib.dp_init(str(p).encode(), None, ctypes.byref(h)) == -2
    assert not h.value
    p.write_bytes(b"NOTAMODEL" * 20)
    assert lib.dp_init(str(p).encode(), None, ctypes.byref(h)) == -2
    assert b"magic" in lib.dp_last_error(None)
    assert lib.dp_init(str(tmp_path / "missing.bin").encode(), None, ctypes.byref(h)) == -2

    class Opt(ctypes.Structure):
        _fields_ = [("precision", ctypes.c_int32), ("deterministic", ctypes.c_int32), ("skin", ctypes.c_double)]
    bad = Opt(7, 0, 0.0)
    assert lib.dp_init(str(p).encode(), ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = Opt(0, 0, -1.0)
    assert lib.dp_init(str(p).encode(), ctypes.byref(bad), ctypes.byref(h)) == -1
