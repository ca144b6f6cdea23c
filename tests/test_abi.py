"""The C-ABI library loads and exports every entry point include/nsg.h
declares; host-side argument checks reject bad calls before any device work
(no compute calls here: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1707_00143_amd", "libnsg.so")
HDR = os.path.join(ROOT, "include", "nsg.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nsg_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnsg.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"{n} declared in nsg.h but not exported"


def test_host_argument_checks(lib):
    P = ctypes.c_void_p
    lib.nsg_last_error.restype = ctypes.c_char_p
    lib.nsg_search.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P]
    assert lib.nsg_search(None, None, 0, 10, 10, None, None, None) == -1
    assert b"index is NULL" in lib.nsg_last_error()
    lib.nsg_load_index.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_uint32,
                                   ctypes.c_int32, P, P, ctypes.POINTER(P)]
    out = P()
    fake = P(16)   # never dereferenced: rejected before any copy
    assert lib.nsg_load_index(fake, 0, 8, fake, 4, 0, 0, None, None, ctypes.byref(out)) == -1
    assert lib.nsg_load_index(fake, 10, 8, fake, 4, 10, 0, None, None, ctypes.byref(out)) == -1
    assert b"navigating node" in lib.nsg_last_error()
    assert lib.nsg_load_index(fake, 10, 8, fake, 200, 0, 0, None, None, ctypes.byref(out)) == -1
    assert lib.nsg_load_index(fake, 10, 2000, fake, 4, 0, 0, None, None, ctypes.byref(out)) == -1
    assert lib.nsg_load_index(fake, 10, 8, fake, 4, 0, 7, None, None, ctypes.byref(out)) == -1
    lib.nsg_knn_bruteforce.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, P, P, P]
    assert lib.nsg_knn_bruteforce(fake, 100, fake, 5, 8, 0, 0, fake, fake, None) == -1
    assert lib.nsg_knn_bruteforce(fake, 100, fake, 5, 8, 1000, 0, fake, fake, None) == -1
    assert lib.nsg_knn_bruteforce(fake, 100, fake, 0, 8, 10, 0, fake, fake, None) == 0   # empty batch
    lib.nsg_set_stop_mode.argtypes = [P, ctypes.c_int32, ctypes.c_float]
    assert lib.nsg_set_stop_mode(None, 1, 1.0) == -1


def test_oracle_shares_no_code_with_gpu_library():
    ora = open(os.path.join(ROOT, "oracle", "nsg_oracle.c")).read()
    assert "#include" in ora and "nsg.h" not in ora and "common.hpp" not in ora
    for f in os.listdir(os.path.join(ROOT, "paper_1707_00143_amd", "csrc")):
        src = open(os.path.join(ROOT, "paper_1707_00143_amd", "csrc", f)).read()
        assert "oracle" not in src.lower()
    pkg = open(os.path.join(ROOT, "paper_1707_00143_amd", "__init__.py")).read()
    assert "import oracle" not in pkg
