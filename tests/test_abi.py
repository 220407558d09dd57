"""CPU-side checks of the C ABI: the library loads, and exports every function that
include/ht.h declares (no compute calls: no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ht.h")
LIB = os.path.join(ROOT, "paper_0906_2704_amd", "libht.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ht_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for fn in ("ht_eigs", "ht_transform_inv", "ht_transform_fwd", "ht_tikhonov_filter", "ht_gcv_scan",
               "ht_plan_create", "ht_plan_destroy"):
        assert fn in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libht.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libht.so not built")
def test_status_strings_and_argument_validation_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.ht_status_str.restype = ctypes.c_char_p
    lib.ht_last_error.restype = ctypes.c_char_p
    assert lib.ht_status_str(0) == b"HT_OK"
    assert lib.ht_status_str(3) == b"HT_ERR_PSF_TOO_WIDE"
    # host-side validation fails before any device call
    out = ctypes.c_void_p()
    n = (ctypes.c_int64 * 1)(3)
    lib.ht_plan_create.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int64, ctypes.c_void_p]
    assert lib.ht_plan_create(1, n, 1, 1, 0, 1, ctypes.byref(out)) == 1
    assert b"n must be" in lib.ht_last_error()
    assert lib.ht_plan_create(3, n, 1, 1, 0, 1, ctypes.byref(out)) == 1
