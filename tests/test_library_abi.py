"""The C-ABI library loads on the CPU and exports every declared entry point.

No compute call is made here (there is no GPU); only argument checks that fail
before any HIP call are exercised.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aiwc_rf.h")
LIB = os.path.join(ROOT, "paper_1811_00156_amd", "libaiwc_rf.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aiwc_rf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1811_00156_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), f"{name} is declared in aiwc_rf.h but not exported"


def test_binding_covers_the_header():
    from paper_1811_00156_amd import rf

    assert sorted(rf.SYMBOLS) == declared()


def test_argument_checks_without_gpu(lib):
    lib.aiwc_rf_bin.restype = ctypes.c_int
    lib.aiwc_rf_last_error.restype = ctypes.c_char_p
    P = ctypes.c_void_p
    lib.aiwc_rf_bin.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P]
    assert lib.aiwc_rf_bin(None, None, 10, 3, 1, 8, None, None, None) == -1
    assert b"null" in lib.aiwc_rf_last_error()
    buf = ctypes.create_string_buffer(64)
    h = ctypes.c_void_p()
    assert lib.aiwc_rf_bin(buf, buf, 0, 3, 1, 8, ctypes.byref(h), buf, None) == -1
    assert lib.aiwc_rf_bin(buf, buf, 10, 256, 1, 8, ctypes.byref(h), buf, None) == -1
    # column ids stay below the leaf marker 255: at most 254 features
    assert lib.aiwc_rf_bin(buf, buf, 10, 255, 1, 8, ctypes.byref(h), buf, None) == -1
    assert b"254" in lib.aiwc_rf_last_error()
    rc = lib.aiwc_rf_bin(buf, buf, 10, 254, 1, 8, ctypes.byref(h), buf, None)
    assert rc != 0 and b"p must" not in lib.aiwc_rf_last_error()  # passes the check, then needs a GPU
    assert lib.aiwc_rf_bin(buf, buf, 10, 3, 0, 8, ctypes.byref(h), buf, None) == -1
    assert lib.aiwc_rf_bin(buf, buf, 10, 3, 1, 1, ctypes.byref(h), buf, None) == -1
    lib.aiwc_rf_binner_from_counts.argtypes = [P, ctypes.c_int32, P]
    counts = (ctypes.c_int32 * 3)(4, 0, 2)
    assert lib.aiwc_rf_binner_from_counts(counts, 3, ctypes.byref(h)) == -1
    many = (ctypes.c_int32 * 256)(*([2] * 256))
    assert lib.aiwc_rf_binner_from_counts(many, 256, ctypes.byref(h)) == -1
    assert b"n_cols" in lib.aiwc_rf_last_error()
    rc = lib.aiwc_rf_binner_from_counts(many, 255, ctypes.byref(h))
    assert rc != 0 and b"n_cols" not in lib.aiwc_rf_last_error()  # 255 columns pass the check
    lib.aiwc_rf_server_submit.argtypes = [P, P, ctypes.c_int64, P, P]
    assert lib.aiwc_rf_server_submit(None, None, 1, None, None) == -1
    assert b"null" in lib.aiwc_rf_last_error()  # submit failures set the message too


def test_group_and_heldout_argument_checks_without_gpu(lib):
    P = ctypes.c_void_p
    lib.aiwc_rf_fit_groups.restype = ctypes.c_int
    lib.aiwc_rf_fit_groups.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, ctypes.c_int32,
                                       ctypes.c_uint32, P, P]
    h = ctypes.c_void_p()
    assert lib.aiwc_rf_fit_groups(None, 10, 3, None, None, None, None, None, 1, 0, ctypes.byref(h), None) == -1
    lib.aiwc_rf_heldout_error.restype = ctypes.c_int
    lib.aiwc_rf_heldout_error.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P]
    assert lib.aiwc_rf_heldout_error(None, 0, 1, None, None, None, None, None, None, None) == -1
    lib.aiwc_rf_heldout_rows.restype = ctypes.c_int
    lib.aiwc_rf_heldout_rows.argtypes = [P, ctypes.c_int32, P, P]
    n = ctypes.c_int32()
    assert lib.aiwc_rf_heldout_rows(None, 0, None, ctypes.byref(n)) == -1


PROBE_HEADER = os.path.join(ROOT, "include", "aiwc_rf_probe.h")
PROBE_LIB = os.path.join(ROOT, "paper_1811_00156_amd", "libaiwc_rf_probe.so")


def test_probe_library_exports_its_header():
    if not os.path.exists(PROBE_LIB):
        from paper_1811_00156_amd import build

        build.build()
    plib = ctypes.CDLL(PROBE_LIB)
    text = re.sub(r"/\*.*?\*/", "", open(PROBE_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(aiwc_rf_probe_[a-z0-9_]+)\s*\(", text)))
    assert names == ["aiwc_rf_probe_divide", "aiwc_rf_probe_last_error", "aiwc_rf_probe_lds_add"]
    for name in names:
        assert hasattr(plib, name), f"{name} is declared in aiwc_rf_probe.h but not exported"
    P = ctypes.c_void_p
    plib.aiwc_rf_probe_lds_add.argtypes = [ctypes.c_int32] * 4 + [P, P, P]
    plib.aiwc_rf_probe_last_error.restype = ctypes.c_char_p
    r, ms = ctypes.c_double(), ctypes.c_double()
    # argument checks fail before any HIP call
    assert plib.aiwc_rf_probe_lds_add(64, 0, 8, 10, None, None, None) == -1
    assert plib.aiwc_rf_probe_lds_add(16, 0, 8, 10, ctypes.byref(r), ctypes.byref(ms), None) == -1
    assert b"width_bits" in plib.aiwc_rf_probe_last_error()
    assert plib.aiwc_rf_probe_lds_add(64, 2, 8, 10, ctypes.byref(r), ctypes.byref(ms), None) == -1
    assert plib.aiwc_rf_probe_lds_add(64, 0, 0, 10, ctypes.byref(r), ctypes.byref(ms), None) == -1
    plib.aiwc_rf_probe_divide.argtypes = [ctypes.c_int64, ctypes.c_uint64, P, P]
    n_bad = ctypes.c_uint64()
    assert plib.aiwc_rf_probe_divide(0, 1, ctypes.byref(n_bad), None) == -1
    assert b"samples" in plib.aiwc_rf_probe_last_error()
    assert plib.aiwc_rf_probe_divide((1 << 40) + 1, 1, ctypes.byref(n_bad), None) == -1
    assert plib.aiwc_rf_probe_divide(100, 1, None, None) == -1
