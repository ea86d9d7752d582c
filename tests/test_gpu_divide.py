"""The grow kernel's split-score division against IEEE division (GPU).

The kernel divides with the IEEE sequence minus its operand scaling and
special-value fixup, which leave the score's operands unchanged: numerators
that are zero or squares below 2^82, denominators that are weights in
[1, 2^18].  On 2^31 quotients of that domain the two must agree bit for bit.
"""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE_LIB = os.path.join(ROOT, "paper_1811_00156_amd", "libaiwc_rf_probe.so")


def test_split_score_division_is_ieee():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    plib = ctypes.CDLL(PROBE_LIB)
    plib.aiwc_rf_probe_divide.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    plib.aiwc_rf_probe_last_error.restype = ctypes.c_char_p
    for seed in (181100163, 7):
        n_bad = ctypes.c_uint64(1)
        rc = plib.aiwc_rf_probe_divide(1 << 30, seed, ctypes.byref(n_bad), None)
        assert rc == 0, plib.aiwc_rf_probe_last_error()
        assert n_bad.value == 0, f"{n_bad.value} quotients differ from IEEE division (seed {seed})"
