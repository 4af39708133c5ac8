"""The C-ABI library loads without a GPU and exports every entry point its header declares.

Also checks the host-side argument validation paths that return before any
HIP call (no device work is issued here).
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semilin.h")
LIB = os.path.join(ROOT, "paper_1101_5803_amd", "libsemilin.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(sl_[A-Za-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("libsemilin.so not built (run python -m paper_1101_5803_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("sl_lens_trace", "sl_apply_L", "sl_apply_LT", "sl_apply_B", "sl_apply_BT", "sl_apply_HtH",
              "sl_solve_workspace_size", "sl_solve_semilinear", "sl_lcurve_corner", "sl_mlp_forward",
              "sl_mlp_train_step", "sl_mlp_workspace_size", "sl_last_error", "sl_version"):
        assert n in names, n


def test_library_exports_every_declared_symbol():
    _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_host_validation_without_gpu():
    L = _lib()
    L.sl_last_error.restype = ctypes.c_char_p
    L.sl_mlp_workspace_size.restype = ctypes.c_size_t
    L.sl_mlp_workspace_size.argtypes = [ctypes.c_int]
    assert L.sl_mlp_workspace_size(1024) > 5 * 1024 * 256 * 4
    assert L.sl_mlp_workspace_size(-1) == 0
    assert b"batch" in L.sl_last_error()
    L.sl_mlp_forward.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int] + [ctypes.c_void_p] * 3
    assert L.sl_mlp_forward(None, None, 0, None, None, None) == -1
    # the host L-curve corner needs >= 4 points
    dp = ctypes.POINTER(ctypes.c_double)
    L.sl_lcurve_corner.argtypes = [dp, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), dp]
    a = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
    k = ctypes.c_int32(0)
    assert L.sl_lcurve_corner(a, a, 3, ctypes.byref(k), None) == -1
    L.sl_version.restype = ctypes.c_char_p
    assert L.sl_version()
