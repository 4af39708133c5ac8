"""ctypes wrapper and build step of the plain-C FP64 oracle (``csolve.c``).

Test infrastructure only (tests, smoke check, CPU-baseline timing).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csolve.c")
_LIB = os.path.join(_HERE, "libcsolve.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile csolve.c with gcc (-O2, OpenMP) into oracle/libcsolve.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_eval.argtypes = [ctypes.c_int, dp, ip, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_int, dp, ctypes.c_double, dp, ctypes.c_int,
                                    ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    dp, dp, ip, ip, dp, ctypes.c_int, ctypes.c_int]
        lib.oracle_eval.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def evaluate(lens, ns, half_width, nx, ny, pix, nsub, d, sigma, psf, reg, lambdas,
             tol=1e-10, maxit=0, want_s=False, threads=0):
    """Per-member, per-lambda chi2 / reg / iterations / status (and solutions).

    ``lens`` (M, 7) genomes, ``ns`` (M,) source-grid sides.
    """
    lib = _load()
    lens = np.ascontiguousarray(np.atleast_2d(lens), dtype=np.float64)
    M = lens.shape[0]
    ns = np.ascontiguousarray(np.broadcast_to(np.asarray(ns, dtype=np.int32), (M,)))
    d = np.ascontiguousarray(d, dtype=np.float64)
    psf = np.ascontiguousarray(psf, dtype=np.float64)
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    nl = lam.size
    chi2 = np.zeros((M, nl))
    regv = np.zeros((M, nl))
    iters = np.zeros((M, nl), dtype=np.int32)
    status = np.zeros((M, nl), dtype=np.int32)
    stride = int(ns.max()) ** 2
    s = np.zeros((M, nl, stride)) if want_s else None
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    kind = 0 if reg == "identity" else 1
    lib.oracle_eval(M, lens.ctypes.data_as(dp), ns.ctypes.data_as(ip), half_width, nx, ny, pix, nsub,
                    d.ctypes.data_as(dp), sigma, psf.ctypes.data_as(dp), psf.shape[0], kind,
                    lam.ctypes.data_as(dp), nl, tol, maxit, chi2.ctypes.data_as(dp),
                    regv.ctypes.data_as(dp), iters.ctypes.data_as(ip), status.ctypes.data_as(ip),
                    s.ctypes.data_as(dp) if want_s else None, stride, threads)
    return dict(chi2=chi2, reg=regv, iters=iters, status=status, s=s)
