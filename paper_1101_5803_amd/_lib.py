"""ctypes binding of libsemilin.so (argument marshalling only).

Every computation happens inside the HIP library; this module turns torch
device tensors into raw pointers, passes torch's current HIP stream, and
turns non-zero return codes into exceptions.  Import fails loudly when the
built library is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsemilin.so")

SL_OK, SL_EINVAL, SL_EHIP, SL_ENOIMPL = 0, -1, -2, -3
SL_F32, SL_F64 = 0, 1
SL_H_IDENTITY, SL_H_CURVATURE = 0, 1
ST_OK, ST_MAXIT, ST_EMPTY, ST_BREAKDOWN, ST_INVALID, ST_LCURVE = range(6)
MAX_LAMBDA = 64
MLP_NPARAM = 7 * 256 + 256 + 256 * 256 + 256 + 256 + 1
MLP_MAX_BATCH = 1 << 20


class SemilinError(RuntimeError):
    pass


class ImageGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("pix", ctypes.c_double),
                ("nsub", ctypes.c_int)]


class Problem(ctypes.Structure):
    _fields_ = [("img", ImageGrid), ("d", ctypes.c_void_p), ("sigma", ctypes.c_double),
                ("psf", ctypes.c_void_p), ("k", ctypes.c_int), ("half_width", ctypes.c_double),
                ("reg", ctypes.c_int), ("dtype", ctypes.c_int), ("psf_general", ctypes.c_int),
                ("interp", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("wide_window", ctypes.c_int), ("lt_csr", ctypes.c_int), ("blur_direct", ctypes.c_int),
                ("plain_cg", ctypes.c_int), ("pc_theta_pct", ctypes.c_int), ("heavy", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("tuning", ctypes.POINTER(Tuning)),
                ("mc_noise", ctypes.c_void_p)]


N_VARIANTS = 16
SL_INTERP_BILINEAR, SL_INTERP_NEAREST, SL_INTERP_BICUBIC = 0, 1, 2


class Result(ctypes.Structure):
    _fields_ = [("s_corner", ctypes.c_void_p), ("s_off", ctypes.c_void_p), ("chi2", ctypes.c_void_p),
                ("reg", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("k_star", ctypes.c_void_p), ("corner_status", ctypes.c_void_p), ("dof", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SemilinError(f"HIP library not built: {LIB_PATH} missing "
                               "(run python -m paper_1101_5803_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, ip, dp, i32p = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int32)
        L.sl_last_error.restype = ctypes.c_char_p
        L.sl_version.restype = ctypes.c_char_p
        L.sl_lens_trace.argtypes = [vp, ip, ctypes.POINTER(ImageGrid), i32p, dp, vp, vp]
        for name in ("sl_apply_L", "sl_apply_LT"):
            getattr(L, name).argtypes = [ip, vp, ip, ctypes.POINTER(ImageGrid), i32p, vp, vp, vp]
        L.sl_apply_LT_ordered_workspace_size.argtypes = [ctypes.POINTER(ImageGrid), i32p, ip]
        L.sl_apply_LT_ordered_workspace_size.restype = ctypes.c_size_t
        L.sl_apply_LT_ordered.argtypes = [ip, vp, ip, ctypes.POINTER(ImageGrid), i32p, vp, vp, vp, ctypes.c_size_t,
                                          vp]
        for name in ("sl_apply_B", "sl_apply_BT"):
            getattr(L, name).argtypes = [ip, ip, ip, ip, vp, ip, vp, vp, vp]
        L.sl_apply_HtH.argtypes = [ip, ip, ip, i32p, vp, vp, vp]
        L.sl_solve_workspace_size.argtypes = [ctypes.POINTER(Problem), ip, ip, ip]
        L.sl_solve_workspace_size.restype = ctypes.c_size_t
        L.sl_solve_semilinear.argtypes = [ctypes.POINTER(Problem), vp, vp, ip, ip,
                                          ctypes.POINTER(ctypes.c_double), ip, ctypes.POINTER(SolveOpts),
                                          vp, ctypes.c_size_t, ctypes.POINTER(Result), vp]
        L.sl_solve_implicit.argtypes = [ctypes.POINTER(Problem), vp, vp, ip, ip, ip, ctypes.POINTER(SolveOpts), vp,
                                        ctypes.c_size_t, ctypes.POINTER(Result), vp]
        L.sl_solve_autotune.argtypes = [ctypes.POINTER(Problem), vp, vp, ip, ip, ctypes.POINTER(ctypes.c_double), ip,
                                        ctypes.POINTER(SolveOpts), vp, ctypes.c_size_t, ctypes.POINTER(Result), vp,
                                        ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double)]
        L.sl_plan_create.argtypes = [ctypes.POINTER(Problem), vp, vp, ip, ip, ctypes.POINTER(ctypes.c_double), ip,
                                     ctypes.POINTER(SolveOpts), vp, ctypes.c_size_t, ctypes.POINTER(Result),
                                     ctypes.POINTER(vp)]
        L.sl_plan_launch.argtypes = [vp, vp]
        L.sl_chi2_sources_workspace_size.argtypes = [ctypes.POINTER(Problem), ip]
        L.sl_chi2_sources_workspace_size.restype = ctypes.c_size_t
        L.sl_chi2_sources.argtypes = [ctypes.POINTER(Problem), vp, ip, vp, ip, vp, ctypes.c_size_t, vp, vp]
        L.sl_plan_destroy.argtypes = [vp]
        L.sl_fft_blur_workspace_size.argtypes = [ip, ip, ip, ip]
        L.sl_fft_blur_workspace_size.restype = ctypes.c_size_t
        L.sl_fft_blur.argtypes = [ip, ip, ip, ip, vp, ip, vp, vp, vp, ctypes.c_size_t, vp]
        L.sl_solve_large_workspace_size.argtypes = [ctypes.POINTER(Problem), ip, ip]
        L.sl_solve_large_workspace_size.restype = ctypes.c_size_t
        L.sl_solve_large.argtypes = [ctypes.POINTER(Problem), vp, ip, ip, vp, ctypes.c_size_t,
                                     ctypes.POINTER(Result), vp]
        L.sl_solve_member_info.argtypes = [ctypes.POINTER(Problem), ip, ip, ip, vp, vp]
        L.sl_profile_enable.argtypes = [ip]
        L.sl_profile_solve_ms.argtypes = [ctypes.POINTER(ctypes.c_double), i32p]
        L.sl_lcurve_corner.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ip, i32p, ctypes.POINTER(ctypes.c_double)]
        L.sl_mlp_workspace_size.argtypes = [ip]
        L.sl_mlp_workspace_size.restype = ctypes.c_size_t
        L.sl_mlp_forward.argtypes = [vp, vp, ip, vp, vp, vp]
        L.sl_mlp_forward_noalloc.argtypes = [vp, vp, ip, vp, vp]
        L.sl_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, ip, ctypes.c_float, ip, vp, vp, vp, vp]
        for name in ("sl_lens_trace", "sl_apply_L", "sl_apply_LT", "sl_apply_LT_ordered", "sl_apply_B", "sl_apply_BT",
                     "sl_apply_HtH", "sl_solve_semilinear", "sl_solve_implicit", "sl_lcurve_corner", "sl_mlp_forward", "sl_mlp_forward_noalloc",
                     "sl_mlp_train_step", "sl_solve_member_info", "sl_profile_enable", "sl_profile_solve_ms",
                     "sl_solve_autotune", "sl_plan_create", "sl_plan_launch", "sl_plan_destroy", "sl_fft_blur",
                     "sl_solve_large", "sl_chi2_sources"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc: int, what: str) -> int:
    if rc < 0:
        msg = lib().sl_last_error().decode(errors="replace")
        raise SemilinError(f"{what} failed ({rc}): {msg}")
    return rc


def ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_contiguous():
        raise SemilinError("tensors passed to the library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def i32_array(values):
    arr = (ctypes.c_int32 * len(values))(*[int(v) for v in values])
    return arr


def f64_array(values):
    return (ctypes.c_double * len(values))(*[float(v) for v in values])


def version() -> str:
    return lib().sl_version().decode()
