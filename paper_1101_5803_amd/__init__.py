"""MI355X-native matrix-free semilinear lens solver (Rogers & Fiege 2011 hot path).

The compute lives in libsemilin.so (hand-written gfx950 HIP behind a C ABI,
declared in include/semilin.h); this package is its thin Python binding.
"""
from . import _lib  # noqa: F401
from .ops import (Grid, Solver, apply_B, apply_BT, apply_HtH, apply_L, apply_LT,  # noqa: F401
                  apply_LT_ordered, fft_blur, lcurve_corner,
                  lens_trace, mlp_forward, mlp_forward_noalloc, mlp_pack, mlp_train_step, mlp_unpack, profile_enable,
                  profile_solve_ms)

__all__ = ["Grid", "Solver", "apply_B", "apply_BT", "apply_HtH", "apply_L", "apply_LT", "apply_LT_ordered", "fft_blur",
           "lcurve_corner",
           "lens_trace", "mlp_forward", "mlp_forward_noalloc", "mlp_pack", "mlp_train_step", "mlp_unpack", "profile_enable",
           "profile_solve_ms"]
