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


def _host_corner(L, reg, chi2):
    dp = ctypes.POINTER(ctypes.c_double)
    L.sl_lcurve_corner.argtypes = [dp, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), dp]
    import numpy as np
    reg = np.ascontiguousarray(reg, dtype=np.float64)
    chi2 = np.ascontiguousarray(chi2, dtype=np.float64)
    kap = np.zeros(reg.size)
    k = ctypes.c_int32(-7)
    rc = L.sl_lcurve_corner(reg.ctypes.data_as(dp), chi2.ctypes.data_as(dp), reg.size, ctypes.byref(k),
                            kap.ctypes.data_as(dp))
    return rc, int(k.value), kap


def _valid_curves():
    """Valid L-curves: the stored oracle curves of the c2, c3 and c4 goldens and constructed curves."""
    import numpy as np
    gold = os.path.join(ROOT, "tests", "golden")
    curves = []
    g = np.load(os.path.join(gold, "c2_oracle.npz"))
    curves.append((g["reg"], g["chi2"]))
    for name in ("c3_sample.npz", "c4_sample.npz"):
        g = np.load(os.path.join(gold, name))
        curves += list(zip(g["reg"], g["chi2"]))
    full = os.path.join(gold, "c3_full.npz")
    if os.path.exists(full):
        g = np.load(full)
        curves += list(zip(g["reg"], g["chi2"]))
    lam = np.logspace(-3, 2, 12)
    reg = 1.0 / (1.0 + lam) ** 2 + 1e-3
    chi2 = 1.0 + lam / (1.0 + lam)
    curves.append((reg, chi2))
    curves.append((np.insert(reg, 6, reg[5]), np.insert(chi2, 6, chi2[5])))   # a repeated point
    first = np.array([(0, 4), (0.02, 3.2), (0.05, 2.5), (0.1, 2.1), (0.25, 1.95), (0.6, 1.88), (1.0, 1.8),
                      (1.35, 1.65)], dtype=float)
    P = np.vstack([first, [[1.5, 1.5]], first[::-1][:, ::-1]])     # two equal bends
    curves.append((10 ** P[:, 0], 10 ** P[:, 1]))
    return curves


def test_host_lcurve_corner_matches_oracle():
    """sl_lcurve_corner (host, FP64) on valid curves: the oracle's k* exactly, the same dropped
    points, and the curvature at every kept knot within 1e-11 of the curve's largest curvature
    (the two solve the spline systems by different eliminations; small curvatures come from a
    cancelling difference, so the bound is on the absolute error relative to the maximum)."""
    import numpy as np
    from oracle import lcurve
    L = _lib()
    curves = _valid_curves()
    assert len(curves) >= 8
    for reg, chi2 in curves:
        rc, k, kap = _host_corner(L, reg, chi2)
        k_ref, kap_ref = lcurve.corner(reg, chi2)
        assert rc == 0 and k_ref >= 0
        assert k == k_ref, (k, k_ref)
        assert np.array_equal(np.isnan(kap), np.isnan(kap_ref))
        ok = ~np.isnan(kap_ref)
        assert np.max(np.abs(kap[ok] - kap_ref[ok])) <= 1e-11 * np.max(kap_ref[ok])


def test_interp_enum_and_workspace_on_host():
    """The header's interpolation codes match the binding's, the workspace
    grows with bicubic L (16 nodes per subpixel instead of 4: four times the
    transposed-operator storage), and an unknown code is refused on the host."""
    from paper_1101_5803_amd import _lib as B
    src = open(HEADER).read()
    for name in ("SL_INTERP_BILINEAR", "SL_INTERP_NEAREST", "SL_INTERP_BICUBIC"):
        m = re.search(name + r"\s*=\s*(\d+)", src)
        assert m and int(m.group(1)) == getattr(B, name), name
    L = _lib()
    L.sl_last_error.restype = ctypes.c_char_p
    L.sl_solve_workspace_size.argtypes = [ctypes.POINTER(B.Problem)] + [ctypes.c_int] * 3
    L.sl_solve_workspace_size.restype = ctypes.c_size_t

    def size(interp):
        pb = B.Problem()
        pb.img = B.ImageGrid(64, 64, 0.05, 2)
        pb.sigma, pb.k, pb.half_width = 1.0, 7, 1.0
        pb.reg, pb.dtype, pb.psf_general, pb.interp = B.SL_H_CURVATURE, B.SL_F32, 0, interp
        return L.sl_solve_workspace_size(ctypes.byref(pb), 48, 8, 6)

    bil, near, cub = size(B.SL_INTERP_BILINEAR), size(B.SL_INTERP_NEAREST), size(B.SL_INTERP_BICUBIC)
    assert bil > 0 and near == bil
    slot_cap_min = 64 * 64                   # every pixel may map
    assert cub - bil >= 8 * 8 * 24 * 4 * slot_cap_min   # 8 members, 24 more entries of 8 bytes per subpixel
    assert size(3) == 0
    assert b"interp" in L.sl_last_error()


def test_large_and_fft_blur_sizes_on_host():
    """Workspace queries of the Fourier-space blur and of the large solve, and
    their refusals, without a GPU."""
    from paper_1101_5803_amd import _lib as B
    L = _lib()
    L.sl_last_error.restype = ctypes.c_char_p
    L.sl_fft_blur_workspace_size.argtypes = [ctypes.c_int] * 4
    L.sl_fft_blur_workspace_size.restype = ctypes.c_size_t
    L.sl_solve_large_workspace_size.argtypes = [ctypes.POINTER(B.Problem), ctypes.c_int, ctypes.c_int]
    L.sl_solve_large_workspace_size.restype = ctypes.c_size_t
    small = L.sl_fft_blur_workspace_size(B.SL_F32, 640, 640, 65)
    assert small >= 2 * 8 * 513 * 1024            # PSF spectrum and work spectrum, 1024 x 1024 frame
    assert L.sl_fft_blur_workspace_size(B.SL_F64, 640, 640, 65) > small
    assert L.sl_fft_blur_workspace_size(B.SL_F32, 640, 640, 64) == 0 and b"odd" in L.sl_last_error()
    assert L.sl_fft_blur_workspace_size(B.SL_F32, 640, 640, 131) == 0
    assert L.sl_fft_blur_workspace_size(B.SL_F32, 4097, 8, 3) == 0

    def size(ns, n_iter, k=65, interp=B.SL_INTERP_BILINEAR, nx=640):
        pb = B.Problem()
        pb.img = B.ImageGrid(nx, 640, 0.008, 2)
        pb.sigma, pb.k, pb.half_width = 1.0, k, 1.6
        pb.reg, pb.dtype, pb.psf_general, pb.interp = B.SL_H_IDENTITY, B.SL_F32, 1, interp
        return L.sl_solve_large_workspace_size(ctypes.byref(pb), ns, n_iter)

    base = size(512, 40)
    # the L^T table alone: 640^2 pixels x 4 subpixels x 4 taps x (key, weight, pixel, weight)
    assert base > 640 * 640 * 4 * 4 * 16
    assert size(512, 40, interp=B.SL_INTERP_BICUBIC) > base
    assert size(1025, 40) == 0 and b"ns" in L.sl_last_error()
    assert size(512, 65) == 0
    assert size(512, 40, k=131) == 0
    assert size(512, 40, nx=2049) == 0
