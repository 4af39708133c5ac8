"""GPU parity of the blur in Fourier space (sl_fft_blur) and of the large
single-lens solve (sl_solve_large) against the oracle.

Sec. 2.2: the paper convolves with the PSF in Fourier space; the FFT blur
must give the operator of the direct sums (oracle.operators.apply_B /
apply_BT, which are pinned to their definition).  Sec. 4: the large-scale
test runs 40 CGLS iterations on a 640 x 640 image with a 512 x 512 source
grid and a 65 x 65 PSF; the solve is compared iterate by iterate with
oracle.implicit.cgls_iterates (FP64, blur in Fourier space), within the
spread of the oracle under Monte Carlo arithmetic at the GPU's rounding
level (tests/cgls_envelope.py).

FFT blur tolerance: the transform of a frame of side N rounds at about
log2(N) u relative to the largest input, so the bound is 64 u max|x| per
output (FP32: 3.8e-6, FP64: 7e-15), plus 2 K u64 max|x| for the rounding of
the oracle's own sums of K^2 terms.
"""
import os

import numpy as np
import pytest
import torch

import cgls_envelope
import synthgen
from cgls_envelope import FLOOR
from oracle import implicit, lcurve, mock, solve
from oracle import operators as ops

pytestmark = pytest.mark.gpu
DEV = "cuda"
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


@pytest.fixture(scope="module")
def sl():
    import paper_1101_5803_amd as sl
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sl


def _np(out):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("ny,nx,K", [(7, 9, 3), (40, 33, 15), (31, 12, 65), (128, 96, 65), (100, 200, 129),
                                     (1, 1, 1), (2, 257, 5)])
def test_fft_blur_vs_direct_sums(sl, dtype, ny, nx, K):
    print(f"fft blur {ny}x{nx} K={K} {dtype}", flush=True)
    rng = np.random.default_rng(ny * 1000 + nx + K)
    P = synthgen.sinc_moffat_psf(K, fwhm_px=max(1.0, K / 8)) if K > 1 else np.ones((1, 1))
    x = rng.standard_normal((ny, nx))
    u = 2.0 ** -24 if dtype == torch.float32 else 2.0 ** -53
    psf = torch.tensor(P, device=DEV)
    xt = torch.tensor(x, device=DEV, dtype=dtype)
    xr = xt.double().cpu().numpy()            # the values the GPU sees
    for transpose, ref in ((False, ops.apply_B), (True, ops.apply_BT)):
        got = sl.fft_blur(psf, xt, transpose=transpose).double().cpu().numpy()
        want = ref(P, xr)
        err = np.abs(got - want).max()
        # plus the rounding of the oracle's own K^2-term sums (FP64)
        assert err <= (64 * u + 2 * K * 2.0 ** -53) * np.abs(xr).max(), (transpose, err)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_fft_blur_full_frame(sl, dtype):
    """The large-scale shape: 640 x 640 with the 65 x 65 PSF, against the
    oracle's Fourier-space form (pinned to the direct sums)."""
    z = np.load(os.path.join(HERE, "data", "large.npz"))
    P = z["psf"]
    x = z["d"].astype(np.float64)
    u = 2.0 ** -24 if dtype == torch.float32 else 2.0 ** -53
    xt = torch.tensor(x, device=DEV, dtype=dtype)
    for transpose, ref in ((False, ops.apply_B_fft), (True, ops.apply_BT_fft)):
        got = sl.fft_blur(torch.tensor(P, device=DEV), xt, transpose=transpose).double().cpu().numpy()
        err = np.abs(got - ref(P, x)).max()
        assert err <= 64 * u * np.abs(x).max(), (transpose, err)


def _medium():
    """A scaled-down version of the large-scale shape: 96 x 80 image, 48 x 48
    nodes, the 65 x 65 sinc-Moffat PSF (wider than the image is tall)."""
    nx, ny, pix, K = 96, 80, 0.04, 65
    psf = synthgen.sinc_moffat_psf(K, 6.0)
    w = synthgen.Workload("medium", 12, nx, ny, pix, 2, 4, 48, 1.4, K, 6.0, 60.0, "identity", (), 0.0,
                          "sersic", 4, psf_kind="sinc-moffat")
    lens = np.array([1.0, 0.8, 0.4, 0.03, 0.2, 0.01, -0.02])
    clean = mock.clean_image(lens, synthgen.source_blobs(w), nx, ny, pix, 4, psf)
    sigma = clean.max() / 60.0
    d = clean + sigma * synthgen.noise_unit(w)
    return w, lens, d, sigma, psf


def _solver(sl, d, sigma, psf, w, dtype, interp="bilinear"):
    return sl.Solver(torch.tensor(d, device=DEV), sigma, torch.tensor(psf, device=DEV),
                     sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width, reg="identity", dtype=dtype,
                     interp=interp)


@pytest.mark.parametrize("interp", ["bilinear", "bicubic", "nearest"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_large_solve_medium_vs_oracle(sl, prec, interp):
    w, lens, d, sigma, psf = _medium()
    print(f"large solve medium {prec} {interp}", flush=True)
    dtype = torch.float64 if prec == "f64" else torch.float32
    dd = d if prec == "f64" else d.astype(np.float32).astype(np.float64)
    out = _np(_solver(sl, dd, sigma, psf, w, dtype, interp).solve_large(lens, w.ns, 40))

    def make(x):
        return solve.Problem(lens, x, sigma, psf, w.nx, w.ny, w.pix, w.nsub_model, w.ns, w.half_width,
                             "identity", interp, blur="fft")
    # FP32 rounding moves the corner over a wide stretch of this curve (64 draws put it anywhere from the 7th
    # to the 22nd iterate), so the FP32 envelope takes 64 draws
    ref, dev, ds, corners = cgls_envelope.envelope(make, dd, prec, psf.shape[0], 40,
                                                   draws=8 if prec == "f64" else 64)
    assert np.all(out["status"][0] == 0), out["status"]
    assert np.array_equal(out["iters"][0], np.arange(1, 41))
    for key in ("chi2", "reg"):
        err = np.abs(out[key][0] - ref[key])
        bound = 10 * dev[key] + FLOOR[prec] * np.abs(ref[key])
        assert np.all(err <= bound), (key, np.nonzero(err > bound)[0], err / np.abs(ref[key]))
    k = int(out["k_star"][0])
    assert k == lcurve.corner(out["reg"][0], out["chi2"][0])[0]
    if prec == "f64":
        assert k in corners, (k, corners)
    else:
        assert min(corners) <= k <= max(corners), (k, corners)
    s_ref = ref["s"][k]
    err = np.linalg.norm(out["s_corner"] - s_ref)
    assert err <= 10 * ds[k] + FLOOR[prec] * np.linalg.norm(s_ref), (k, err / np.linalg.norm(s_ref))
    assert out["s_off"].tolist() == [0, w.ns * w.ns]


@pytest.mark.parametrize("nx,ny,K", [(70, 130, 1), (100, 60, 15), (24, 20, 9), (96, 80, 81)])
def test_large_solve_psf_sizes_fp32(sl, nx, ny, K):
    """FP32 solves with other PSF widths and ragged image sizes: K = 1, 9 and
    15 take the overlap-save tiles (32 x 64 owned blocks, the image's last
    row and column of tiles cut; the 24 x 20 image is smaller than one owned
    block), K = 81 is wider than a tile's halo and takes the padded frame;
    each against the oracle within its Monte Carlo arithmetic envelope
    (24 draws), 16 iterations."""
    n_iter = 16
    psf = np.ones((1, 1)) if K == 1 else synthgen.sinc_moffat_psf(K, 3.0 if K < 30 else 6.0)
    w = synthgen.Workload("psf-sizes", 13, nx, ny, 0.04, 2, 4, 40, 1.4, K, 3.0, 60.0, "identity", (), 0.0,
                          "sersic", 4, psf_kind="sinc-moffat")
    lens = np.array([1.0, 0.8, 0.4, 0.03, 0.2, 0.01, -0.02])
    clean = mock.clean_image(lens, synthgen.source_blobs(w), nx, ny, w.pix, 4, psf)
    sigma = clean.max() / 60.0
    d = (clean + sigma * synthgen.noise_unit(w)).astype(np.float32).astype(np.float64)
    print(f"large solve fp32 {nx}x{ny} K={K}", flush=True)
    out = _np(_solver(sl, d, sigma, psf, w, torch.float32).solve_large(lens, w.ns, n_iter))

    def make(x):
        return solve.Problem(lens, x, sigma, psf, nx, ny, w.pix, w.nsub_model, w.ns, w.half_width,
                             "identity", "bilinear", blur="fft")
    ref, dev, ds, corners = cgls_envelope.envelope(make, d, "f32", K, n_iter, draws=24)
    assert np.all(out["status"][0] == 0), out["status"]
    for key in ("chi2", "reg"):
        err = np.abs(out[key][0] - ref[key])
        bound = 10 * dev[key] + FLOOR["f32"] * np.abs(ref[key])
        assert np.all(err <= bound), (key, np.nonzero(err > bound)[0], err / np.abs(ref[key]))
    k = int(out["k_star"][0])
    assert k == lcurve.corner(out["reg"][0], out["chi2"][0])[0]
    assert min(corners) <= k <= max(corners), (k, corners)
    s_ref = ref["s"][k]
    err = np.linalg.norm(out["s_corner"] - s_ref)
    assert err <= 10 * ds[k] + FLOOR["f32"] * np.linalg.norm(s_ref), (k, err / np.linalg.norm(s_ref))


def test_large_solve_full_shape_fp32(sl):
    """The large-scale shape (synthgen.LARGE) in FP32, the configuration bench.py
    times, against the oracle (computed here) within the stored FP32 envelope
    (tests/golden/large_envelope.npz); a second call gives the same bits."""
    w = synthgen.LARGE
    z = np.load(os.path.join(HERE, "data", "large.npz"))
    d = z["d"].astype(np.float64)
    g = np.load(os.path.join(GOLD, "large_envelope.npz"))
    print("large solve full shape fp32", flush=True)
    solver = _solver(sl, d, float(z["sigma"]), z["psf"], w, torch.float32)
    out = _np(solver.solve_large(z["lens"], w.ns, synthgen.LARGE_ITERS))
    again = _np(solver.solve_large(z["lens"], w.ns, synthgen.LARGE_ITERS))
    for key in out:
        if key != "dof":
            assert np.array_equal(out[key], again[key]), key
    pb = solve.Problem(z["lens"], d, float(z["sigma"]), z["psf"], w.nx, w.ny, w.pix, w.nsub_model, w.ns,
                       w.half_width, w.reg, blur="fft")
    ref = implicit.cgls_iterates(pb, synthgen.LARGE_ITERS)
    # the stored envelope is of this oracle run, up to the FP64 rounding of this host (far inside the
    # FP32 envelope: CGLS amplifies rounding in its late iterates on any machine)
    assert np.all(np.abs(ref["chi2"] - g["chi2"]) <= 0.1 * g["dev_chi2"] + 1e-12 * g["chi2"])
    assert np.all(out["status"][0] == 0)
    for key, dev in (("chi2", g["dev_chi2"]), ("reg", g["dev_reg"])):
        err = np.abs(out[key][0] - ref[key])
        bound = 10 * dev + FLOOR["f32"] * np.abs(ref[key])
        assert np.all(err <= bound), (key, np.nonzero(err > bound)[0], err / np.abs(ref[key]))
    k = int(out["k_star"][0])
    corners = set(g["corners"].tolist())
    assert min(corners) <= k <= max(corners), (k, corners)
    s_ref = ref["s"][k]
    err = np.linalg.norm(out["s_corner"] - s_ref)
    assert err <= 10 * g["ds"][k] + FLOOR["f32"] * np.linalg.norm(s_ref), (k, err / np.linalg.norm(s_ref))


@pytest.mark.parametrize("interp", ["bilinear", "bicubic"])
def test_large_solve_fp64_repeatable(sl, interp):
    """The FP64 solve (frame form, fixed-order reductions and sorted L^T rows)
    gives the same bits on a second call with the same inputs."""
    w, lens, d, sigma, psf = _medium()
    print(f"large solve fp64 repeat {interp}", flush=True)
    s = _solver(sl, d, sigma, psf, w, torch.float64, interp)
    first = _np(s.solve_large(lens, w.ns, 40))
    again = _np(s.solve_large(lens, w.ns, 40))
    for key in first:
        if key != "dof":
            assert np.array_equal(first[key], again[key]), key


def test_large_solve_edge_cases(sl):
    """A genome outside the prior's domain is flagged, a lens that maps nothing
    gives empty iterates, fewer than four iterations skip the L-curve, and
    bad sizes are refused on the host."""
    w, lens, d, sigma, psf = _medium()
    s = _solver(sl, d, sigma, psf, w, torch.float32)
    out = _np(s.solve_large([1.0, 1.5, 0, 0, 0, 0, 0], w.ns, 8))          # q > 1
    assert np.all(out["status"][0] == 4) and out["corner_status"][0] == 4
    out = _np(s.solve_large([5.0, 1.0, 0, 0, 0, 5.0, 5.0], w.ns, 8))      # maps nothing
    assert np.all(out["status"][0] == 2) and out["corner_status"][0] == 2
    assert np.allclose(out["s_corner"], 0.0)
    np.testing.assert_allclose(out["chi2"][0], (d.astype(np.float32).astype(np.float64) ** 2).sum() / sigma ** 2,
                               rtol=1e-6)
    out = _np(s.solve_large(lens, w.ns, 3))
    assert np.all(out["status"][0] == 0) and out["corner_status"][0] == 5 and out["k_star"][0] == 0
    out = _np(s.solve_large(lens, w.ns, 1))
    assert out["corner_status"][0] == 0 and out["k_star"][0] == 0
    with pytest.raises(sl._lib.SemilinError):
        s.solve_large(lens, 1025, 8)
    with pytest.raises(sl._lib.SemilinError):
        s.solve_large(lens, w.ns, 65)
    with pytest.raises(sl._lib.SemilinError):
        sl.fft_blur(torch.ones((131, 131), device=DEV, dtype=torch.float64), torch.ones((8, 8), device=DEV))


def test_large_solve_graph_replay(sl):
    """sl_solve_large captured in a HIP graph (stream capture through torch) and
    replayed three times, with an eager solve of another lens and a
    synchronisation between replays: every replay gives the eager result's bits."""
    w, lens, d, sigma, psf = _medium()
    s = _solver(sl, d, sigma, psf, w, torch.float32)
    lens = torch.tensor(lens, device=DEV)            # no host-to-device copy inside the capture
    ref = _np(s.solve_large(lens, w.ns, 40))
    out = s.alloc_result(w.ns * w.ns, 1, 40)
    s.solve_large(lens, w.ns, 40, out=out)          # workspace allocated before the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.solve_large(lens, w.ns, 40, out=out)
    other = [1.05, 0.7, 0.2, 0.02, 0.5, 0.0, 0.01]
    for _ in range(3):
        for v in out.values():
            v.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = _np(out)
        for key in ref:
            if key != "dof":
                assert np.array_equal(got[key], ref[key]), key
        s.solve_large(other, w.ns, 40)               # eager work on the same workspace in between
        torch.cuda.synchronize()
