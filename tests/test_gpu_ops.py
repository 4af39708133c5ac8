"""GPU parity of the operator-level C-ABI calls against the FP64 oracle.

Tolerances: FP64 kernels agree with the oracle to rounding (relative 1e-11
on sums of O(K^2) products); FP32 kernels to a relative 2e-6 of the output's
scale (a few FP32 ulps accumulated over <= K^2 = 441 terms).  Inside/outside
decisions of the trace are compared exactly, except for rays within 1e-9 of
the grid border, where FP64 rounding may legitimately differ.
"""
import numpy as np
import pytest
import torch

import synthgen
from oracle import lens as olens
from oracle import mock
from oracle import operators as oops

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def semilin():
    import paper_1101_5803_amd as sl
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sl


def _genomes(n, seed):
    return synthgen.population(seed, n)


@pytest.mark.parametrize("nsub", [1, 2, 3])
def test_lens_trace(semilin, nsub):
    grid = semilin.Grid(37, 29, 0.07, nsub)
    G = _genomes(4, 11)
    G[1, 1] = 1.0          # SIS member (q = 1, k = 0)
    ns = [9, 16, 31, 64]
    R = 1.0
    uv = semilin.lens_trace(torch.tensor(G, device=DEV), grid, ns, R).cpu().numpy()
    for m in range(4):
        bx, by = olens.trace_image(G[m], grid.nx, grid.ny, grid.pix, nsub)
        h = 2 * R / (ns[m] - 1)
        u = (bx + R) / h
        v = (by + R) / h
        inside = (u >= 0) & (u <= ns[m] - 1) & (v >= 0) & (v <= ns[m] - 1)
        gu = uv[m, :, 0].reshape(u.shape)
        gv = uv[m, :, 1].reshape(v.shape)
        g_in = ~np.isnan(gu)
        near = (np.minimum(np.abs(u), np.abs(u - ns[m] + 1)) < 1e-9) | \
               (np.minimum(np.abs(v), np.abs(v - ns[m] + 1)) < 1e-9)
        assert np.all((g_in == inside) | near)
        both = g_in & inside
        np.testing.assert_allclose(gu[both], u[both], rtol=0, atol=1e-11)
        np.testing.assert_allclose(gv[both], v[both], rtol=0, atol=1e-11)


def test_lens_trace_invalid_genome(semilin):
    grid = semilin.Grid(8, 8, 0.1, 2)
    G = _genomes(2, 1)
    G[0, 1] = 1.5      # q outside (0, 1]
    G[1, 0] = np.nan
    uv = semilin.lens_trace(torch.tensor(G, device=DEV), grid, [10, 10], 1.0).cpu().numpy()
    assert np.isnan(uv).all()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 2e-6)])
def test_apply_L_LT(semilin, dtype, tol):
    grid = semilin.Grid(33, 27, 0.09, 2)
    G = _genomes(3, 5)
    ns = [7, 20, 45]
    R = 1.2
    uv = semilin.lens_trace(torch.tensor(G, device=DEV), grid, ns, R)
    rng = np.random.default_rng(0)
    s = rng.standard_normal(sum(n * n for n in ns))
    img = rng.standard_normal((3, grid.J))
    Ls = semilin.apply_L(uv, grid, ns, torch.tensor(s, dtype=dtype, device=DEV)).cpu().double().numpy()
    LTi = semilin.apply_LT(uv, grid, ns, torch.tensor(img, dtype=dtype, device=DEV)).cpu().double().numpy()
    off = 0
    for m in range(3):
        bx, by = olens.trace_image(G[m], grid.nx, grid.ny, grid.pix, grid.nsub)
        tab = oops.bilinear_table(bx, by, ns[m], R)
        I = ns[m] ** 2
        ref_L = oops.apply_L(tab, s[off:off + I], grid.nsub)
        ref_LT = oops.apply_LT(tab, img[m], I, grid.nsub)
        scale = max(np.abs(ref_L).max(), 1e-30)
        assert np.abs(Ls[m] - ref_L).max() <= tol * scale * 4
        scale = max(np.abs(ref_LT).max(), 1e-30)
        assert np.abs(LTi[off:off + I] - ref_LT).max() <= tol * scale * 8
        off += I
    # adjoint on the GPU path itself
    if dtype == torch.float64:
        lhs = float((Ls * img).sum())
        rhs = float((s * LTi).sum())
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("K,fwhm", [(5, 1.5), (15, 3.0), (21, 4.0), (9, 0.0)])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_apply_B_BT(semilin, K, fwhm, dtype, tol):
    rng = np.random.default_rng(K)
    if fwhm > 0:
        P = mock.gaussian_psf(K, fwhm)
    else:                                  # an asymmetric, non-separable PSF
        P = rng.uniform(0, 1, (K, K))
        P /= P.sum()
    x = rng.standard_normal((3, 45, 38))
    psf_d = torch.tensor(P, device=DEV)
    xd = torch.tensor(x, dtype=dtype, device=DEV)
    Bx = semilin.apply_B(psf_d, xd).cpu().double().numpy()
    BTx = semilin.apply_BT(psf_d, xd).cpu().double().numpy()
    for i in range(3):
        rb = oops.apply_B(P, x[i])
        rbt = oops.apply_BT(P, x[i])
        assert np.abs(Bx[i] - rb).max() <= tol * np.abs(rb).max() * 4
        assert np.abs(BTx[i] - rbt).max() <= tol * np.abs(rbt).max() * 4


@pytest.mark.parametrize("reg", ["identity", "curvature"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 1e-6)])
def test_apply_HtH(semilin, reg, dtype, tol):
    ns = [2, 3, 17, 40]
    rng = np.random.default_rng(3)
    s = rng.standard_normal(sum(n * n for n in ns))
    out = semilin.apply_HtH(reg, ns, torch.tensor(s, dtype=dtype, device=DEV)).cpu().double().numpy()
    off = 0
    for n in ns:
        ref = oops.apply_HtH(s[off:off + n * n], n, reg)
        assert np.abs(out[off:off + n * n] - ref).max() <= tol * max(np.abs(ref).max(), 1.0) * 16
        off += n * n


def test_errors_are_reported(semilin):
    grid = semilin.Grid(8, 8, 0.1, 2)
    with pytest.raises(semilin._lib.SemilinError, match="ns"):
        semilin.lens_trace(torch.zeros((1, 7), dtype=torch.float64, device=DEV), grid, [1], 1.0)
    with pytest.raises(semilin._lib.SemilinError, match="odd"):
        semilin.apply_B(torch.zeros((4, 4), dtype=torch.float64, device=DEV),
                        torch.zeros((8, 8), device=DEV))
