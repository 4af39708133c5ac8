"""Gaussian PSF, analytic sources and noisy mock images (FP64 oracle).

Paper: mock data are built by evaluating an analytic source at the
back-traced positions of a fine subpixel grid (10 x 10 per pixel),
averaging (conservation of surface brightness, Eq. 2), convolving with a
Gaussian PSF given by its FWHM in pixels on a K x K grid, and adding
Gaussian noise whose standard deviation is the peak image intensity divided
by the quoted S/N (Sec. 2.3).

Readings: the PSF is sampled at pixel centres about (K-1)/2 and normalised
to unit sum; sigma_psf = FWHM / (2 sqrt(2 ln 2)).  The paper's spiral source
lacks its parameters, so elliptical Gaussians and Sersic profiles stand in
(with b_n from the Ciotti & Bertin 1999 asymptotic series).
"""
from __future__ import annotations

import math

import numpy as np

from . import lens as _lens
from . import operators as _ops


def gaussian_psf(K: int, fwhm_px: float) -> np.ndarray:
    ck = (K - 1) / 2.0
    sig = fwhm_px / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    a = np.arange(K) - ck
    P = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sig * sig))
    return P / P.sum()


def sersic_bn(n: float) -> float:
    """Ciotti & Bertin (1999) asymptotic expansion of b_n."""
    return (2.0 * n - 1.0 / 3.0 + 4.0 / (405.0 * n) + 46.0 / (25515.0 * n * n)
            + 131.0 / (1148175.0 * n ** 3) - 2194697.0 / (30690717750.0 * n ** 4))


def source_brightness(bx, by, blobs) -> np.ndarray:
    """Sum of analytic blobs at source-plane positions (bx, by)."""
    bx = np.asarray(bx, dtype=np.float64)
    by = np.asarray(by, dtype=np.float64)
    out = np.zeros_like(bx)
    for b in blobs:
        dx = bx - b["xc"]
        dy = by - b["yc"]
        c, s = math.cos(b["pa"]), math.sin(b["pa"])
        xm = c * dx + s * dy
        ym = -s * dx + c * dy
        rr = xm * xm + (ym / b["q"]) ** 2
        if b["kind"] == "gauss":
            out += b["amp"] * np.exp(-rr / (2.0 * b["size"] ** 2))
        else:
            bn = sersic_bn(b["n"])
            out += b["amp"] * np.exp(-bn * ((np.sqrt(rr) / b["size"]) ** (1.0 / b["n"]) - 1.0))
    return out


def clean_image(lens, blobs, nx, ny, pix, nsub_data, psf):
    """Lensed (subpixel-averaged) then blurred noise-free image, (ny, nx)."""
    bx, by = _lens.trace_image(lens, nx, ny, pix, nsub_data)
    unblurred = source_brightness(bx, by, blobs).mean(axis=1).reshape(ny, nx)
    return _ops.apply_B(psf, unblurred)


def mock_data(w, lens, blobs, noise_unit):
    """Noisy mock image for workload ``w``; returns (d, sigma, clean, psf)."""
    if getattr(w, "psf_kind", "gauss") == "sinc-moffat":
        import synthgen
        psf = synthgen.sinc_moffat_psf(w.k_psf, w.fwhm_px)
    else:
        psf = gaussian_psf(w.k_psf, w.fwhm_px)
    clean = clean_image(lens, blobs, w.nx, w.ny, w.pix, w.nsub_data, psf)
    sigma = clean.max() / w.snr
    d = clean + sigma * noise_unit
    return d, sigma, clean, psf


def workload_data(w):
    """Mock image of a named workload from its seeded draws.

    Returns dict(d, sigma, psf, lens) with d of shape (ny, nx).
    """
    import synthgen
    lens = synthgen.lens_truth(w)
    blobs = synthgen.source_blobs(w)
    d, sigma, _clean, psf = mock_data(w, lens, blobs, synthgen.noise_unit(w))
    return dict(d=d, sigma=float(sigma), psf=psf, lens=lens)
