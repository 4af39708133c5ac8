"""Seeded synthetic-input recipes shared by the oracle, the tests and the benchmark.

This module holds *inputs only*: workload shapes, parameter boxes and the
random draws that feed them.  It contains none of the lens-solve arithmetic
(no ray tracing, interpolation, blurring or solving); the forward model that
turns these draws into a mock image lives in the oracle.

Workloads (names follow the paper's notation: J image pixels, n x n subpixels
per pixel, I = n_s^2 source nodes, K x K PSF, lambda grid of size N_lambda):

* ``c1`` -- plain single solve: 32x32 image of 0.05", SIS with theta_E = 0.8"
  at the centre, 16x16 nodes spanning +-0.5", two elliptical Gaussians, 5x5
  Gaussian PSF of FWHM 1.5 px, noise sigma = peak/30, H = I, one lambda=1e-2,
  FP64, CG to relative residual 1e-10.
* ``c2`` -- single SIE + external shear lens on a 128x128 image, 64x64
  nodes spanning +-1", three Sersic blobs, 15x15 PSF of FWHM 3 px,
  noise sigma = peak/50, curvature H, 16 lambdas log-spaced over 1e-4..1e2.
* ``c3`` -- 256 SIE+shear parameter sets drawn uniformly in the prior box,
  scored against the c2 image, per-member source grids n_s in [32, 96].
* ``c4`` -- GA at scale: 200x200 image, 100x100 nodes, 21x21 PSF of FWHM
  4 px, noise sigma = peak/100, 24 lambdas, population 1024.
* ``c5`` -- surrogate training / screening workload on the c2 image with a
  fixed 64x64 grid.
* ``large`` -- the shape of the paper's large-scale test: 640x640 image of
  0.008", 512x512 nodes spanning +-1.6", 65x65 sinc-Moffat PSF of FWHM 6 px,
  twelve Sersic blobs (mock subpixels 4x4), noise sigma = peak/100, H = I,
  40 CGLS iterations (implicit regularisation).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Prior box for the 7-gene genome (theta_E, q, pa, gamma, gamma_pa, x0, y0);
# angles in radians, lengths in arcsec.
PRIOR_LO = np.array([0.7, 0.4, 0.0, 0.0, 0.0, -0.1, -0.1])
PRIOR_HI = np.array([1.3, 1.0, math.pi, 0.15, math.pi, 0.1, 0.1])
GENE_NAMES = ("theta_e", "q", "pa", "gamma", "gamma_pa", "x0", "y0")


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    nx: int            # image columns
    ny: int            # image rows
    pix: float         # arcsec per pixel
    nsub_model: int    # n (subpixels per side) used when modelling
    nsub_data: int     # subpixels per side used to synthesise the mock image
    ns: int            # source nodes per side (fixed-grid workloads)
    half_width: float  # source grid spans +-half_width (node extent)
    k_psf: int         # PSF side K
    fwhm_px: float     # PSF FWHM in pixels
    snr: float         # peak / noise sigma
    reg: str           # "identity" or "curvature"
    lambdas: tuple     # ascending lambda grid
    tol: float         # CG relative-residual tolerance
    source_kind: str   # "gauss" or "sersic"
    n_blobs: int
    psf_kind: str = "gauss"   # "gauss" or "sinc-moffat" (sinc_moffat_psf at fwhm_px)


def log_grid(lo: float, hi: float, n: int) -> tuple:
    """lambda_k = 10^(log10 lo + k*delta), endpoints inclusive, ascending."""
    if n == 1:
        return (float(lo),)
    a, b = math.log10(lo), math.log10(hi)
    return tuple(float(10.0 ** (a + k * (b - a) / (n - 1))) for k in range(n))


C1 = Workload("c1", 1, 32, 32, 0.05, 2, 10, 16, 0.5, 5, 1.5, 30.0, "identity",
              (1e-2,), 1e-10, "gauss", 2)
C2 = Workload("c2", 2, 128, 128, 0.05, 2, 10, 64, 1.0, 15, 3.0, 50.0, "curvature",
              log_grid(1e-4, 1e2, 16), 1e-7, "sersic", 3)
C3 = dataclasses.replace(C2, name="c3", seed=3)
C4 = Workload("c4", 4, 200, 200, 0.05, 2, 10, 100, 1.0, 21, 4.0, 100.0, "curvature",
              log_grid(1e-4, 1e2, 24), 1e-7, "sersic", 3)
C5 = dataclasses.replace(C2, name="c5", seed=5)
# The shape of the paper's large-scale test (Sec. 4, the M51 figure): a 640 x 640
# image, a 512 x 512 source grid, a 65 x 65 PSF with low-level structure, 40
# CGLS iterations of the implicit regularisation.  The galaxy image is not
# available; twelve Sersic blobs stand in for it.
LARGE = Workload("large", 6, 640, 640, 0.008, 2, 4, 512, 1.6, 65, 6.0, 100.0, "identity", (), 0.0,
                 "sersic", 12, psf_kind="sinc-moffat")
LARGE_ITERS = 40
WORKLOADS = {w.name: w for w in (C1, C2, C3, C4, C5, LARGE)}

# c2's lens: theta_E 1.0", q 0.7, PA 30 deg, gamma 0.05 at 60 deg; the centre
# offset (<= 0.05") is drawn from the seed.
C2_LENS_FIXED = (1.0, 0.7, math.radians(30.0), 0.05, math.radians(60.0))


def lens_truth(w: Workload) -> np.ndarray:
    """True lens genome (7 doubles) of a workload's mock image."""
    rng = np.random.default_rng(w.seed)
    if w.name == "c1":
        return np.array([0.8, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    off = rng.uniform(-0.05, 0.05, size=2)
    return np.array(list(C2_LENS_FIXED) + [off[0], off[1]])


def source_blobs(w: Workload) -> list:
    """Analytic source blobs as dicts; amplitudes A ~ U(0.5, 1).

    Gaussians (c1): centre U(-0.25,0.25)^2, major-axis sigma U(0.05,0.15)",
    axis ratio U(0.5,1), PA U(0,pi).  Sersics (c2..c5): index n U(0.5,2),
    half-light radius U(0.05,0.2)", axis ratio U(0.5,1), PA U(0,pi),
    centre U(-0.3,0.3)^2.
    """
    rng = np.random.default_rng(1000 + w.seed)
    blobs = []
    for _ in range(w.n_blobs):
        if w.source_kind == "gauss":
            c = rng.uniform(-0.25, 0.25, size=2)
            blobs.append(dict(kind="gauss", amp=rng.uniform(0.5, 1.0), xc=c[0], yc=c[1],
                              size=rng.uniform(0.05, 0.15), q=rng.uniform(0.5, 1.0),
                              pa=rng.uniform(0.0, math.pi)))
        else:
            c = rng.uniform(-0.3, 0.3, size=2)
            blobs.append(dict(kind="sersic", amp=rng.uniform(0.5, 1.0), xc=c[0], yc=c[1],
                              n=rng.uniform(0.5, 2.0), size=rng.uniform(0.05, 0.2),
                              q=rng.uniform(0.5, 1.0), pa=rng.uniform(0.0, math.pi)))
    return blobs


def noise_unit(w: Workload) -> np.ndarray:
    """Standard-normal image (ny, nx); the mock image adds sigma times this."""
    rng = np.random.default_rng(2000 + w.seed)
    return rng.standard_normal((w.ny, w.nx))


def population(seed: int, n: int) -> np.ndarray:
    """n genomes uniform in the prior box, shape (n, 7)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=(n, 7))
    return PRIOR_LO + u * (PRIOR_HI - PRIOR_LO)


def member_grids(seed: int, n: int, lo: int = 32, hi: int = 96) -> np.ndarray:
    """Per-member source-grid sides n_s, uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed + 7)
    return rng.integers(lo, hi + 1, size=n).astype(np.int32)


def ga_draws(seed: int, pop: int, ngen: int, dims: int = 7) -> dict:
    """Random numbers one GA generation consumes, for reproducible GA steps.

    Returned per generation g (arrays of shape (ngen, ...)):
      partner   -- crossover partner index for each individual
      xstrength -- N(0, 1) draw scaled later by the crossover strength
      mut_mask  -- U(0,1) per gene, compared with the mutation probability
      mut_step  -- N(0, 1) per gene, scaled later by the mutation scale
      perm      -- tournament pairing permutation of the offspring
    """
    rng = np.random.default_rng(seed)
    return dict(
        partner=rng.integers(0, pop, size=(ngen, pop)),
        xstrength=rng.standard_normal((ngen, pop)),
        mut_mask=rng.uniform(size=(ngen, pop, dims)),
        mut_step=rng.standard_normal((ngen, pop, dims)),
        perm=np.stack([rng.permutation(pop) for _ in range(ngen)]),
    )


def mlp_init(seed: int, dims=(7, 256, 256, 1)) -> list:
    """He-uniform initial MLP weights and zero biases as FP64 arrays.

    Returns [(W0, b0), (W1, b1), (W2, b2)] with W of shape (fan_in, fan_out).
    """
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = math.sqrt(6.0 / a)
        out.append((rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)))
    return out


def mlp_batch(seed: int, batch: int) -> tuple:
    """A random (x, y) batch for MLP tests: x ~ N(0,1)^7, y ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, 7)), rng.standard_normal(batch)


def random_vector(seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n)


def mc_draws(seed: int, ny: int, nx: int) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian image (ny, nx): the random vector of the
    Monte Carlo degrees-of-freedom estimate, drawn once and handed to both sides."""
    rng = np.random.default_rng(seed + 1000)
    return rng.standard_normal((ny, nx))


def sinc_moffat_psf(K: int, fwhm_px: float = 3.0, q: float = 0.7, pa: float = 0.6, beta: float = 2.5,
                    sinc_period_px: float = 6.0) -> np.ndarray:
    """A non-separable K x K PSF of the kind the paper's large test uses
    (Sec. 4): an elliptical Moffat profile (axis ratio q, major axis at angle
    pa from +x, FWHM fwhm_px along the major axis, index beta) times the
    square of a radial sinc (so that it stays non-negative), sampled at pixel
    centres about (K-1)/2 and normalised to sum 1.
    Rotated and elliptical, so it is not rank 1 and takes the direct blur."""
    ck = (K - 1) / 2.0
    a = np.arange(K) - ck
    x, y = np.meshgrid(a, a)
    c, s = np.cos(pa), np.sin(pa)
    u, v = c * x + s * y, -s * x + c * y
    alpha = fwhm_px / (2.0 * np.sqrt(2.0 ** (1.0 / beta) - 1.0))
    moffat = (1.0 + (u * u + (v / q) ** 2) / (alpha * alpha)) ** (-beta)
    r = np.hypot(x, y)
    P = moffat * np.sinc(r / sinc_period_px) ** 2
    return P / P.sum()


def pso_draws(seed: int, n: int, steps: int, dims: int = 7) -> dict:
    """Random numbers of a particle swarm run: initial unit-box positions x0
    (n, dims) and the spring draws xi_p, xi_g (steps, n), all U(0, 1)."""
    rng = np.random.default_rng(seed + 2000)
    return dict(x0=rng.uniform(size=(n, dims)), xi_p=rng.uniform(size=(steps, n)),
                xi_g=rng.uniform(size=(steps, n)))
