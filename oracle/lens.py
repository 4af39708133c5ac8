"""Ray tracing through an SIE/SIS lens with external shear (FP64 oracle).

Paper: thin-lens mapping beta = theta - alpha(theta) (Sec. 2, Eq. 1); SIE
deflection in Keeton's form (Sec. 2.3, Eqs. 10-11) with core s = 0; SIS is
the q = 1 case (Sec. 4); subpixel ray tracing, N_p subpixels per image pixel
(Sec. 2.2).

Readings where the paper is silent:
* pixel (r, c) has centre ((c-(Nx-1)/2) p, (r-(Ny-1)/2) p); its n x n
  subpixels sit at offsets ((a+1/2)/n - 1/2) p; subpixel k = sr*n + sc with
  sr along y and sc along x.
* theta_E is the paper's b.  The mass major axis lies along the lens-frame x'
  axis; PA is counter-clockwise from +x.
* psi = 0 gives zero deflection; for k = sqrt(1-q^2) < 1e-4 the SIS limit
  alpha' = b q (x', y') / psi is used.
* External shear (gamma, phi_gamma) about the lens centre:
  alpha_sh = (g1 dx + g2 dy, g2 dx - g1 dy), g1 = gamma cos 2phi,
  g2 = gamma sin 2phi.
"""
from __future__ import annotations

import math

import numpy as np


def pixel_centres(nx: int, ny: int, pix: float):
    """Image-plane pixel centres, arrays of shape (ny, nx)."""
    xs = (np.arange(nx) - (nx - 1) / 2.0) * pix
    ys = (np.arange(ny) - (ny - 1) / 2.0) * pix
    return np.meshgrid(xs, ys)  # X[r, c] = xs[c], Y[r, c] = ys[r]


def subpixel_positions(nx: int, ny: int, pix: float, nsub: int):
    """Subpixel positions, arrays of shape (ny*nx, nsub*nsub).

    Row j = r*nx + c is the pixel; column k = sr*nsub + sc the subpixel.
    """
    X, Y = pixel_centres(nx, ny, pix)
    off = ((np.arange(nsub) + 0.5) / nsub - 0.5) * pix
    ox = np.tile(off, nsub)        # sc varies fastest
    oy = np.repeat(off, nsub)      # sr
    x = X.reshape(-1, 1) + ox.reshape(1, -1)
    y = Y.reshape(-1, 1) + oy.reshape(1, -1)
    return x, y


def sie_deflection(x, y, theta_e, q, pa, x0=0.0, y0=0.0):
    """SIE deflection (Eqs. 10-11 with s = 0), rotated by PA, centred at (x0, y0)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    dx = x - x0
    dy = y - y0
    cp, sp = math.cos(pa), math.sin(pa)
    xp = cp * dx + sp * dy
    yp = -sp * dx + cp * dy
    psi = np.sqrt(q * q * xp * xp + yp * yp)
    k = math.sqrt(max(0.0, 1.0 - q * q))
    safe = psi > 0.0
    psis = np.where(safe, psi, 1.0)
    if k < 1e-4:
        axp = theta_e * q * xp / psis
        ayp = theta_e * q * yp / psis
    else:
        axp = (theta_e * q / k) * np.arctan(k * xp / psis)
        ayp = (theta_e * q / k) * np.arctanh(k * yp / psis)
    axp = np.where(safe, axp, 0.0)
    ayp = np.where(safe, ayp, 0.0)
    ax = cp * axp - sp * ayp
    ay = sp * axp + cp * ayp
    return ax, ay


def shear_deflection(x, y, gamma, gamma_pa, x0=0.0, y0=0.0):
    """Uniform external shear about (x0, y0); linear in (dx, dy)."""
    dx = np.asarray(x, dtype=np.float64) - x0
    dy = np.asarray(y, dtype=np.float64) - y0
    g1 = gamma * math.cos(2.0 * gamma_pa)
    g2 = gamma * math.sin(2.0 * gamma_pa)
    return g1 * dx + g2 * dy, g2 * dx - g1 * dy


def trace(x, y, lens):
    """Thin-lens mapping beta = theta - alpha(theta) (Eq. 1).

    ``lens`` is the genome (theta_e, q, pa, gamma, gamma_pa, x0, y0).
    """
    theta_e, q, pa, gamma, gamma_pa, x0, y0 = [float(v) for v in lens]
    ax, ay = sie_deflection(x, y, theta_e, q, pa, x0, y0)
    sx, sy = shear_deflection(x, y, gamma, gamma_pa, x0, y0)
    return np.asarray(x) - ax - sx, np.asarray(y) - ay - sy


def trace_image(lens, nx, ny, pix, nsub):
    """Back-traced source-plane positions of every subpixel, (J, n^2) each."""
    x, y = subpixel_positions(nx, ny, pix, nsub)
    return trace(x, y, lens)
