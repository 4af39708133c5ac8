"""Lens operator L, blur B and regularisation H (FP64 oracle).

Paper: the model image is f = B L applied to the source vector (Sec. 2.1,
Eq. 3); L interpolates the source at the stored back-traced subpixel
positions and its transpose redistributes image values to the same
positions (Sec. 2.2); bilinear source interpolation (Sec. 2.1); subpixel
intensities are averaged and pixels that do not map get no intensity
(Sec. 2.2); B convolves with the PSF (Sec. 2.2); H = I or a finite-difference
second-derivative operator (Eq. 7).

Readings where the paper is silent:
* source grid: n_s x n_s nodes at (-R + c h, -R + r h), h = 2R/(n_s-1),
  node i = r n_s + c.
* a subpixel at (u, v) = ((beta_x+R)/h, (beta_y+R)/h) is inside iff
  0 <= u <= n_s-1 and 0 <= v <= n_s-1; c0 = min(floor u, n_s-2),
  r0 = min(floor v, n_s-2), fx = u-c0, fy = v-r0; the bilinear weights
  (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy go to nodes (r0,c0), (r0,c0+1),
  (r0+1,c0), (r0+1,c0+1), each divided by n^2 (always n^2, also when some
  subpixels of the pixel fall outside).
* B is the zero-padded "same"-size linear convolution
  (Bx)[r][c] = sum_{a,b} P[a][b] x[r-a+cK][c-b+cK], cK = (K-1)/2;
  B^T is the matching correlation.
* curvature H stacks D_xx and D_yy: second differences along x and along y
  with the source taken as zero outside the grid, one row per node per axis.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# bilinear lens operator
# --------------------------------------------------------------------------
def bilinear_table(bx, by, ns: int, half_width: float, nearest: bool = False):
    """Per-subpixel node indices and weights (before the 1/n^2 average).

    Returns (idx, w, inside): idx int64 (J, n2, 4), w float64 (J, n2, 4),
    inside bool (J, n2).  Outside subpixels get idx 0 and weight 0.
    nearest: nearest-neighbour interpolation instead (Sec. 2.1): the node of
    the cell nearest the subpixel gets weight 1 (reading: a fraction of
    exactly 1/2 goes to the upper node), written as the bilinear weights of
    the fractions rounded to 0 or 1.
    """
    h = 2.0 * half_width / (ns - 1)
    u = (np.asarray(bx) + half_width) / h
    v = (np.asarray(by) + half_width) / h
    inside = (u >= 0.0) & (u <= ns - 1) & (v >= 0.0) & (v <= ns - 1)
    us = np.where(inside, u, 0.0)
    vs = np.where(inside, v, 0.0)
    c0 = np.minimum(np.floor(us), ns - 2).astype(np.int64)
    r0 = np.minimum(np.floor(vs), ns - 2).astype(np.int64)
    fx = us - c0
    fy = vs - r0
    if nearest:
        fx = np.where(fx >= 0.5, 1.0, 0.0)
        fy = np.where(fy >= 0.5, 1.0, 0.0)
    i00 = r0 * ns + c0
    idx = np.stack([i00, i00 + 1, i00 + ns, i00 + ns + 1], axis=-1)
    w = np.stack([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy], axis=-1)
    w = np.where(inside[..., None], w, 0.0)
    idx = np.where(inside[..., None], idx, 0)
    return idx, w, inside


def keys_weights(t):
    """Cubic convolution weights (Keys 1981, a = -1/2) of the taps at offsets
    -1, 0, 1, 2 from the cell's first node, for the fraction t in [0, 1]."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([((-0.5 * t + 1.0) * t - 0.5) * t,
                     (1.5 * t - 2.5) * t * t + 1.0,
                     ((-1.5 * t + 2.0) * t + 0.5) * t,
                     (0.5 * t - 0.5) * t * t], axis=-1)


def bicubic_table(bx, by, ns: int, half_width: float):
    """Bicubic source interpolation (Sec. 2.1): the 4 x 4 nodes about the
    subpixel's cell, weighted by cubic convolution in x and in y (Keys, a =
    -1/2).  Reading: the cell and its fractions are those of the bilinear
    table; a tap on a node outside the grid takes the source there as zero
    (weight 0).  Returns (idx, w, inside) with a last axis of 16 taps
    (row offset j, column offset i: tap 4 (j + 1) + (i + 1))."""
    h = 2.0 * half_width / (ns - 1)
    u = (np.asarray(bx) + half_width) / h
    v = (np.asarray(by) + half_width) / h
    inside = (u >= 0.0) & (u <= ns - 1) & (v >= 0.0) & (v <= ns - 1)
    us = np.where(inside, u, 0.0)
    vs = np.where(inside, v, 0.0)
    c0 = np.minimum(np.floor(us), ns - 2).astype(np.int64)
    r0 = np.minimum(np.floor(vs), ns - 2).astype(np.int64)
    wx = keys_weights(us - c0)
    wy = keys_weights(vs - r0)
    idx = np.zeros(c0.shape + (16,), dtype=np.int64)
    w = np.zeros(c0.shape + (16,))
    for j in range(4):
        for i in range(4):
            r, c = r0 + j - 1, c0 + i - 1
            ok = inside & (r >= 0) & (r < ns) & (c >= 0) & (c < ns)
            idx[..., 4 * j + i] = np.where(ok, r * ns + c, 0)
            w[..., 4 * j + i] = np.where(ok, wy[..., j] * wx[..., i], 0.0)
    return idx, w, inside


def apply_L(table, s, nsub: int):
    """Unblurred lensed image: img_j = n^-2 sum_sub sum_corner w s[node]."""
    idx, w, _ = table
    s = np.asarray(s, dtype=np.float64)
    return (w * s[idx]).sum(axis=(1, 2)) / (nsub * nsub)


def apply_LT(table, img, n_nodes: int, nsub: int):
    """Exact transpose of ``apply_L``: s[node] += n^-2 w img_j."""
    idx, w, _ = table
    img = np.asarray(img, dtype=np.float64).reshape(-1)
    out = np.zeros(n_nodes)
    np.add.at(out, idx.reshape(-1), (w * img[:, None, None]).reshape(-1) / (nsub * nsub))
    return out


def dense_L(table, n_nodes: int, nsub: int):
    """Explicit (J, I) matrix of L."""
    idx, w, _ = table
    J = idx.shape[0]
    Lm = np.zeros((J, n_nodes))
    rows = np.repeat(np.arange(J), idx.shape[1] * idx.shape[2])
    np.add.at(Lm, (rows, idx.reshape(-1)), w.reshape(-1) / (nsub * nsub))
    return Lm


# --------------------------------------------------------------------------
# PSF blur
# --------------------------------------------------------------------------
def apply_B(psf, img):
    """(Bx)[r][c] = sum_{a,b} P[a][b] x[r-a+cK][c-b+cK], zero outside."""
    P = np.asarray(psf, dtype=np.float64)
    x = np.asarray(img, dtype=np.float64)
    K = P.shape[0]
    ck = (K - 1) // 2
    ny, nx = x.shape
    xp = np.zeros((ny + 2 * ck, nx + 2 * ck))
    xp[ck:ck + ny, ck:ck + nx] = x
    out = np.zeros_like(x)
    for a in range(K):
        for b in range(P.shape[1]):
            # x[r - a + ck][c - b + ck] -> padded index r - a + 2ck
            out += P[a, b] * xp[2 * ck - a:2 * ck - a + ny, 2 * ck - b:2 * ck - b + nx]
    return out


def apply_BT(psf, img):
    """(B^T z)[r][c] = sum_{a,b} P[a][b] z[r+a-cK][c+b-cK], zero outside."""
    P = np.asarray(psf, dtype=np.float64)
    z = np.asarray(img, dtype=np.float64)
    K = P.shape[0]
    ck = (K - 1) // 2
    ny, nx = z.shape
    zp = np.zeros((ny + 2 * ck, nx + 2 * ck))
    zp[ck:ck + ny, ck:ck + nx] = z
    out = np.zeros_like(z)
    for a in range(K):
        for b in range(P.shape[1]):
            out += P[a, b] * zp[a:a + ny, b:b + nx]
    return out


def apply_B_fft(psf, img):
    """apply_B computed in Fourier space (Sec. 2.2: the convolution with the
    PSF is done there): the full linear convolution of the image with the PSF
    from the product of their discrete Fourier transforms on a frame of
    (ny + K - 1) x (nx + K - 1), large enough that nothing wraps, cropped to
    the image: (B x)[r][c] = full[r + cK][c + cK]."""
    P = np.asarray(psf, dtype=np.float64)
    x = np.asarray(img, dtype=np.float64)
    K = P.shape[0]
    ck = (K - 1) // 2
    ny, nx = x.shape
    shape = (ny + K - 1, nx + K - 1)
    full = np.fft.irfft2(np.fft.rfft2(x, shape) * np.fft.rfft2(P, shape), shape)
    return full[ck:ck + ny, ck:ck + nx]


def apply_BT_fft(psf, img):
    """apply_BT in Fourier space: the correlation with P is the convolution
    with P turned by 180 degrees, (B^T z)[r][c] = sum P[K-1-a][K-1-b]
    z[r-a+cK][c-b+cK]."""
    P = np.asarray(psf, dtype=np.float64)
    return apply_B_fft(P[::-1, ::-1], img)


def dense_B(psf, nx: int, ny: int):
    """Explicit (J, J) matrix of B, column by column from unit images."""
    J = nx * ny
    Bm = np.zeros((J, J))
    e = np.zeros((ny, nx))
    for j in range(J):
        e.flat[j] = 1.0
        Bm[:, j] = apply_B(psf, e).reshape(-1)
        e.flat[j] = 0.0
    return Bm


# --------------------------------------------------------------------------
# regularisation
# --------------------------------------------------------------------------
def apply_H(s, ns: int, kind: str):
    """H s: identity, or stacked [D_xx s; D_yy s] (Dirichlet second differences)."""
    s = np.asarray(s, dtype=np.float64)
    if kind == "identity":
        return s.copy()
    g = np.zeros((ns + 2, ns + 2))
    g[1:-1, 1:-1] = s.reshape(ns, ns)
    dxx = g[1:-1, :-2] - 2.0 * g[1:-1, 1:-1] + g[1:-1, 2:]
    dyy = g[:-2, 1:-1] - 2.0 * g[1:-1, 1:-1] + g[2:, 1:-1]
    return np.concatenate([dxx.reshape(-1), dyy.reshape(-1)])


def apply_HT(hs, ns: int, kind: str):
    """H^T of ``apply_H`` (each second-difference operator is symmetric)."""
    hs = np.asarray(hs, dtype=np.float64)
    if kind == "identity":
        return hs.copy()
    I = ns * ns
    out = np.zeros(I)
    for part, axis in ((hs[:I], "x"), (hs[I:], "y")):
        g = np.zeros((ns + 2, ns + 2))
        g[1:-1, 1:-1] = part.reshape(ns, ns)
        if axis == "x":
            d = g[1:-1, :-2] - 2.0 * g[1:-1, 1:-1] + g[1:-1, 2:]
        else:
            d = g[:-2, 1:-1] - 2.0 * g[1:-1, 1:-1] + g[2:, 1:-1]
        out += d.reshape(-1)
    return out


def apply_HtH(s, ns: int, kind: str):
    return apply_HT(apply_H(s, ns, kind), ns, kind)


def dense_H(ns: int, kind: str):
    """Explicit H: (I, I) identity or (2I, I) stacked second differences."""
    I = ns * ns
    if kind == "identity":
        return np.eye(I)
    Hm = np.zeros((2 * I, I))
    for r in range(ns):
        for c in range(ns):
            i = r * ns + c
            Hm[i, i] = -2.0
            if c > 0:
                Hm[i, i - 1] = 1.0
            if c < ns - 1:
                Hm[i, i + 1] = 1.0
            Hm[I + i, i] = -2.0
            if r > 0:
                Hm[I + i, i - ns] = 1.0
            if r < ns - 1:
                Hm[I + i, i + ns] = 1.0
    return Hm
