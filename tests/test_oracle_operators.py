"""Pins of the oracle's L, B, H operators (Sec. 2.1-2.2, Eq. 7)."""
import numpy as np
import pytest

from oracle import lens, mock
import synthgen
from oracle import operators as ops


def _table(seed=0, n=200, ns=9, R=1.0):
    rng = np.random.default_rng(seed)
    bx = rng.uniform(-1.3, 1.3, (n, 4))
    by = rng.uniform(-1.3, 1.3, (n, 4))
    return bx, by, ops.bilinear_table(bx, by, ns, R)


def test_bilinear_reproduces_bilinear_functions():
    ns, R = 9, 1.0
    bx, by, tab = _table(ns=ns, R=R)
    h = 2 * R / (ns - 1)
    nodes = -R + np.arange(ns) * h
    NX, NY = np.meshgrid(nodes, nodes)
    f = lambda x, y: 0.3 + 1.7 * x - 0.9 * y + 2.2 * x * y
    s = f(NX, NY).reshape(-1)
    idx, w, inside = tab
    vals = (w * s[idx]).sum(axis=2)
    np.testing.assert_allclose(vals[inside], f(bx, by)[inside], atol=1e-13)
    # weights sum to one per inside subpixel, zero outside
    np.testing.assert_allclose(w.sum(axis=2)[inside], 1.0, atol=1e-15)
    assert np.all(w.sum(axis=2)[~inside] == 0)


def test_L_of_ones_counts_inside_subpixels():
    bx, by, tab = _table()
    img = ops.apply_L(tab, np.ones(81), 2)
    np.testing.assert_allclose(img, tab[2].sum(axis=1) / 4.0, atol=1e-15)


def test_grid_edges_inclusive():
    # a subpixel exactly on the last node row/column is inside and uses the last cell
    ns, R = 5, 1.0
    tab = ops.bilinear_table(np.array([[1.0, -1.0, 1.0 + 1e-12, 0.0]]),
                             np.array([[1.0, -1.0, 0.0, -1.0 - 1e-12]]), ns, R)
    idx, w, inside = tab
    assert list(inside[0]) == [True, True, False, False]
    assert idx[0, 0, 3] == ns * ns - 1 and w[0, 0, 3] == pytest.approx(1.0)
    assert idx[0, 1, 0] == 0 and w[0, 1, 0] == pytest.approx(1.0)


def test_adjoint_L():
    bx, by, tab = _table(seed=5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(81)
    y = rng.standard_normal(200)
    lhs = ops.apply_L(tab, x, 2) @ y
    rhs = x @ ops.apply_LT(tab, y, 81, 2)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    Lm = ops.dense_L(tab, 81, 2)
    np.testing.assert_allclose(Lm @ x, ops.apply_L(tab, x, 2), atol=1e-14)


@pytest.mark.parametrize("K", [3, 5, 7])
def test_adjoint_and_fft_B(K):
    rng = np.random.default_rng(K)
    P = rng.uniform(0, 1, (K, K))
    P /= P.sum()
    x = rng.standard_normal((11, 13))
    y = rng.standard_normal((11, 13))
    bx = ops.apply_B(P, x)
    assert abs((bx * y).sum() - (x * ops.apply_BT(P, y)).sum()) < 1e-12
    # zero-padded linear convolution via FFT padded to >= N + K - 1 (independent)
    ny, nx = x.shape
    sy, sx = ny + K - 1, nx + K - 1
    full = np.real(np.fft.ifft2(np.fft.fft2(x, (sy, sx)) * np.fft.fft2(P, (sy, sx))))
    ck = (K - 1) // 2
    np.testing.assert_allclose(bx, full[ck:ck + ny, ck:ck + nx], atol=1e-12)


def test_B_delta_and_flux():
    P = mock.gaussian_psf(5, 1.5)
    assert abs(P.sum() - 1) < 1e-15
    e = np.zeros((9, 9))
    e[4, 4] = 1.0
    np.testing.assert_allclose(ops.apply_B(P, e)[2:7, 2:7], P, atol=1e-16)
    rng = np.random.default_rng(0)
    x = np.zeros((20, 20))
    x[5:15, 5:15] = rng.uniform(size=(10, 10))
    assert abs(ops.apply_B(P, x).sum() - x.sum()) < 1e-12


def test_gaussian_psf_fwhm():
    # the sampled profile along a row through the centre is exp(-a^2/(2 sig^2)),
    # with half maximum at a = FWHM/2
    P = mock.gaussian_psf(15, 3.0)
    row = P[7] / P[7, 7]
    sig = 3.0 / (2 * np.sqrt(2 * np.log(2)))
    np.testing.assert_allclose(row, np.exp(-(np.arange(15) - 7.0) ** 2 / (2 * sig * sig)), rtol=1e-14)
    assert abs(np.exp(-(1.5 ** 2) / (2 * sig * sig)) - 0.5) < 1e-15


def test_dense_B_matches_operator():
    P = mock.gaussian_psf(3, 1.0)
    Bm = ops.dense_B(P, 5, 4)
    x = np.random.default_rng(1).standard_normal((4, 5))
    np.testing.assert_allclose(Bm @ x.reshape(-1), ops.apply_B(P, x).reshape(-1), atol=1e-15)
    np.testing.assert_allclose(Bm.T @ x.reshape(-1), ops.apply_BT(P, x).reshape(-1), atol=1e-15)


def test_curvature_H_rows():
    ns = 6
    Hm = ops.dense_H(ns, "curvature")
    HtH = Hm.T @ Hm
    # along one axis the 1-D Dirichlet D^2 has rows [5,-4,1], [-4,6,-4,1], [1,-4,6,-4,1]
    D = np.diag(-2.0 * np.ones(ns)) + np.diag(np.ones(ns - 1), 1) + np.diag(np.ones(ns - 1), -1)
    D2 = D @ D
    assert list(D2[0, :3]) == [5, -4, 1] and list(D2[1, :4]) == [-4, 6, -4, 1]
    assert list(D2[2, :5]) == [1, -4, 6, -4, 1]
    Id = np.eye(ns)
    np.testing.assert_allclose(HtH, np.kron(Id, D2) + np.kron(D2, Id), atol=0)
    # SPD
    assert np.linalg.eigvalsh(HtH).min() > 0
    rng = np.random.default_rng(2)
    x = rng.standard_normal(ns * ns)
    y = rng.standard_normal(ns * ns)
    hx = ops.apply_H(x, ns, "curvature")
    np.testing.assert_allclose(hx, Hm @ x, atol=1e-14)
    assert abs(hx @ ops.apply_H(y, ns, "curvature") - x @ ops.apply_HtH(y, ns, "curvature")) < 1e-11


@pytest.mark.parametrize("ns", [2, 7, 12])
def test_curvature_HtH_diagonalised_by_sine_transform(ns):
    """The spectral preconditioner of the FP32 solve applies (c I + lambda H^T H)^-1
    through the 2-D type-I sine transform: S = DST-I (orthonormal, scipy's own
    routine) must diagonalise the oracle's dense H^T H with eigenvalues
    mu_j + mu_k, mu_k = 16 sin^4(pi (k+1) / (2 (ns+1)))."""
    from scipy.fft import dst
    Hm = ops.dense_H(ns, "curvature")
    HtH = Hm.T @ Hm
    S = dst(np.eye(ns), type=1, norm="ortho", axis=0)
    np.testing.assert_allclose(S @ S, np.eye(ns), atol=1e-13)
    S2 = np.kron(S, S)
    mu = 16.0 * np.sin(np.pi * np.arange(1, ns + 1) / (2.0 * (ns + 1))) ** 4
    lam2 = (mu[:, None] + mu[None, :]).reshape(-1)
    np.testing.assert_allclose(S2 @ HtH @ S2, np.diag(lam2), atol=1e-11)
    # the preconditioner's inverse through the transform equals the dense inverse
    c, lam = 0.37, 2.5
    Minv = S2 @ np.diag(1.0 / (c + lam * lam2)) @ S2
    np.testing.assert_allclose(Minv @ (c * np.eye(ns * ns) + lam * HtH), np.eye(ns * ns), atol=1e-11)


def test_identity_H():
    x = np.arange(9.0)
    np.testing.assert_array_equal(ops.apply_HtH(x, 3, "identity"), x)


@pytest.mark.parametrize("n", [0.5, 0.8, 1.0, 1.5, 2.0])
def test_sersic_bn_against_incomplete_gamma(n):
    """b_n is defined by gamma(2n, b_n) = Gamma(2n) / 2 (half the light inside R_e);
    the asymptotic series must agree with that root to its known accuracy."""
    from scipy.special import gammaincinv
    exact = gammaincinv(2.0 * n, 0.5)
    assert abs(mock.sersic_bn(n) - exact) <= 2e-3 * exact


@pytest.mark.parametrize("n", [0.7, 1.6])
def test_sersic_profile_half_light_radius(n):
    """A circular Sersic blob holds half its flux inside R_e (quadrature of the
    profile that source_brightness evaluates)."""
    blob = dict(kind="sersic", xc=0.0, yc=0.0, pa=0.3, q=1.0, size=0.2, n=n, amp=1.0)
    r = np.linspace(0.0, 40 * blob["size"], 400001)
    I = mock.source_brightness(r, np.zeros_like(r), [blob])
    ring = 2 * np.pi * r * I
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (ring[1:] + ring[:-1]) * np.diff(r))])
    inside = np.interp(blob["size"], r, cum)
    assert abs(inside / cum[-1] - 0.5) <= 3e-3


def test_nearest_neighbour_L_picks_the_nearest_node():
    """Nearest-neighbour interpolation (Sec. 2.1): each subpixel takes the value
    of the grid node nearest its back-traced position (rounded half up),
    computed here directly from the positions; L^T is its transpose."""
    from oracle import lens as olens
    ns, R, nsub, nx, ny, pix = 9, 0.6, 2, 16, 14, 0.08
    g = np.array([0.3, 0.8, 0.5, 0.02, 0.1, 0.01, -0.02])
    bx, by = olens.trace_image(g, nx, ny, pix, nsub)
    tab = ops.bilinear_table(bx, by, ns, R, nearest=True)
    s = np.random.default_rng(2).standard_normal(ns * ns)
    h = 2 * R / (ns - 1)
    u, v = (bx + R) / h, (by + R) / h
    inside = (u >= 0) & (u <= ns - 1) & (v >= 0) & (v <= ns - 1)
    cu = np.clip(np.floor(u + 0.5), 0, ns - 1).astype(int)
    cv = np.clip(np.floor(v + 0.5), 0, ns - 1).astype(int)
    want = np.where(inside, s[cv * ns + cu], 0.0).sum(axis=1) / nsub ** 2
    got = ops.apply_L(tab, s, nsub)
    assert np.allclose(got, want, rtol=0, atol=1e-14)
    y = np.random.default_rng(3).standard_normal(nx * ny)
    assert abs(got @ y - s @ ops.apply_LT(tab, y, ns * ns, nsub)) <= 1e-12 * np.abs(got).sum()


def test_bicubic_weights_and_quadratic_reproduction():
    """Bicubic interpolation (Sec. 2.1) by cubic convolution (Keys 1981,
    a = -1/2): the four weights sum to one, t = 0 and t = 1 hit the nodes, and
    the scheme reproduces quadratics exactly, so wherever the 4 x 4 stencil
    lies inside the grid L returns the quadratic's value at the subpixel;
    L^T is its transpose."""
    t = np.linspace(0, 1, 11)
    W = ops.keys_weights(t)
    assert np.allclose(W.sum(axis=-1), 1.0, atol=1e-15)
    assert np.allclose(W[0], [0, 1, 0, 0]) and np.allclose(W[-1], [0, 0, 1, 0])
    ns, R, nsub, nx, ny, pix = 12, 0.6, 2, 18, 16, 0.06
    g = np.array([0.3, 0.8, 0.5, 0.02, 0.1, 0.01, -0.02])
    bx, by = lens.trace_image(g, nx, ny, pix, nsub)
    tab = ops.bicubic_table(bx, by, ns, R)
    h = 2 * R / (ns - 1)
    cc, rr = np.meshgrid(np.arange(ns), np.arange(ns))
    quad = lambda x, y: 0.3 + 0.2 * x - 0.1 * y + 0.05 * x * x + 0.07 * x * y - 0.03 * y * y   # noqa: E731
    s = quad(cc, rr).reshape(-1).astype(np.float64)
    idx, w, inside = tab
    u, v = (bx + R) / h, (by + R) / h
    interior = inside & (u >= 1) & (u <= ns - 2) & (v >= 1) & (v <= ns - 2)
    got = (w * s[idx]).sum(axis=-1)
    assert interior.sum() > 50
    assert np.allclose(got[interior], quad(u, v)[interior], rtol=0, atol=1e-12)
    y = np.random.default_rng(3).standard_normal(nx * ny)
    Ls = ops.apply_L(tab, s, nsub)
    assert abs(Ls @ y - s @ ops.apply_LT(tab, y, ns * ns, nsub)) <= 1e-12 * np.abs(Ls).sum()


@pytest.mark.parametrize("shape,K", [((7, 9), 3), ((11, 13), 5), ((40, 33), 15), ((24, 20), 65), ((66, 70), 65)])
def test_fourier_blur_equals_the_direct_sums(shape, K):
    """B and B^T through the Fourier transform (Sec. 2.2) equal the direct sums
    of the definition, also when the PSF is wider than the image, and stay
    adjoint."""
    rng = np.random.default_rng(K + shape[0])
    P = rng.uniform(0, 1, (K, K))
    P /= P.sum()
    x = rng.standard_normal(shape)
    z = rng.standard_normal(shape)
    bx = ops.apply_B(P, x)
    btz = ops.apply_BT(P, z)
    scale = np.abs(x).max()
    np.testing.assert_allclose(ops.apply_B_fft(P, x), bx, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(ops.apply_BT_fft(P, z), btz, rtol=0, atol=1e-13 * np.abs(z).max())
    lhs = (ops.apply_B_fft(P, x) * z).sum()
    rhs = (x * ops.apply_BT_fft(P, z)).sum()
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_problem_fft_blur_matches_direct_problem():
    """The oracle problem with blur="fft" gives the operator of the direct one."""
    from oracle import solve
    w = synthgen.C1
    rng = np.random.default_rng(3)
    d = rng.standard_normal((w.ny, w.nx))
    psf = mock.gaussian_psf(9, 2.5)
    lens = np.array([0.8, 0.8, 0.3, 0.02, 0.1, 0.01, -0.02])
    a = solve.Problem(lens, d, 1.0, psf, w.nx, w.ny, w.pix, 2, 16, 0.5, "identity")
    b = solve.Problem(lens, d, 1.0, psf, w.nx, w.ny, w.pix, 2, 16, 0.5, "identity", blur="fft")
    s = rng.standard_normal(a.I)
    np.testing.assert_allclose(b.F(s), a.F(s), rtol=0, atol=1e-12 * np.abs(a.F(s)).max())
    np.testing.assert_allclose(b.FT(d), a.FT(d), rtol=0, atol=1e-12 * np.abs(a.FT(d)).max())
