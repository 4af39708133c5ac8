"""Pins of the oracle's ray tracing against closed forms (Eq. 1, Eqs. 10-11)."""
import math

import numpy as np
import pytest

from oracle import lens


def test_sis_closed_form():
    # SIS (q = 1): beta = theta (1 - b/|theta|)
    rng = np.random.default_rng(0)
    x = rng.uniform(-2, 2, 500)
    y = rng.uniform(-2, 2, 500)
    b = 0.8
    bx, by = lens.trace(x, y, [b, 1.0, 0.3, 0.0, 0.0, 0.0, 0.0])
    r = np.hypot(x, y)
    np.testing.assert_allclose(bx, x * (1 - b / r), rtol=0, atol=1e-13)
    np.testing.assert_allclose(by, y * (1 - b / r), rtol=0, atol=1e-13)


def test_einstein_ring_maps_to_origin():
    b = 0.8
    phi = np.linspace(0, 2 * math.pi, 97)
    bx, by = lens.trace(b * np.cos(phi), b * np.sin(phi), [b, 1.0, 0.0, 0, 0, 0, 0])
    assert np.abs(bx).max() < 1e-14 and np.abs(by).max() < 1e-14


def _fd_jacobian(f, x, y, h=1e-6):
    axp, ayp = f(x + h, y)
    axm, aym = f(x - h, y)
    dxx = (axp - axm) / (2 * h)
    dyx = (ayp - aym) / (2 * h)
    axp, ayp = f(x, y + h)
    axm, aym = f(x, y - h)
    dxy = (axp - axm) / (2 * h)
    dyy = (ayp - aym) / (2 * h)
    return dxx, dxy, dyx, dyy


@pytest.mark.parametrize("q,pa", [(0.7, 0.0), (0.4, 0.9), (0.95, 2.5)])
def test_sie_divergence_and_curl(q, pa):
    # div alpha = 2 kappa = b q / psi and alpha is curl-free (it is a gradient)
    b = 1.1
    rng = np.random.default_rng(1)
    x = rng.uniform(-2, 2, 200)
    y = rng.uniform(-2, 2, 200)
    keep = np.hypot(x, y) > 0.2
    x, y = x[keep], y[keep]
    f = lambda xx, yy: lens.sie_deflection(xx, yy, b, q, pa)
    dxx, dxy, dyx, dyy = _fd_jacobian(f, x, y)
    c, s = math.cos(pa), math.sin(pa)
    xp = c * x + s * y
    yp = -s * x + c * y
    psi = np.sqrt(q * q * xp * xp + yp * yp)
    np.testing.assert_allclose(dxx + dyy, b * q / psi, rtol=1e-6)
    np.testing.assert_allclose(dxy, dyx, atol=1e-6)


def test_sie_on_axis():
    # on the x' axis psi = q|x'| so alpha'_x = (b q / k) atan(k/q) sign(x')
    b, q = 1.0, 0.6
    k = math.sqrt(1 - q * q)
    x = np.array([-1.3, -0.2, 0.5, 2.0])
    ax, ay = lens.sie_deflection(x, np.zeros_like(x), b, q, 0.0)
    np.testing.assert_allclose(ax, b * q / k * math.atan(k / q) * np.sign(x), rtol=1e-14)
    np.testing.assert_allclose(ay, 0.0, atol=1e-15)


def test_sie_limits_and_symmetry():
    rng = np.random.default_rng(2)
    x = rng.uniform(-2, 2, 100)
    y = rng.uniform(-2, 2, 100)
    # q -> 1 reduces to SIS
    a1 = lens.sie_deflection(x, y, 1.0, 1.0 - 1e-7, 0.4)
    r = np.hypot(x, y)
    np.testing.assert_allclose(a1[0], x / r, atol=1e-6)
    np.testing.assert_allclose(a1[1], y / r, atol=1e-6)
    # alpha is odd about the centre
    ap = lens.sie_deflection(x, y, 1.2, 0.5, 0.7, 0.03, -0.02)
    am = lens.sie_deflection(0.06 - x, -0.04 - y, 1.2, 0.5, 0.7, 0.03, -0.02)
    np.testing.assert_allclose(ap[0], -am[0], atol=1e-14)
    np.testing.assert_allclose(ap[1], -am[1], atol=1e-14)
    # zero deflection exactly at the centre
    a0 = lens.sie_deflection(np.array([0.1]), np.array([0.2]), 1.0, 0.5, 0.3, 0.1, 0.2)
    assert a0[0][0] == 0.0 and a0[1][0] == 0.0


def test_sie_rotation_covariance():
    # rotating the lens by PA rotates the deflection field
    rng = np.random.default_rng(3)
    x = rng.uniform(-2, 2, 50)
    y = rng.uniform(-2, 2, 50)
    pa = 0.8
    a_rot = lens.sie_deflection(x, y, 1.0, 0.6, pa)
    c, s = math.cos(pa), math.sin(pa)
    xp, yp = c * x + s * y, -s * x + c * y
    a_unrot = lens.sie_deflection(xp, yp, 1.0, 0.6, 0.0)
    np.testing.assert_allclose(a_rot[0], c * a_unrot[0] - s * a_unrot[1], atol=1e-14)
    np.testing.assert_allclose(a_rot[1], s * a_unrot[0] + c * a_unrot[1], atol=1e-14)


def test_shear_is_gradient_of_its_potential():
    # psi_sh = gamma/2 r^2 cos 2(phi - phi_g) = g1 (x^2-y^2)/2 + g2 x y
    g, gp = 0.07, 0.6
    rng = np.random.default_rng(4)
    x = rng.uniform(-2, 2, 50)
    y = rng.uniform(-2, 2, 50)
    pot = lambda xx, yy: 0.5 * g * (xx * xx + yy * yy) * np.cos(2 * (np.arctan2(yy, xx) - gp))
    h = 1e-6
    ax, ay = lens.shear_deflection(x, y, g, gp)
    np.testing.assert_allclose(ax, (pot(x + h, y) - pot(x - h, y)) / (2 * h), atol=1e-8)
    np.testing.assert_allclose(ay, (pot(x, y + h) - pot(x, y - h)) / (2 * h), atol=1e-8)


def test_subpixel_layout():
    x, y = lens.subpixel_positions(4, 3, 0.1, 2)
    assert x.shape == (12, 4)
    # pixel (r=0, c=0) centre (-0.15, -0.1); subpixel 1 is +x, subpixel 2 is +y
    np.testing.assert_allclose(x[0], [-0.175, -0.125, -0.175, -0.125])
    np.testing.assert_allclose(y[0], [-0.125, -0.125, -0.075, -0.075])
    # pixel j = r*nx + c
    np.testing.assert_allclose(x[5].mean(), (1 - 1.5) * 0.1)
    np.testing.assert_allclose(y[5].mean(), (1 - 1.0) * 0.1)
