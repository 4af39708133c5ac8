"""Pins of the oracle's L-curve (Sec. 2.6, Eq. 20), MLP and GA step."""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy.interpolate import CubicSpline

import synthgen
from oracle import ga, lcurve, mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- L-curve
def test_spline_matches_scipy_notaknot():
    rng = np.random.default_rng(0)
    t = np.cumsum(rng.uniform(0.1, 1.0, 9))
    y = rng.standard_normal(9)
    d1, d2 = lcurve.knot_derivatives(t, y)
    cs = CubicSpline(t, y, bc_type="not-a-knot")
    np.testing.assert_allclose(d1, cs(t, 1), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(d2, cs(t, 2), rtol=1e-10, atol=1e-12)


def test_spline_exact_on_cubics():
    t = np.array([0.0, 0.3, 1.1, 1.5, 2.6, 3.0])
    f = lambda x: 1 - 2 * x + 0.5 * x ** 2 - 0.7 * x ** 3
    d1, d2 = lcurve.knot_derivatives(t, f(t))
    np.testing.assert_allclose(d1, -2 + t - 2.1 * t ** 2, atol=1e-11)
    np.testing.assert_allclose(d2, 1 - 4.2 * t, atol=1e-11)


def test_circle_curvature():
    rho = 2.5
    phi = np.linspace(0.2, 1.4, 25)
    kappa, keep = lcurve.curvature_at_knots(rho * np.cos(phi), rho * np.sin(phi))
    np.testing.assert_allclose(kappa[2:-2], 1 / rho, rtol=1e-3)


def test_l_shaped_corner_on_arc():
    # vertical line, quarter circle of radius 0.2, horizontal line (an "L")
    ys = np.linspace(3.0, 0.3, 10)
    arc = np.linspace(math.pi, 1.5 * math.pi, 7)[1:-1]
    xs = np.linspace(0.3, 3.0, 10)
    X = np.concatenate([np.zeros(10), 0.2 + 0.2 * np.cos(arc), xs])
    Y = np.concatenate([ys, 0.2 + 0.2 * np.sin(arc), np.zeros(10)]) + 0.1
    k, kap = lcurve.corner(10 ** X, 10 ** Y)
    assert 10 <= k < 15


def _with_kappa(monkeypatch, kappa):
    """corner() with the spline stage replaced by fixed knot curvatures (all points kept)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    monkeypatch.setattr(lcurve, "curvature_at_knots", lambda X, Y: (kappa.copy(), np.arange(kappa.size)))
    n = kappa.size
    return lcurve.corner(np.logspace(0, 1, n), np.logspace(1, 0, n))[0]


def test_corner_tie_goes_to_smallest_index(monkeypatch):
    # equal maxima, and maxima within the relative 1e-12 tie band: the first wins
    assert _with_kappa(monkeypatch, [1.0, 3.0, 2.0, 3.0, 1.0]) == 1
    assert _with_kappa(monkeypatch, [1.0, 3.0, 2.0, 3.0 * (1 + 5e-13), 1.0]) == 1
    assert _with_kappa(monkeypatch, [1.0, 3.0 * (1 + 5e-13), 2.0, 3.0, 1.0]) == 1
    # outside the band the larger one wins, wherever it is
    assert _with_kappa(monkeypatch, [1.0, 3.0, 2.0, 3.0 * (1 + 1e-9), 1.0]) == 3
    assert _with_kappa(monkeypatch, [3.0 * (1 + 1e-9), 3.0, 2.0, 3.0, 1.0]) == 0
    assert _with_kappa(monkeypatch, [1.0, 2.0, 2.5, 2.0, 4.0]) == 4     # endpoints count


def test_corner_tie_on_a_mirror_symmetric_curve():
    # a curve with two identical bends: mirror image of itself under (X, Y) -> (Y, X) with
    # the order reversed, so kappa_k = kappa_{n-1-k} up to rounding; the corner is the first bend
    first = np.array([(0, 4), (0.02, 3.2), (0.05, 2.5), (0.1, 2.1), (0.25, 1.95), (0.6, 1.88), (1.0, 1.8),
                      (1.35, 1.65)], dtype=float)
    P = np.vstack([first, [[1.5, 1.5]], first[::-1][:, ::-1]])
    X, Y = P[:, 0], P[:, 1]
    kappa, keep = lcurve.curvature_at_knots(X, Y)
    assert keep.size == X.size
    np.testing.assert_allclose(kappa, kappa[::-1], rtol=1e-12)
    k, kap = lcurve.corner(10 ** X, 10 ** Y)
    i, j = np.argsort(-kappa)[:2]
    assert abs(kappa[i] - kappa[j]) <= 1e-12 * kappa[i]
    assert k == min(i, j) < X.size // 2


def test_corner_drops_repeated_points():
    # an L-curve with one point repeated exactly, and one repeated to within 1e-13 of the
    # total chord length: both repeats are dropped (NaN curvature) and the corner is that of
    # the curve without them; a point 1e-6 of the length away is kept
    lam = np.logspace(-3, 2, 12)
    reg = 1.0 / (1.0 + lam) ** 2 + 1e-3
    chi2 = 1.0 + lam / (1.0 + lam)
    k0, kap0 = lcurve.corner(reg, chi2)
    X, Y = np.log10(reg), np.log10(chi2)
    total = np.hypot(np.diff(X), np.diff(Y)).sum()
    reg2 = np.insert(reg, 6, reg[5])
    chi22 = np.insert(chi2, 6, chi2[5])
    k, kap = lcurve.corner(reg2, chi22)
    assert np.isnan(kap[6]) and np.isfinite(kap[5]) and np.sum(np.isnan(kap)) == 1
    assert k == (k0 if k0 <= 5 else k0 + 1)
    np.testing.assert_allclose(np.delete(kap, 6), kap0, rtol=1e-12)
    eps = 1e-13 * total / np.log10(np.e)
    reg3 = np.insert(reg, 3, reg[2] * (1 + eps))
    chi23 = np.insert(chi2, 3, chi2[2])
    _, kap3 = lcurve.corner(reg3, chi23)
    assert np.isnan(kap3[3]) and np.sum(np.isnan(kap3)) == 1
    reg4 = np.insert(reg, 3, reg[2] * (1 + 1e-6 * total / np.log10(np.e)))
    _, kap4 = lcurve.corner(reg4, np.insert(chi2, 3, chi2[2]))
    assert not np.isnan(kap4).any()


def test_corner_degenerate():
    assert lcurve.corner([1.0, 2.0, 3.0], [3.0, 2.0, 1.0])[0] == -1
    assert lcurve.corner([1.0, 0.0, 3.0, 4.0], [3.0, 2.0, 1.0, 0.5])[0] == -1
    # fewer than 4 distinct points after dropping repeats
    assert lcurve.corner([1.0, 1.0, 2.0, 3.0], [3.0, 3.0, 2.0, 1.0])[0] == -1


# --------------------------------------------------------------------------- MLP
def test_bf16_round_matches_torch():
    x = np.random.default_rng(0).standard_normal(4096) * 10.0
    x = np.concatenate([x, [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


def test_gelu_matches_torch():
    z = np.linspace(-6, 6, 1001)
    ref = torch.nn.functional.gelu(torch.tensor(z)).numpy()
    np.testing.assert_allclose(mlp.gelu(z), ref, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-8)


def test_mlp_gradients_finite_difference():
    params = synthgen.mlp_init(0, dims=(7, 16, 16, 1))
    x, y = synthgen.mlp_batch(1, 5)
    loss, grads = mlp.loss_and_grads(params, x, y)
    h = 1e-6
    rng = np.random.default_rng(2)
    for layer in range(3):
        for which in range(2):
            arr = params[layer][which]
            g = grads[layer][which]
            for _ in range(4):
                ix = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[ix]
                arr[ix] = old + h
                lp, _ = mlp.loss_and_grads(params, x, y)
                arr[ix] = old - h
                lm, _ = mlp.loss_and_grads(params, x, y)
                arr[ix] = old
                assert abs((lp - lm) / (2 * h) - g[ix]) <= 1e-6 * (1 + abs(g[ix]))


def test_mlp_matches_torch_autograd_and_adam():
    params = synthgen.mlp_init(3, dims=(7, 32, 32, 1))
    x, y = synthgen.mlp_batch(4, 9)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    xt = torch.tensor(x)
    h = torch.nn.functional.gelu(xt @ tp[0][0] + tp[0][1])
    h = torch.nn.functional.gelu(h @ tp[1][0] + tp[1][1])
    yt = (h @ tp[2][0] + tp[2][1]).reshape(-1)
    lt = ((yt - torch.tensor(y)) ** 2).mean()
    lt.backward()
    loss, grads = mlp.loss_and_grads(params, x, y)
    assert abs(loss - lt.item()) < 1e-12
    for (gW, gb), (W, b) in zip(grads, tp):
        np.testing.assert_allclose(gW, W.grad.numpy(), atol=1e-12)
        np.testing.assert_allclose(gb, b.grad.numpy(), atol=1e-12)
    flat = [p for pair in tp for p in pair]
    opt = torch.optim.Adam(flat, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m, v = mlp.zeros_like(params), mlp.zeros_like(params)
    p_or = params
    for t in range(1, 4):
        if t > 1:
            for p in flat:
                p.grad = None
            h = torch.nn.functional.gelu(xt @ tp[0][0] + tp[0][1])
            h = torch.nn.functional.gelu(h @ tp[1][0] + tp[1][1])
            yt = (h @ tp[2][0] + tp[2][1]).reshape(-1)
            ((yt - torch.tensor(y)) ** 2).mean().backward()
        _, g = mlp.loss_and_grads(p_or, x, y)
        opt.step()
        p_or, m, v = mlp.adam_step(p_or, g, m, v, t, 1e-2)
    for (W, b), (tW, tb) in zip(p_or, tp):
        np.testing.assert_allclose(W, tW.detach().numpy(), atol=1e-12)
        np.testing.assert_allclose(b, tb.detach().numpy(), atol=1e-12)


# --------------------------------------------------------------------------- GA
def test_ga_defaults_are_papers():
    with open(os.path.join(GOLDEN, "ferret_defaults.json")) as f:
        gold = json.load(f)
    import inspect
    sig = inspect.signature(ga.offspring)
    assert sig.parameters["xstrength"].default == gold["XOver.strength"]
    assert sig.parameters["pmutate"].default == gold["mutation.PMutate"]
    assert sig.parameters["mscale"].default == gold["mutation.scale"]


def test_ga_operators():
    P = 64
    X = np.random.default_rng(0).uniform(size=(P, 7))
    dr = {k: v[0] for k, v in synthgen.ga_draws(1, P, 1).items()}
    # no crossover and no mutation -> unchanged
    z = dict(dr, xstrength=np.zeros(P), mut_mask=np.ones((P, 7)))
    np.testing.assert_array_equal(ga.offspring(X, z), X)
    Y = ga.offspring(X, dr)
    assert Y.min() >= 0 and Y.max() <= 1
    # crossover-only offspring lie on the segment towards the partner (before clipping)
    z = dict(dr, mut_mask=np.ones((P, 7)), xstrength=np.full(P, 0.5))
    Y = ga.offspring(X, z, xstrength=1.0)
    np.testing.assert_allclose(Y, 0.5 * (X + X[dr["partner"]]), atol=1e-15)
    fX = np.arange(P, dtype=float)
    fY = np.full(P, 10.5)
    Xn, fn = ga.tournament(X, fX, Y, fY, dr["perm"])
    assert np.all(fn == np.minimum(fX, 10.5))
    assert np.all(Xn[fX <= 10.5] == X[fX <= 10.5])
