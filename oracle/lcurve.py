"""L-curve corner by arclength-parameterised cubic splines (FP64 oracle).

Paper (Sec. 2.6, Eq. 20): each solution contributes a point (regularisation
term, image chi^2); the curve is parameterised by arclength, x(t) and y(t)
are fitted with cubic splines, and the curvature
kappa = |x'y'' - y'x''| / (x'^2 + y'^2)^(3/2) is evaluated from the spline
derivatives; the solution of maximum curvature scores the lens.

Readings: the axes are log10(reg) and log10(chi^2); the parameter is the
chord length t_0 = 0, t_k = t_{k-1} + hypot(dX, dY); a point whose step is
<= 1e-12 of the total length is dropped; the splines are not-a-knot;
kappa is evaluated at the knots only (the corner must be a computed
solution); k* = argmax kappa over all knots, ties within a relative 1e-12 go
to the smallest index.  At least 4 distinct points are required.
"""
from __future__ import annotations

import numpy as np


def notaknot_moments(t, y):
    """Second derivatives M_i at the knots of the not-a-knot cubic spline.

    Interior rows are the usual C2 continuity conditions; the first and last
    rows make the third derivative continuous at t_1 and t_{n-2}.
    Solved as a dense linear system.
    """
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = t.size
    h = np.diff(t)
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    A[0, 0], A[0, 1], A[0, 2] = h[1], -(h[0] + h[1]), h[0]
    for i in range(1, n - 1):
        A[i, i - 1] = h[i - 1]
        A[i, i] = 2.0 * (h[i - 1] + h[i])
        A[i, i + 1] = h[i]
        rhs[i] = 6.0 * ((y[i + 1] - y[i]) / h[i] - (y[i] - y[i - 1]) / h[i - 1])
    A[n - 1, n - 3], A[n - 1, n - 2], A[n - 1, n - 1] = h[n - 2], -(h[n - 3] + h[n - 2]), h[n - 3]
    return np.linalg.solve(A, rhs)


def knot_derivatives(t, y):
    """(S'(t_i), S''(t_i)) of the not-a-knot spline at every knot."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    M = notaknot_moments(t, y)
    h = np.diff(t)
    n = t.size
    d1 = np.zeros(n)
    for i in range(n - 1):
        d1[i] = (y[i + 1] - y[i]) / h[i] - h[i] * (2.0 * M[i] + M[i + 1]) / 6.0
    d1[n - 1] = (y[n - 1] - y[n - 2]) / h[n - 2] + h[n - 2] * (M[n - 2] + 2.0 * M[n - 1]) / 6.0
    return d1, M


def curvature_at_knots(X, Y):
    """Curvature of the arclength-parameterised spline curve at the knots.

    Returns (kappa, keep): kappa for the kept points and the indices kept.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    steps = np.hypot(np.diff(X), np.diff(Y))
    total = steps.sum()
    keep = [0]
    t = [0.0]
    acc = 0.0
    for k in range(1, X.size):
        acc += steps[k - 1]
        if acc - t[-1] <= 1e-12 * total:
            continue
        keep.append(k)
        t.append(acc)
    keep = np.array(keep)
    t = np.array(t)
    if keep.size < 4:
        return None, keep
    x1, x2 = knot_derivatives(t, X[keep])
    y1, y2 = knot_derivatives(t, Y[keep])
    kappa = np.abs(x1 * y2 - y1 * x2) / (x1 * x1 + y1 * y1) ** 1.5
    return kappa, keep


def corner(reg, chi2):
    """Index k* of maximum curvature on the log-log L-curve, and kappa[N].

    Returns (k_star, kappa) with kappa = NaN at dropped points; k_star = -1
    when fewer than 4 distinct finite points exist.
    """
    reg = np.asarray(reg, dtype=np.float64)
    chi2 = np.asarray(chi2, dtype=np.float64)
    n = reg.size
    kap_full = np.full(n, np.nan)
    if n < 4 or not (np.all(reg > 0) and np.all(chi2 > 0)):
        return -1, kap_full
    X = np.log10(reg)
    Y = np.log10(chi2)
    kappa, keep = curvature_at_knots(X, Y)
    if kappa is None:
        return -1, kap_full
    kap_full[keep] = kappa
    best = 0
    for j in range(1, kappa.size):
        if kappa[j] > kappa[best] * (1.0 + 1e-12):
            best = j
    return int(keep[best]), kap_full


def corner_set(reg, chi2, rel=1e-5, draws=64, seed=12345):
    """Indices that are the corner of the curve for some small perturbation.

    The corner is a discrete argmax, so two knots of nearly equal curvature
    make it unstable.  Returns the set of corners of the unperturbed points
    and of ``draws`` seeded copies whose reg and chi^2 are scaled by
    independent factors 1 + rel * N(0, 1) (rel 1e-5 is the FP32 path's chi^2
    tolerance).  For a well-separated maximum the set is one index.
    """
    reg = np.asarray(reg, dtype=np.float64)
    chi2 = np.asarray(chi2, dtype=np.float64)
    rng = np.random.default_rng(seed)
    ks = {corner(reg, chi2)[0]}
    for _ in range(draws):
        ks.add(corner(reg * (1 + rel * rng.standard_normal(reg.size)),
                      chi2 * (1 + rel * rng.standard_normal(chi2.size)))[0])
    return ks
