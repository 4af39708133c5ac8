"""Pins of the source-refinement oracle (Sec. 3.2, Sec. 4).

* The windows of Sec. 3.2 on hand-worked nodes, and the full box of Sec. 4.
* The D-gene generation agrees with the seven-gene GA oracle on genes that
  the latter does not wrap (the same operators).
* On a tiny bounded least-squares problem (dense operator) the search brings
  chi^2 most of the way from the start to the optimum that scipy's bounded
  least-squares solver finds within the same bounds, and never leaves them.
"""
import numpy as np
import pytest
from scipy.optimize import lsq_linear

import synthgen
from oracle import ga, mock, refine, solve


def test_windows_by_hand():
    lo, hi = refine.windows([2.0, 0.0, -1.0, 0.4])
    assert np.allclose(lo, [1.5, 0.0, 0.0, 0.3]) and np.allclose(hi, [2.5, 0.0, 1.15, 0.5])
    lo, hi = refine.full_box([2.0, -1.0, 0.5])
    assert np.allclose(lo, 0.0) and np.allclose(hi, 2.2)
    u = refine.start_genes([2.0, 0.0, -1.0], *refine.windows([2.0, 0.0, -1.0]))
    assert np.allclose(u, [0.5, 0.0, 0.0])


def test_generation_matches_the_lens_ga():
    d = synthgen.ga_draws(7, 12, 1, dims=7)
    dg = {k: v[0] for k, v in d.items()}
    X = np.random.default_rng(1).uniform(size=(12, 7))
    a = refine.offspring(X, dg)
    b = ga.offspring(X, dg)
    keep = [g for g in range(7) if g not in ga.PERIODIC]
    assert np.allclose(a[:, keep], b[:, keep], rtol=0, atol=1e-15)


def test_search_approaches_the_bounded_optimum():
    nx = ny = 14
    psf = mock.gaussian_psf(5, 1.5)
    rng = np.random.default_rng(3)
    lens = np.array([0.25, 0.8, 0.3, 0.02, 0.2, 0.01, -0.01])
    pb0 = solve.Problem(lens, np.zeros((ny, nx)), 0.05, psf, nx, ny, 0.08, 2, 5, 0.3, "identity")
    A = pb0.dense_F()
    s_true = rng.uniform(0.2, 1.0, A.shape[1])
    d = (A @ s_true + 0.02 * rng.standard_normal(A.shape[0])).reshape(ny, nx)
    pb = solve.Problem(lens, d, 0.05, psf, nx, ny, 0.08, 2, 5, 0.3, "identity")
    s_star = solve.solve_cg(pb, 1e-2, tol=1e-12)[0]
    lo, hi = refine.windows(s_star)
    opt = lsq_linear(A / 0.05, d.reshape(-1) / 0.05, bounds=(lo, np.maximum(hi, lo + 1e-300)))
    chi_opt = float(np.sum((A @ opt.x - d.reshape(-1)) ** 2)) / 0.05 ** 2
    fit = lambda S: np.array([pb.chi2(s) for s in S])   # noqa: E731
    P, G = 40, 150
    X0 = np.random.default_rng(4).uniform(size=(P, s_star.size))
    X0[0] = refine.start_genes(s_star, lo, hi)
    r = refine.run(fit, X0, lo, hi, synthgen.ga_draws(8, P, G, dims=s_star.size), G)
    h = r["history"]
    assert np.all(np.diff(h) <= 0)
    assert h[-1] - chi_opt < 0.5 * (h[0] - chi_opt), (h[0], h[-1], chi_opt)
    S = refine.to_phys(r["X"], lo, hi)
    assert np.all(S >= lo - 1e-12) and np.all(S <= hi + 1e-12)
