"""The source-refinement driver (search.SourceRefinement, host logic) against
the oracle (oracle/refine.py) on the same seeded draws, with the oracle's
chi^2 as fitness: bounds, the start individual, every generation's
population and fitness, for the window and the full-box bounds."""
import numpy as np
import pytest

import synthgen
from oracle import mock, refine, solve

search = pytest.importorskip("paper_1101_5803_amd.search")


@pytest.mark.parametrize("bounds", ["window", "box"])
def test_refinement_matches_oracle(bounds):
    nx = ny = 12
    psf = mock.gaussian_psf(5, 1.5)
    rng = np.random.default_rng(5)
    d = rng.uniform(0, 1, (ny, nx))
    pb = solve.Problem(np.array([0.2, 0.7, 0.4, 0.03, 0.2, 0.02, -0.01]), d, 0.1, psf, nx, ny, 0.08, 2, 5, 0.3,
                       "identity")
    s_star = solve.solve_cg(pb, 1e-2, tol=1e-12)[0]
    lo, hi = refine.windows(s_star) if bounds == "window" else refine.full_box(s_star)
    fit = lambda S: np.array([pb.chi2(s) for s in S])   # noqa: E731
    P, G = 16, 12
    X0 = np.random.default_rng(6).uniform(size=(P, s_star.size))
    X0r = X0.copy()
    X0r[0] = refine.start_genes(s_star, lo, hi)
    draws = synthgen.ga_draws(9, P, G, dims=s_star.size)
    ref = refine.run(fit, X0r, lo, hi, draws, G)
    r = search.SourceRefinement(None, None, 5, s_star, X0, bounds=bounds, fitness=fit, n_pixels=nx * ny)
    assert np.allclose(r.lo, lo, rtol=0, atol=1e-15) and np.allclose(r.hi, hi, rtol=0, atol=1e-15)
    for g in range(G):
        r.step({k: v[g] for k, v in draws.items()})
    assert np.allclose(r.X, ref["X"], rtol=0, atol=1e-13)
    assert np.allclose(r.fX, ref["fX"], rtol=1e-13, atol=0)
    assert np.allclose(r.history, ref["history"], rtol=1e-13, atol=0)
    assert r.evals == ref["evals"]
