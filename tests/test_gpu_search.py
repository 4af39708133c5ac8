"""GA driver with the device solve as fitness, and the surrogate-screened variant.

Data: the c2 mock image (128x128, 15x15 PSF, curvature H, 16 lambdas); every
member uses a 32x32 source grid so that a generation solves in milliseconds.
"""
import os

import numpy as np
import pytest
import torch

import synthgen

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEV = "cuda"


def _fitness(ns=32):
    import paper_1101_5803_amd as sl
    from paper_1101_5803_amd import search
    w = synthgen.C2
    z = np.load(os.path.join(ROOT, "tests", "data", "c2.npz"))
    solver = sl.Solver(torch.tensor(z["d"], device=DEV), float(z["sigma"]), torch.tensor(z["psf"], device=DEV),
                       sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width, reg=w.reg, dtype=torch.float32)
    box = search.Box(synthgen.PRIOR_LO, synthgen.PRIOR_HI)
    return search.SolverFitness(solver, box, ns, w.lambdas, tol=w.tol), solver, box, w


def test_fitness_is_corner_chi2_and_deterministic():
    fit, solver, box, w = _fitness()
    U = np.random.default_rng(1).uniform(size=(40, 7))
    f1 = fit(U)
    f2 = fit(U)
    assert np.array_equal(f1, f2)
    lens = torch.tensor(box.to_phys(U), device=DEV)
    ns = torch.full((40,), 32, dtype=torch.int32, device=DEV)
    out = solver.solve_semilinear(lens, ns, w.lambdas, tol=w.tol, max_ns=32)
    chi2 = out["chi2"].cpu().numpy()
    k = out["k_star"].cpu().numpy()
    for m in range(40):
        if k[m] >= 0:
            assert f1[m] == chi2[m, k[m]]
        else:
            assert np.isinf(f1[m])
    assert np.isfinite(f1).sum() >= 30
    assert fit.evals == 80


def test_plain_ga_improves_monotonically():
    from paper_1101_5803_amd import search
    fit, *_ = _fitness()
    P, G = 64, 5
    X0 = np.random.default_rng(2).uniform(size=(P, 7))
    dr = synthgen.ga_draws(3, P, G)
    s = search.GeneticSearch(fit, X0)
    for g in range(G):
        s.step({k: v[g] for k, v in dr.items()})
    h = np.array(s.history)
    assert np.all(np.diff(h) <= 0)
    assert h[-1] < h[0]
    assert s.full_solves == fit.evals == P * (G + 1)


def test_screened_ga_resume_exact(tmp_path):
    from paper_1101_5803_amd import search
    fit, *_ = _fitness()
    P, F, G = 32, 4, 3
    X0 = np.random.default_rng(4).uniform(size=(P, 7))
    dr = synthgen.ga_draws(5, P * F, G)
    gen = lambda g: {k: v[g] for k, v in dr.items()}  # noqa: E731
    one = search.ScreenedSearch(fit, X0, search.Surrogate(DEV, seed=9), fanout=F, train_steps=10, pretrain_steps=20)
    for g in range(G):
        one.step(gen(g))
    two = search.ScreenedSearch(fit, X0, search.Surrogate(DEV, seed=9), fanout=F, train_steps=10, pretrain_steps=20)
    two.step(gen(0))
    path = str(tmp_path / "screened.npz")
    two.save(path)
    three = search.ScreenedSearch.resume(path, fit, surrogate=search.Surrogate(DEV, seed=123))
    for g in range(1, G):
        three.step(gen(g))
    assert np.array_equal(one.X, three.X) and np.array_equal(one.fX, three.fX)
    assert torch.equal(one.surrogate.params, three.surrogate.params)
    assert one.full_solves == three.full_solves == P * (G + 1)
    assert np.all(np.diff(one.history) <= 0)
