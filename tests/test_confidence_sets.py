"""Confidence regions from the optimal set (Sec. 3, the standard method).

* Textbook thresholds: one parameter at 68.3 % is Delta chi^2 = 1; two
  parameters at 68.3 % is 2.30 (Press et al., Numerical Recipes Sec. 15.6).
* Calibration: solutions drawn from the Gaussian posterior of a quadratic
  chi^2 surface fall inside the level-p region with frequency p.
* Rescaling: multiplying every chi^2 by a constant (a misestimated noise)
  leaves the regions unchanged once the best fit's reduced chi^2 is used.
"""
import numpy as np
import pytest

search = pytest.importorskip("paper_1101_5803_amd.search")


def test_textbook_thresholds():
    P = np.zeros((3, 1))
    r = search.confidence_sets(P, np.array([10.0, 11.0, 12.0]), dof=10.0, levels=(0.6827,))
    assert r["levels"][0.6827]["delta_chi2"] == pytest.approx(1.0, abs=2e-4)
    r = search.confidence_sets(np.zeros((3, 2)), np.array([10.0, 11.0, 12.0]), dof=10.0, levels=(0.6827,))
    assert r["levels"][0.6827]["delta_chi2"] == pytest.approx(2.30, abs=5e-3)


def test_calibration_on_a_quadratic_surface():
    rng = np.random.default_rng(0)
    k, n = 7, 20000
    C = np.diag(rng.uniform(0.5, 2.0, k))
    L = np.linalg.cholesky(C)
    theta = rng.standard_normal((n, k)) @ L.T
    dof = 1000.0
    f = dof + np.einsum("ij,jk,ik->i", theta, np.linalg.inv(C), theta)   # chi^2_min = dof: chi^2_r = 1
    P = np.vstack([np.zeros(k), theta])
    f = np.concatenate([[dof], f])
    r = search.confidence_sets(P, f, dof=dof)
    for p, lev in r["levels"].items():
        frac = lev["mask"][1:].mean()
        assert frac == pytest.approx(p, abs=0.01), (p, frac)
    assert r["optimal"].sum() >= r["levels"][0.99]["mask"].sum()


def test_rescaling_by_reduced_chi2():
    rng = np.random.default_rng(1)
    P = rng.uniform(size=(500, 3))
    f = 100.0 + 50.0 * np.sum((P - 0.5) ** 2, axis=1)
    a = search.confidence_sets(P, f, dof=100.0)
    b = search.confidence_sets(P, 1.7 * f, dof=100.0)
    for p in a["levels"]:
        assert np.array_equal(a["levels"][p]["mask"], b["levels"][p]["mask"])
