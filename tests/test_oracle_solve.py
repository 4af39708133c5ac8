"""Pins of the oracle's regularised solve (Eqs. 4-7, 13-19) and of the C oracle."""
import numpy as np
import pytest

import synthgen
from oracle import coracle, lcurve, mock, solve


def _tiny(reg="curvature", ns=6, lens_=(0.2, 0.7, 0.4, 0.03, 0.2, 0.02, -0.01), K=5, seed=0):
    nx = ny = 12
    pix = 0.08
    psf = mock.gaussian_psf(K, 1.5)
    rng = np.random.default_rng(seed)
    d = rng.uniform(0, 1, (ny, nx))
    return solve.Problem(np.array(lens_), d, 0.1, psf, nx, ny, pix, 2, ns, 0.3, reg)


@pytest.mark.parametrize("reg", ["identity", "curvature"])
def test_cg_matches_cholesky(reg):
    pb = _tiny(reg)
    for lam in (1e-3, 1e-1, 10.0):
        s_d = solve.solve_dense(pb, lam)
        s_c, it, st = solve.solve_cg(pb, lam, tol=1e-13)
        assert st == solve.ST_OK
        assert np.linalg.norm(s_c - s_d) <= 1e-9 * np.linalg.norm(s_d)


def test_matrix_free_equals_dense_operator():
    pb = _tiny()
    Fm = pb.dense_F()
    x = np.random.default_rng(1).standard_normal(pb.I)
    np.testing.assert_allclose(Fm @ x, pb.F(x).reshape(-1), atol=1e-13)
    y = np.random.default_rng(2).standard_normal(pb.nx * pb.ny)
    np.testing.assert_allclose(Fm.T @ y, pb.FT(y.reshape(pb.ny, pb.nx)), atol=1e-13)


def test_identity_svd_filter_factors():
    pb = _tiny("identity")
    Fm = pb.dense_F()
    for lam in (1e-4, 3e-2, 5.0):
        np.testing.assert_allclose(solve.tikhonov_svd(Fm, pb.d, lam), solve.solve_dense(pb, lam, Fm),
                                   rtol=1e-8, atol=1e-10)


def test_dof_equals_influence_trace():
    pb = _tiny("identity")
    Fm = pb.dense_F()
    lam = 0.05
    A = Fm @ np.linalg.solve(Fm.T @ Fm + lam * np.eye(pb.I), Fm.T)
    assert abs(np.trace(A) - solve.dof_gamma(Fm, lam)) < 1e-8
    # gamma -> rank as lambda -> 0 and -> 0 as lambda -> inf
    assert solve.dof_gamma(Fm, 1e-14) == pytest.approx(np.linalg.matrix_rank(Fm), abs=1e-3)
    assert solve.dof_gamma(Fm, 1e14) < 1e-6


def test_lambda_limits():
    pb = _tiny("curvature")
    big = solve.solve_dense(pb, 1e12)
    assert np.linalg.norm(big) < 1e-8
    assert pb.chi2(big) == pytest.approx((pb.d ** 2).sum() / pb.sigma ** 2, rel=1e-8)
    # lambda -> 0 on a full-rank system is the least-squares solution
    Fm = pb.dense_F()
    assert np.linalg.matrix_rank(Fm) == pb.I
    ls = np.linalg.lstsq(Fm, pb.d.reshape(-1), rcond=None)[0]
    np.testing.assert_allclose(solve.solve_dense(pb, 1e-12, Fm), ls, rtol=1e-5, atol=1e-7)


def test_tikhonov_monotone():
    pb = _tiny("curvature")
    lams = synthgen.log_grid(1e-4, 1e2, 12)
    out = solve.sweep(pb, lams, method="dense")
    assert np.all(np.diff(out["reg"]) <= 1e-12 * out["reg"][:-1])
    assert np.all(np.diff(out["chi2"]) >= -1e-12 * out["chi2"][:-1])


def test_empty_mapping():
    # a lens that sends every ray off the source grid: b = L^T B^T d = 0
    pb = _tiny(lens_=(5.0, 1.0, 0.0, 0.0, 0.0, 5.0, 5.0))
    assert not pb.table[2].any()
    s, it, st = solve.solve_cg(pb, 1.0)
    assert st == solve.ST_EMPTY and not s.any()


@pytest.mark.parametrize("reg", ["identity", "curvature"])
def test_c_oracle_matches_numpy(reg):
    pb = _tiny(reg)
    lams = [1e-3, 1e-1, 10.0]
    out = coracle.evaluate(pb.lens, pb.ns, pb.half_width, pb.nx, pb.ny, pb.pix, pb.nsub, pb.d, pb.sigma,
                           pb.psf, reg, lams, tol=1e-13, want_s=True, threads=1)
    ref = solve.sweep(pb, lams, method="dense")
    np.testing.assert_allclose(out["chi2"][0], ref["chi2"], rtol=1e-10)
    np.testing.assert_allclose(out["reg"][0], ref["reg"], rtol=1e-8)
    for k in range(3):
        s = out["s"][0, k]
        assert np.linalg.norm(s - ref["s"][k]) <= 1e-9 * np.linalg.norm(ref["s"][k])


def test_c1_plain_workload():
    """c1: SIS, H = I, one lambda; C oracle == numpy CG == dense, statistically sane."""
    w = synthgen.C1
    D = mock.workload_data(w)
    pb = solve.Problem(D["lens"], D["d"], D["sigma"], D["psf"], w.nx, w.ny, w.pix, w.nsub_model,
                       w.ns, w.half_width, w.reg)
    lam = w.lambdas[0]
    s_d = solve.solve_dense(pb, lam)
    s_c, it, st = solve.solve_cg(pb, lam, tol=w.tol)
    assert st == solve.ST_OK
    assert np.linalg.norm(s_c - s_d) <= 1e-8 * np.linalg.norm(s_d)
    out = coracle.evaluate(D["lens"], w.ns, w.half_width, w.nx, w.ny, w.pix, w.nsub_model, D["d"],
                           D["sigma"], D["psf"], w.reg, w.lambdas, tol=w.tol, want_s=True, threads=1)
    assert np.linalg.norm(out["s"][0, 0] - s_d) <= 1e-8 * np.linalg.norm(s_d)
    assert out["chi2"][0, 0] == pytest.approx(pb.chi2(s_d), rel=1e-10)
    # the noise-level fit at the true lens gives chi^2/J of order one
    assert 0.5 < pb.chi2(s_d) / (w.nx * w.ny) < 2.0


def test_theta_e_scan_has_interior_minimum():
    """Statistical sanity (Sec. 4, Fig. 9): corner chi^2 over a theta_E scan
    of the c1 data is smallest near the true value."""
    w = synthgen.C1
    D = mock.workload_data(w)
    lams = synthgen.log_grid(1e-4, 1e1, 8)
    thetas = [0.6, 0.7, 0.8, 0.9, 1.0]
    lens_ = np.array([[t, 1.0, 0.0, 0, 0, 0, 0] for t in thetas])
    out = coracle.evaluate(lens_, w.ns, w.half_width, w.nx, w.ny, w.pix, w.nsub_model, D["d"],
                           D["sigma"], D["psf"], "identity", lams, tol=1e-10, threads=2)
    fit = []
    for m in range(len(thetas)):
        k, _ = lcurve.corner(out["reg"][m], out["chi2"][m])
        fit.append(out["chi2"][m, k])
    best = int(np.argmin(fit))
    assert 0 < best < len(thetas) - 1 and abs(thetas[best] - 0.8) < 0.11
