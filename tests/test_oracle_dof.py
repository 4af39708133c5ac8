"""Pins of the oracle's Monte Carlo degrees of freedom (Sec. 2.5, Eq. 19).

* Converged: the lockstep solution xhat equals the exact solution of the
  normal equations with right-hand side A^T bhat (dense Cholesky), and nu
  equals bhat^T (I - A M^-1 A^T) bhat computed from explicit matrices.
* Stopped early (fixed iteration count, where "the same coefficients"
  matters): xhat equals the CG filter applied to A^T bhat through the
  eigen-decomposition of M, with the filter 1 - R_k(mu) whose roots are the
  Ritz values (the eigenvalues of the Lanczos tridiagonal matrix that CG's
  alpha and beta define).  Advancing the second system with its own
  coefficients would give a different polynomial and fail.
* Statistical: over seeded draws of bhat, the mean of nu is J - gamma with
  gamma = sum mu/(mu + lambda) from the eigenvalues (Eq. 19), within four
  standard errors of the Gaussian trace estimator (variance 2 tr(S^2)).
"""
import numpy as np
import pytest

from oracle import dof, mock, solve


def _tiny(reg, ns=6, seed=0):
    nx = ny = 12
    psf = mock.gaussian_psf(5, 1.5)
    rng = np.random.default_rng(seed)
    d = rng.uniform(0, 1, (ny, nx))
    return solve.Problem(np.array([0.2, 0.7, 0.4, 0.03, 0.2, 0.02, -0.01]), d, 0.1, psf, nx, ny, 0.08, 2, ns, 0.3,
                         reg)


@pytest.mark.parametrize("reg", ["identity", "curvature"])
def test_converged_lockstep_is_the_exact_second_solve(reg):
    pb = _tiny(reg)
    Fm = pb.dense_F()
    G = pb.dense_HtH()
    bhat = np.random.default_rng(3).standard_normal((pb.ny, pb.nx))
    for lam in (1e-2, 1.0):
        out = dof.mc_dof(pb, lam, bhat, tol=1e-14, maxit=2000)
        Mm = Fm.T @ Fm + lam * G
        x = np.linalg.solve(Mm, Fm.T @ bhat.reshape(-1))
        assert np.linalg.norm(out["xhat"] - x) <= 1e-8 * np.linalg.norm(x), lam
        nu = float(bhat.reshape(-1) @ (bhat.reshape(-1) - Fm @ x))
        assert abs(out["nu"] - nu) <= 1e-8 * abs(nu)
        assert abs(out["gamma"] + out["nu"] - (bhat ** 2).sum()) <= 1e-9 * (bhat ** 2).sum()
        # the data system is the ordinary CG solve
        s_c, it, st = solve.solve_cg(pb, lam, tol=1e-14, maxit=2000)
        assert out["iters"] == it and np.array_equal(out["s"], s_c)


@pytest.mark.parametrize("k", [3, 6])
def test_fixed_iterations_follow_the_data_polynomial(k):
    pb = _tiny("curvature")
    lam = 1e-3
    Fm = pb.dense_F()
    Mm = Fm.T @ Fm + lam * pb.dense_HtH()
    bhat = np.random.default_rng(4).standard_normal((pb.ny, pb.nx))
    out = dof.mc_dof(pb, lam, bhat, n_iter=k)
    a, b = out["alpha"], out["beta"]
    assert a.size == k
    # Lanczos tridiagonal of the k CG steps: T[0,0] = 1/a0, T[j,j] = 1/a_j + b_{j-1}/a_{j-1},
    # T[j,j-1] = T[j-1,j] = sqrt(b_{j-1})/a_{j-1}
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / a[j] + (b[j - 1] / a[j - 1] if j else 0.0)
        if j:
            T[j, j - 1] = T[j - 1, j] = np.sqrt(b[j - 1]) / a[j - 1]
    theta = np.linalg.eigvalsh(T)
    mu, V = np.linalg.eigh(Mm)
    R = np.prod(1.0 - mu[:, None] / theta[None, :], axis=1)   # CG residual polynomial at the eigenvalues
    x = V @ (((1.0 - R) / mu) * (V.T @ (Fm.T @ bhat.reshape(-1))))
    assert np.linalg.norm(out["xhat"] - x) <= 1e-8 * np.linalg.norm(x)
    # the exact second solve is a different vector at this k
    x_exact = np.linalg.solve(Mm, Fm.T @ bhat.reshape(-1))
    assert np.linalg.norm(out["xhat"] - x_exact) > 1e-3 * np.linalg.norm(x_exact)


def test_mean_matches_eq19_gamma():
    pb = _tiny("identity")
    Fm = pb.dense_F()
    lam = 0.05
    J = pb.nx * pb.ny
    gamma = solve.dof_gamma(Fm, lam)
    S = Fm @ np.linalg.solve(Fm.T @ Fm + lam * np.eye(pb.I), Fm.T)
    rng = np.random.default_rng(11)
    n = 300
    nus = [dof.mc_dof(pb, lam, rng.standard_normal((pb.ny, pb.nx)), tol=1e-12)["nu"] for _ in range(n)]
    se = np.sqrt(2.0 * np.trace(S @ S) / n)
    assert abs(np.mean(nus) - (J - gamma)) <= 4 * se, (np.mean(nus), J - gamma, se)


@pytest.mark.parametrize("reg", ["identity", "curvature"])
def test_independent_solve_form(reg):
    """mc_dof_solve: converged, it equals the dense second solve and the converged lockstep form."""
    pb = _tiny(reg)
    Fm = pb.dense_F()
    bhat = np.random.default_rng(7).standard_normal((pb.ny, pb.nx))
    lam = 3e-2
    ind = dof.mc_dof_solve(pb, lam, bhat, tol=1e-14, maxit=2000)
    x = np.linalg.solve(Fm.T @ Fm + lam * pb.dense_HtH(), Fm.T @ bhat.reshape(-1))
    assert np.linalg.norm(ind["xhat"] - x) <= 1e-8 * np.linalg.norm(x)
    lock = dof.mc_dof(pb, lam, bhat, tol=1e-14, maxit=2000)
    assert abs(ind["gamma"] - lock["gamma"]) <= 1e-8 * abs(lock["gamma"])
