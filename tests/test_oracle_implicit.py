"""Pins of the oracle's implicit regularisation by iteration count (Sec. 2.4, Sec. 2.6).

* Each CGLS iterate s_k is the least-squares minimiser of ||A s - d|| over the
  Krylov space K_k(A^T A, A^T d) (the defining property of CG applied to the
  normal equations), computed here from explicit matrices with an
  orthonormal Krylov basis.
* chi^2 of the iterates does not increase and ||s_k|| does not decrease
  (Hestenes and Stiefel's monotonicity of the CG iterate norm from zero).
* Run long enough on a tiny full-rank problem, the iterates reach the
  unregularised least-squares solution (in exact arithmetic after as many
  iterations as unknowns; in floating point CG needs some more).
"""
import numpy as np
import pytest

from oracle import implicit, mock, solve


def _tiny(ns=5, seed=0):
    nx = ny = 12
    psf = mock.gaussian_psf(5, 1.2)
    rng = np.random.default_rng(seed)
    d = rng.uniform(0, 1, (ny, nx))
    return solve.Problem(np.array([0.2, 0.7, 0.4, 0.03, 0.2, 0.02, -0.01]), d, 0.1, psf, nx, ny, 0.08, 2, ns, 0.3,
                         "identity")


def test_iterates_minimise_over_krylov_spaces():
    pb = _tiny()
    A = pb.dense_F()
    d = pb.d.reshape(-1)
    it = implicit.cgls_iterates(pb, 8)
    AtA = A.T @ A
    v = A.T @ d
    basis = []
    for k in range(1, 9):
        basis.append(v)
        v = AtA @ v
        Q, _ = np.linalg.qr(np.stack(basis, axis=1))
        c, *_ = np.linalg.lstsq(A @ Q, d, rcond=None)
        s_k = Q @ c
        assert np.linalg.norm(it["s"][k - 1] - s_k) <= 1e-7 * np.linalg.norm(s_k), k
        r = A @ s_k - d
        assert abs(it["chi2"][k - 1] - (r @ r) / pb.sigma ** 2) <= 1e-9 * it["chi2"][k - 1]
        assert abs(it["reg"][k - 1] - s_k @ s_k) <= 1e-7 * (s_k @ s_k)


def test_monotone_chi2_and_norm():
    pb = _tiny(ns=7, seed=3)
    it = implicit.cgls_iterates(pb, 30)
    assert np.all(np.diff(it["chi2"]) <= 1e-12 * it["chi2"][:-1])
    assert np.all(np.diff(it["reg"]) >= -1e-12 * it["reg"][1:])


def test_full_krylov_space_gives_least_squares():
    pb = _tiny(ns=4)
    A = pb.dense_F()
    assert np.linalg.matrix_rank(A) == pb.I
    it = implicit.cgls_iterates(pb, 4 * pb.I)
    s_ls, *_ = np.linalg.lstsq(A, pb.d.reshape(-1), rcond=None)
    assert np.linalg.norm(it["s"][-1] - s_ls) <= 1e-6 * np.linalg.norm(s_ls)


def test_fitness_is_chi2_at_the_corner():
    pb = _tiny(ns=7, seed=5)
    f = implicit.implicit_fitness(pb, 25)
    assert 0 <= f["k_star"] < 25
    assert f["fitness"] == pytest.approx(pb.chi2(f["s"][f["k_star"]]), rel=1e-12)


def test_carried_residual_and_identity_hook():
    """The carried residual's chi^2 equals the explicit one, and an identity
    perturbation hook leaves every iterate unchanged."""
    pb = _tiny(ns=6, seed=2)
    a = implicit.cgls_iterates(pb, 20)
    b = implicit.cgls_iterates(pb, 20, perturb=lambda x, kind: x)
    assert np.array_equal(a["s"], b["s"]) and np.array_equal(a["chi2"], b["chi2"])
    assert np.all(np.abs(a["chi2_e"] - a["chi2"]) <= 1e-9 * a["chi2"])


def test_rounding_spread_grows_from_rounding_level():
    """Monte Carlo arithmetic at FP64 unit roundoff moves the first iterates
    only at rounding level; the spread is what the parity tests scale."""
    pb = _tiny(ns=7, seed=4)
    ref = implicit.cgls_iterates(pb, 6)
    rng = np.random.default_rng(1)
    run = implicit.cgls_iterates(pb, 6, perturb=lambda x, kind: x * (1 + 2.0 ** -53 * rng.standard_normal(np.shape(x))))
    assert np.all(np.abs(run["chi2"][:3] - ref["chi2"][:3]) <= 1e-12 * ref["chi2"][:3])
    assert not np.array_equal(run["s"], ref["s"])


def test_lockstep_dof_matches_ritz_filter_factors():
    """Sec. 2.5 in the iterative form: the second system advanced with the data
    system's CGLS step lengths applies the data system's k-step filter to bhat,
    so bhat^T (bhat - A xhat_k) = ||bhat||^2 - sum_i f_i (u_i^T bhat)^2 with
    the CGLS filter factors f_i = 1 - prod_j (1 - sigma_i^2 / theta_j), theta_j
    the Ritz values of A^T A on K_k(A^T A, A^T d) (Hansen, Rank-Deficient and
    Discrete Ill-Posed Problems, 1998, Sec. 6.3), from a dense SVD."""
    pb = _tiny(ns=5, seed=7)
    A = pb.dense_F()
    d = pb.d.reshape(-1)
    bhat = np.random.default_rng(11).standard_normal(pb.d.shape)
    n = 6
    it = implicit.cgls_iterates(pb, n)
    got = implicit.lockstep_dof(pb, bhat, it["alpha"], it["beta"], n)
    U, sv, _ = np.linalg.svd(A, full_matrices=False)
    ub = U.T @ bhat.reshape(-1)
    AtA = A.T @ A
    basis, v = [], A.T @ d
    for k in range(1, n + 1):
        basis.append(v)
        v = AtA @ v
        Q, _ = np.linalg.qr(np.stack(basis, axis=1))
        theta = np.linalg.eigvalsh(Q.T @ AtA @ Q)
        f = 1.0 - np.prod(1.0 - sv[:, None] ** 2 / theta[None, :], axis=1)
        want = bhat.reshape(-1) @ bhat.reshape(-1) - np.sum(f * ub ** 2)
        assert abs(got[k - 1] - want) <= 1e-7 * abs(want), (k, got[k - 1], want)


def test_lockstep_dof_mean_is_trace():
    """The estimate is unbiased: over draws its mean approaches
    m - sum_i f_i, the trace of I - A X_k (Girard; Hutchinson)."""
    pb = _tiny(ns=4, seed=8)
    it = implicit.cgls_iterates(pb, 3)
    A = pb.dense_F()
    rng = np.random.default_rng(12)
    vals = [implicit.lockstep_dof(pb, rng.standard_normal(pb.d.shape), it["alpha"], it["beta"], 3)[-1]
            for _ in range(400)]
    # the estimate is the quadratic form of I - A X_k, so its values on the
    # unit vectors are the diagonal of that matrix
    m = A.shape[0]
    tr = sum(implicit.lockstep_dof(pb, np.eye(m)[j].reshape(pb.d.shape), it["alpha"], it["beta"], 3)[-1]
             for j in range(m))
    assert abs(np.mean(vals) - tr) <= 4 * np.std(vals) / np.sqrt(len(vals)), (np.mean(vals), tr)
