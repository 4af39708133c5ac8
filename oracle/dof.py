"""Monte Carlo estimate of the effective degrees of freedom (FP64 oracle).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the GPU library
never imports it.

Paper (Sec. 2.5): the regularised solution is a filtered SVD expansion, and
the sum of its filter factors is the number of effective source degrees of
freedom; for Tikhonov regularisation gamma = sum_i mu_i / (mu_i + lambda)
(Eq. 19).  For iterative solvers the filter factors are not available, so a
zero-mean, unit-variance Gaussian vector bhat with as many elements as the
data vector is carried along: while CG solves the data system, a second
system with right-hand side built from bhat is advanced with the *same* CG
coefficients (alpha_k, beta_k) to give xhat, and bhat^T (bhat - A xhat)
estimates the degrees of freedom that remain for the residual, which turns
chi^2 into a reduced chi^2.

Reading (the paper states the scheme for CGLS on A x = b; here the data
system is the regularised normal equations of Eq. 7 with A = B L):
    data:   (A^T A + lambda H^T H) s = A^T d      CG from s = 0
    second: (A^T A + lambda H^T H) x = A^T bhat   same alpha_k, beta_k, from x = 0
    nu = bhat^T (bhat - A xhat)                   after the data system stops
    chi^2_r = chi^2 / nu
At convergence xhat = (A^T A + lambda H^T H)^-1 A^T bhat, so the expectation
of bhat^T A xhat over bhat is the trace of the influence matrix, which is
gamma of Eq. 19 for H = I; E[nu] = J - gamma.
"""
from __future__ import annotations

import numpy as np

from .solve import ST_BREAKDOWN, ST_EMPTY, ST_MAXIT, ST_OK, Problem


def mc_dof(pb: Problem, lam: float, bhat, tol: float = 1e-10, maxit: int | None = None,
           n_iter: int | None = None):
    """CG on the data system with the bhat system advanced in lockstep.

    Stops on the data system's rule ||r|| <= tol ||b|| (or after exactly
    ``n_iter`` iterations when given, the fixed-iteration form).  Returns a
    dict with the data solution ``s``, the second solution ``xhat``, the
    estimate ``nu`` = bhat^T (bhat - A xhat), ``gamma`` = bhat^T A xhat,
    ``iters``, ``status`` and the coefficient history ``alpha``, ``beta``.
    """
    I = pb.I
    bhat = np.asarray(bhat, dtype=np.float64).reshape(pb.ny, pb.nx)
    maxit = max(10 * I, 2000) if maxit is None else maxit
    b = pb.rhs()
    bh = pb.FT(bhat)
    bnorm = float(np.sqrt(b @ b))
    s = np.zeros(I)
    xh = np.zeros(I)
    alphas, betas = [], []
    status = ST_MAXIT
    it = 0
    if bnorm == 0.0:
        status = ST_EMPTY
    else:
        r, p = b.copy(), b.copy()
        rh, ph = bh.copy(), bh.copy()
        rr = float(r @ r)
        limit = n_iter if n_iter is not None else maxit
        for it in range(limit):
            if n_iter is None and np.sqrt(rr) <= tol * bnorm:
                status = ST_OK
                break
            q = pb.normal(p, lam)
            qh = pb.normal(ph, lam)
            pq = float(p @ q)
            if not pq > 0.0:
                status = ST_BREAKDOWN
                break
            alpha = rr / pq
            s += alpha * p
            r -= alpha * q
            xh += alpha * ph
            rh -= alpha * qh
            rr_new = float(r @ r)
            beta = rr_new / rr
            p = r + beta * p
            ph = rh + beta * ph
            rr = rr_new
            alphas.append(alpha)
            betas.append(beta)
        else:
            it = limit
            if n_iter is not None or np.sqrt(rr) <= tol * bnorm:
                status = ST_OK
    axh = pb.F(xh)
    nu = float((bhat * (bhat - axh)).sum())
    return dict(s=s, xhat=xh, nu=nu, gamma=float((bhat * axh).sum()), iters=it, status=status,
                alpha=np.array(alphas), beta=np.array(betas))


def mc_dof_solve(pb: Problem, lam: float, bhat, tol: float = 1e-10, maxit: int | None = None):
    """The same estimate with the second system solved by its own CG.

    xhat = (A^T A + lambda H^T H)^-1 A^T bhat to the stopping rule
    ||r|| <= tol ||A^T bhat|| (CG from zero, ``solve.solve_cg``), then
    nu = bhat^T (bhat - A xhat).  For the Tikhonov filter this has the same
    target as the lockstep form, the trace gamma of the influence matrix
    (Eq. 19 for H = I), and the two agree once both systems have converged.
    """
    bhat = np.asarray(bhat, dtype=np.float64).reshape(pb.ny, pb.nx)
    from .solve import solve_cg
    xh, it, st = solve_cg(pb, lam, tol=tol, maxit=maxit, b=pb.FT(bhat))
    axh = pb.F(xh)
    return dict(xhat=xh, nu=float((bhat * (bhat - axh)).sum()), gamma=float((bhat * axh).sum()), iters=it,
                status=st)
