"""Implicit regularisation by the iteration count (FP64 oracle).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the GPU library
never imports it.

Paper (Sec. 2.4, Sec. 2.6, Sec. 3): CGLS started from a blank source adds
components of decreasing singular value with every iteration, so the
iteration count acts as the regularisation parameter.  The fitness of a lens
runs a fixed number of CGLS iterations with no lambda, records after every
iteration the image chi^2 and the zeroth-order regularisation measure
sum_i s_i^2, forms the L-curve of those points, and takes chi^2 of the
iterate at the point of maximum curvature (Eq. 20).

CGLS on min ||A s - d|| with A = B L (Sec. 2.2: one L and one L^T, one B and
one B^T per iteration), from s = 0:
    e = d, g = A^T e, p = g
    per iteration: q = A p; alpha = ||g||^2 / ||q||^2; s += alpha p;
                   e -= alpha q; g' = A^T e; beta = ||g'||^2 / ||g||^2;
                   p = g' + beta p
chi^2 of each iterate is computed from the explicit solution, reg = ||s||^2.

Rounding model.  Past the first handful of iterations the sequence is
sensitive to rounding: CG loses orthogonality while it resolves small
singular values, so two correct implementations that round differently
drift apart.  To bound that drift the parity tests run this same routine
under Monte Carlo arithmetic (Parker, Pierce and Eggert, "Monte Carlo
arithmetic: how to gamble with floating point and win", 2000): every
computed quantity x is replaced by x (1 + delta xi) with xi a seeded standard
normal, and the spread over draws shows how far rounding at relative level
delta can move each iterate.  `perturb(x, kind)` applies that replacement;
kind is "A" or "AT" for the two operator outputs, "vec" for the updated
s, e and p, and "scalar" for alpha and beta.  With perturb=None (the
default) the routine is the plain algorithm above.
"""
from __future__ import annotations

import numpy as np

from . import lcurve
from .solve import Problem


def _same(x, kind):
    return x


def cgls_iterates(pb: Problem, n_iter: int, perturb=None):
    """The first n_iter CGLS iterates of the unregularised problem.

    Returns dict(s=(n_iter, I) iterates s_1..s_n, chi2=(n_iter,) from the
    explicit iterate, chi2_e=(n_iter,) from the carried residual e (equal in
    exact arithmetic), reg=(n_iter,) with reg = sum s^2, and the per-iteration
    alpha, beta).  Stops early (the remaining rows repeat the last iterate)
    when ||A^T e|| or ||A p|| is zero.  perturb: see the module docstring.
    """
    pt = perturb or _same
    I = pb.I
    s = np.zeros(I)
    e = pb.d.astype(np.float64).copy()
    g = pt(pb.FT(e), "AT")
    p = g.copy()
    gg = float(g @ g)
    out_s = np.zeros((n_iter, I))
    chi2 = np.zeros(n_iter)
    chi2_e = np.zeros(n_iter)
    reg = np.zeros(n_iter)
    alphas, betas = [], []
    done = gg == 0.0
    ee = float((e * e).sum())
    for k in range(n_iter):
        if not done:
            q = pt(pb.F(p), "A")
            qq = float((q * q).sum())
            if qq > 0.0:
                alpha = pt(gg / qq, "scalar")
                s = pt(s + alpha * p, "vec")
                e = pt(e - alpha * q, "vec")
                ee = float((e * e).sum())
                g = pt(pb.FT(e), "AT")
                gg_new = float(g @ g)
                beta = pt(gg_new / gg, "scalar")
                p = pt(g + beta * p, "vec")
                gg = gg_new
                alphas.append(alpha)
                betas.append(beta)
                done = gg == 0.0
            else:
                done = True
        out_s[k] = s
        chi2[k] = pb.chi2(s)
        chi2_e[k] = ee / pb.sigma ** 2
        reg[k] = float(s @ s)
    return dict(s=out_s, chi2=chi2, chi2_e=chi2_e, reg=reg, alpha=np.array(alphas), beta=np.array(betas))


def implicit_fitness(pb: Problem, n_iter: int = 40):
    """Corner of the L-curve over the iterates and chi^2 there (Sec. 2.6, Sec. 3).

    Returns the iterates of cgls_iterates plus k_star (index into them),
    fitness = chi^2 of iterate k_star, and the knot curvatures."""
    it = cgls_iterates(pb, n_iter)
    k, kappa = lcurve.corner(it["reg"], it["chi2"])
    return dict(k_star=k, fitness=float(it["chi2"][k]) if k >= 0 else float("inf"), kappa=kappa, **it)


def lockstep_dof(pb: Problem, bhat: np.ndarray, alpha, beta, n_iter: int):
    """Monte Carlo degrees of freedom along the CGLS iterates (Sec. 2.5).

    A second system with data bhat (standard normal draws, image shaped) is
    advanced with the data system's CGLS step lengths alpha_k and beta_k
    rather than its own, so that its iterate xhat_k is the data system's
    k-step filter applied to bhat.  After each iteration the estimate is
    bhat^T (bhat - A xhat_k), evaluated from the explicit xhat_k.  alpha and
    beta come from cgls_iterates; past the last recorded step (an early stop)
    the estimate repeats.  Returns (n_iter,)."""
    b = np.asarray(bhat, dtype=np.float64)
    bb = float((b * b).sum())
    xh = np.zeros(pb.I)
    eh = b.copy()
    ph = pb.FT(eh)
    out = np.full(n_iter, bb)
    for k in range(n_iter):
        if k < len(alpha):
            qh = pb.F(ph)
            xh = xh + alpha[k] * ph
            eh = eh - alpha[k] * qh
            ph = pb.FT(eh) + beta[k] * ph
            out[k] = bb - float((b * pb.F(xh)).sum())
        elif k > 0:
            out[k] = out[k - 1]
    return out
