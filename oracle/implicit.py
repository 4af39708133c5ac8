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
"""
from __future__ import annotations

import numpy as np

from . import lcurve
from .solve import Problem


def cgls_iterates(pb: Problem, n_iter: int):
    """The first n_iter CGLS iterates of the unregularised problem.

    Returns dict(s=(n_iter, I) iterates s_1..s_n, chi2=(n_iter,), reg=(n_iter,)
    with reg = sum s^2, and the per-iteration alpha, beta).  Stops early (the
    remaining rows repeat the last iterate) when ||A^T e|| or ||A p|| is zero.
    """
    I = pb.I
    s = np.zeros(I)
    e = pb.d.astype(np.float64).copy()
    g = pb.FT(e)
    p = g.copy()
    gg = float(g @ g)
    out_s = np.zeros((n_iter, I))
    chi2 = np.zeros(n_iter)
    reg = np.zeros(n_iter)
    alphas, betas = [], []
    done = gg == 0.0
    for k in range(n_iter):
        if not done:
            q = pb.F(p)
            qq = float((q * q).sum())
            if qq > 0.0:
                alpha = gg / qq
                s = s + alpha * p
                e = e - alpha * q
                g = pb.FT(e)
                gg_new = float(g @ g)
                beta = gg_new / gg
                p = g + beta * p
                gg = gg_new
                alphas.append(alpha)
                betas.append(beta)
                done = gg == 0.0
            else:
                done = True
        out_s[k] = s
        chi2[k] = pb.chi2(s)
        reg[k] = float(s @ s)
    return dict(s=out_s, chi2=chi2, reg=reg, alpha=np.array(alphas), beta=np.array(betas))


def implicit_fitness(pb: Problem, n_iter: int = 40):
    """Corner of the L-curve over the iterates and chi^2 there (Sec. 2.6, Sec. 3).

    Returns the iterates of cgls_iterates plus k_star (index into them),
    fitness = chi^2 of iterate k_star, and the knot curvatures."""
    it = cgls_iterates(pb, n_iter)
    k, kappa = lcurve.corner(it["reg"], it["chi2"])
    return dict(k_star=k, fitness=float(it["chi2"][k]) if k >= 0 else float("inf"), kappa=kappa, **it)
