"""Source refinement by a bounded genetic search over the source nodes (FP64 oracle).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the GPU library
never imports it.

Paper (Sec. 3.2, Sec. 4): with the best lens held fixed, every source node
is a free parameter of a bounded global search whose fitness is the image
chi^2 of the source (Eq. 4); the bounds keep the source non-negative.  Two
kinds of bounds are described: [0, 1.1 max s] for every node, or a window
about the optimally regularised solution s* of the iterative solve:
+-25 % of |s*_i| for a node with s*_i >= 0, and [0, |s*_i| + 15 %] for a node
with s*_i < 0.  The optimiser may start from a user-supplied solution in its
first generation.

Readings: the genes are unit coordinates u in [0, 1] per node, s = lo + u
(hi - lo); the generation is the simplified Ferret GA of oracle/ga.py over D
genes, none of them periodic, every gene clipped to [0, 1]; the first
generation holds the window's image of s* (its unit coordinates, clipped) as
individual 0.  All random numbers are inputs.
"""
from __future__ import annotations

import numpy as np


def windows(s_star, tol: float = 0.25, neg_up: float = 0.15):
    """Per-node bounds (lo, hi) about s* (Sec. 3.2)."""
    s = np.asarray(s_star, dtype=np.float64)
    lo = np.empty_like(s)
    hi = np.empty_like(s)
    for i in range(s.size):
        if s[i] >= 0.0:
            lo[i] = (1.0 - tol) * s[i]
            hi[i] = (1.0 + tol) * s[i]
        else:
            lo[i] = 0.0
            hi[i] = (1.0 + neg_up) * abs(s[i])
    return lo, hi


def full_box(s_star, factor: float = 1.1):
    """[0, factor * max s*] for every node (Sec. 4)."""
    s = np.asarray(s_star, dtype=np.float64)
    return np.zeros_like(s), np.full_like(s, factor * s.max())


def to_phys(U, lo, hi):
    return np.asarray(lo) + np.asarray(U) * (np.asarray(hi) - np.asarray(lo))


def start_genes(s_star, lo, hi):
    """Unit coordinates of s* inside its bounds (0 where the bound is empty)."""
    s = np.asarray(s_star, dtype=np.float64)
    u = np.zeros_like(s)
    for i in range(s.size):
        span = hi[i] - lo[i]
        u[i] = min(max((s[i] - lo[i]) / span, 0.0), 1.0) if span > 0.0 else 0.0
    return u


def offspring(X, draws, xstrength=0.25, pmutate=0.05, mscale=0.25):
    """One generation's offspring of unit-gene population X (P, D), no periodic genes."""
    X = np.asarray(X, dtype=np.float64)
    P, D = X.shape
    Y = np.empty_like(X)
    for i in range(P):
        frac = abs(draws["xstrength"][i]) * xstrength
        j = draws["partner"][i]
        for g in range(D):
            y = X[i, g] + frac * (X[j, g] - X[i, g])
            if draws["mut_mask"][i, g] < pmutate:
                y += mscale * draws["mut_step"][i, g]
            Y[i, g] = min(max(y, 0.0), 1.0)
    return Y


def run(fitness, X0, lo, hi, draws, gens: int):
    """The bounded GA for `gens` generations.  fitness maps physical sources
    (n, D) to n values.  Returns dict(X, fX, history, evals)."""
    from .ga import tournament
    X = np.array(X0, dtype=np.float64)
    fX = np.asarray(fitness(to_phys(X, lo, hi)), dtype=np.float64)
    history = [fX.min()]
    evals = X.shape[0]
    for g in range(gens):
        dg = {k: v[g] for k, v in draws.items()}
        Y = offspring(X, dg)
        fY = np.asarray(fitness(to_phys(Y, lo, hi)), dtype=np.float64)
        evals += Y.shape[0]
        X, fX = tournament(X, fX, Y, fY, dg["perm"])
        history.append(fX.min())
    return dict(X=X, fX=fX, history=np.array(history), evals=evals)
