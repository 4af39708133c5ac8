"""One generation of the simplified Ferret GA (FP64 oracle).

Paper (Sec. 3.1.1 and App. A.1): real-valued genes; the population is
duplicated before mutation and crossover; X-type crossover moves an
individual along the line towards a partner by a fraction drawn from a
Gaussian of standard deviation XOver.strength (0.25) with crossover
probability 1; mutation perturbs a gene with probability PMutate (0.05) by a
Gaussian step of scale mutation.scale (0.25); binary tournament selection
pits each modified individual against one unmodified individual and the
lower fitness survives.

Readings: genes live in the unit box (the prior box mapped to [0, 1]); the
crossover fraction is |xi| * strength with xi ~ N(0, 1); the two angle genes
(PA and shear angle, indices 2 and 4) wrap modulo the box, the others are
clipped to it; a tie in the tournament keeps the unmodified individual.
Linkage learning, niching, adaptive control and islands are not modelled.
All random numbers are inputs (one generation's slice of the draws).
"""
from __future__ import annotations

import numpy as np

PERIODIC = (2, 4)


def offspring(X, draws, xstrength=0.25, pmutate=0.05, mscale=0.25):
    """Offspring of unit-box population X (P, 7) from one generation's draws."""
    X = np.asarray(X, dtype=np.float64)
    P = X.shape[0]
    partner = draws["partner"]
    frac = np.abs(draws["xstrength"]) * xstrength
    Y = X + frac[:, None] * (X[partner] - X)
    mut = draws["mut_mask"] < pmutate
    Y = Y + np.where(mut, mscale * draws["mut_step"], 0.0)
    for g in range(7):
        if g in PERIODIC:
            Y[:, g] = np.mod(Y[:, g], 1.0)
        else:
            Y[:, g] = np.clip(Y[:, g], 0.0, 1.0)
    assert Y.shape == (P, 7)
    return Y


def tournament(X, fX, Y, fY, perm):
    """Offspring perm[i] competes with parent i; strictly lower fitness wins."""
    Yp = Y[perm]
    fYp = fY[perm]
    win = fYp < fX
    Xn = np.where(win[:, None], Yp, X)
    fn = np.where(win, fYp, fX)
    return Xn, fn
