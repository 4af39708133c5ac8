"""Particle swarm over the lens parameters (FP64 oracle): Eq. 21 and Locust's exact orbits.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the GPU library
never imports it.

Paper (Sec. 3.1.2, Eq. 21; App. A.2): each particle i is pulled towards its
own best position x_p and the swarm's best position x_g by springs of
constants c_p xi_p and c_g xi_g (xi uniform on [0, 1], drawn anew each step)
and is damped over a time t_damp:
    v(t + dt) = v(t) (1 - dt / t_damp) + [c_p xi_p (x_p - x) + c_g xi_g (x_g - x)] dt
    x(t + dt) = x(t) + v(t) dt
(the position moves with the velocity of time t).  Locust instead moves each
particle along the exact solution of the same equations in the limit of
small steps, a damped harmonic oscillator over the step with the springs
held fixed.  Defaults c_p = 1, c_g = 0.5, dt = 1, TDamp = 10 (App. A.2).

Readings (the paper is silent):
* TDamp is the damping time in units of the critical one (App. A.2: 1 is
  critically damped).  With the mean spring constant k = (c_p + c_g) / 2
  (xi has mean 1/2) the oscillator is critically damped at t_damp =
  1 / (2 sqrt(k)), so t_damp = TDamp / (2 sqrt(k)).
* xi_p and xi_g are one draw per particle and step (scalars, as in Eq. 21).
* Positions live in the unit box (the prior box mapped to [0, 1]); the two
  angle genes wrap; another gene that leaves the box is put back on the wall
  and its velocity component is set to zero.
* Initial velocities are zero; the personal bests start at the initial
  positions; a particle's best changes only on a strictly lower fitness; the
  swarm's best is the lowest personal best (lowest index on a tie).
* The swarm is fully connected (the gbest topology); Locust's dynamic
  neighbourhoods are not modelled.
* The exact orbits are the default, as Locust runs them.  Eq. 21 taken
  literally (the position moving with the old velocity) has, for one
  particle with fixed springs k, the recurrence determinant
  (1 - dt / t_damp) + k dt^2, above one at these constants, so its orbits
  grow until the walls stop them (the paper's "particle explosions").
All random numbers are inputs.
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC = (2, 4)


def damping_time(tdamp: float, cp: float, cg: float) -> float:
    """t_damp of Eq. 21 for Locust's TDamp (see the readings)."""
    k = 0.5 * (cp + cg)
    return tdamp / (2.0 * math.sqrt(k))


def euler_step(x, v, xp, xg, xi_p, xi_g, cp, cg, dt, t_damp):
    """Eq. 21 for one particle (vectors x, v, x_p, x_g; scalars xi_p, xi_g)."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    pull = cp * xi_p * (np.asarray(xp) - x) + cg * xi_g * (np.asarray(xg) - x)
    v_new = v * (1.0 - dt / t_damp) + pull * dt
    x_new = x + v * dt
    return x_new, v_new


def _oscillator(y0: float, v0: float, k: float, gamma: float, t: float):
    """y'' = -gamma y' - k y from (y0, v0): (y(t), y'(t)), written out per case."""
    if k <= 0.0:
        if gamma == 0.0:
            return y0 + v0 * t, v0
        e = math.exp(-gamma * t)
        return y0 + v0 * (1.0 - e) / gamma, v0 * e
    disc = gamma * gamma - 4.0 * k
    if disc < 0.0:
        w = math.sqrt(k - 0.25 * gamma * gamma)
        e = math.exp(-0.5 * gamma * t)
        c, s = math.cos(w * t), math.sin(w * t)
        y = e * (y0 * c + (v0 + 0.5 * gamma * y0) / w * s)
        v = e * (v0 * c - (0.5 * gamma * v0 + k * y0) / w * s)
        return y, v
    if disc > 0.0:
        sq = math.sqrt(disc)
        r1, r2 = 0.5 * (-gamma + sq), 0.5 * (-gamma - sq)
        c1 = (v0 - r2 * y0) / (r1 - r2)
        c2 = y0 - c1
        e1, e2 = math.exp(r1 * t), math.exp(r2 * t)
        return c1 * e1 + c2 * e2, r1 * c1 * e1 + r2 * c2 * e2
    b = v0 + 0.5 * gamma * y0
    e = math.exp(-0.5 * gamma * t)
    return (y0 + b * t) * e, (v0 - 0.5 * gamma * b * t) * e


def exact_step(x, v, xp, xg, xi_p, xi_g, cp, cg, dt, t_damp):
    """The exact orbit over dt of x'' = -x'/t_damp + c_p xi_p (x_p - x) + c_g xi_g (x_g - x),
    component by component, with the springs held fixed over the step."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    kp, kg = cp * xi_p, cg * xi_g
    k = kp + kg
    gamma = 1.0 / t_damp
    x_new = np.empty_like(x)
    v_new = np.empty_like(v)
    for j in range(x.size):
        centre = (kp * xp[j] + kg * xg[j]) / k if k > 0.0 else 0.0
        y, vv = _oscillator(x[j] - centre, v[j], k, gamma, dt)
        x_new[j] = y + centre
        v_new[j] = vv
    return x_new, v_new


def confine(x, v):
    """Wrap the angle genes, put the others back on the walls with zero velocity there."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    for j in range(x.size):
        if j in PERIODIC:
            x[j] = x[j] % 1.0
        elif x[j] < 0.0 or x[j] > 1.0:
            x[j] = min(max(x[j], 0.0), 1.0)
            v[j] = 0.0
    return x, v


def run(fitness, x0, xi_p, xi_g, steps: int, cp: float = 1.0, cg: float = 0.5, dt: float = 1.0,
        tdamp: float = 10.0, form: str = "exact"):
    """The swarm from positions x0 (N, D) for `steps` steps, one particle at a time.

    fitness maps an (n, D) array to n values (lower is better).  xi_p, xi_g
    are (steps, N) uniform draws.  Returns dict(x, v, xp, fp, xg, fg,
    history=best fitness after the start and after every step, evals)."""
    step = euler_step if form == "euler" else exact_step
    t_damp = damping_time(tdamp, cp, cg)
    x = np.array(x0, dtype=np.float64)
    N = x.shape[0]
    v = np.zeros_like(x)
    f = np.asarray(fitness(x), dtype=np.float64)
    xp, fp = x.copy(), f.copy()
    g = int(np.argmin(fp))
    history = [fp[g]]
    evals = N
    for t in range(steps):
        for i in range(N):
            xn, vn = step(x[i], v[i], xp[i], xp[g], xi_p[t, i], xi_g[t, i], cp, cg, dt, t_damp)
            x[i], v[i] = confine(xn, vn)
        f = np.asarray(fitness(x), dtype=np.float64)
        evals += N
        for i in range(N):
            if f[i] < fp[i]:
                fp[i] = f[i]
                xp[i] = x[i]
        g = int(np.argmin(fp))
        history.append(fp[g])
    return dict(x=x, v=v, xp=xp, fp=fp, xg=xp[g].copy(), fg=fp[g], history=np.array(history), evals=evals)
