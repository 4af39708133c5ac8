"""Pins of the particle swarm oracle (Sec. 3.1.2, Eq. 21; App. A.2).

* Eq. 21 written out for one particle on numbers worked by hand.
* With no springs the Euler velocity decays as (1 - dt/t_damp)^n and the
  position sums it; the exact orbit then decays as exp(-t/t_damp).
* The exact orbit satisfies the oscillator equation and its initial
  conditions (finite differences), in the under-, over- and critically
  damped cases, and is the limit of Euler steps as the step shrinks.
* TDamp = 1 is critical damping at the mean spring constant.
* Personal bests never get worse; the swarm best is the lowest of them; on a
  convex bowl the swarm approaches the minimum.
"""
import math

import numpy as np
import pytest

import synthgen
from oracle import pso


def test_eq21_by_hand():
    x = np.array([0.2, 0.5]); v = np.array([0.1, -0.2])
    xp = np.array([0.4, 0.5]); xg = np.array([0.0, 1.0])
    xn, vn = pso.euler_step(x, v, xp, xg, 0.5, 0.25, 1.0, 0.5, 1.0, 10.0)
    # v' = v (1 - 1/10) + 1*0.5*(xp - x) + 0.5*0.25*(xg - x)
    assert np.allclose(vn, [0.1 * 0.9 + 0.5 * 0.2 + 0.125 * (-0.2), -0.2 * 0.9 + 0.0 + 0.125 * 0.5], rtol=0, atol=1e-15)
    assert np.allclose(xn, [0.3, 0.3], rtol=0, atol=1e-15)   # moves with the old velocity


def test_free_particle_decay():
    x = np.array([0.5]); v = np.array([0.2]); z = np.zeros(1)
    tau, dt = 4.0, 0.5
    xs, vs = x.copy(), v.copy()
    for n in range(1, 9):
        xs_prev = xs.copy(); vs_prev = vs.copy()
        xs, vs = pso.euler_step(xs, vs, z, z, 0.0, 0.0, 1.0, 0.5, dt, tau)
        assert vs[0] == pytest.approx(0.2 * (1 - dt / tau) ** n, rel=1e-14)
        assert xs[0] == pytest.approx(xs_prev[0] + vs_prev[0] * dt, rel=1e-14)
    xe, ve = pso.exact_step(x, v, z, z, 0.0, 0.0, 1.0, 0.5, 3.0, tau)
    assert ve[0] == pytest.approx(0.2 * math.exp(-3.0 / tau), rel=1e-14)
    assert xe[0] == pytest.approx(0.5 + 0.2 * tau * (1 - math.exp(-3.0 / tau)), rel=1e-14)


@pytest.mark.parametrize("k,gamma", [(1.0, 0.3), (0.1, 2.0), (0.25, 1.0)])   # under-, over-, critically damped
def test_exact_orbit_solves_the_oscillator(k, gamma):
    y0, v0 = 0.7, -0.3
    h = 1e-4
    for t in (0.3, 1.0, 2.5):
        y, v = pso._oscillator(y0, v0, k, gamma, t)
        yp, _ = pso._oscillator(y0, v0, k, gamma, t + h)
        ym, _ = pso._oscillator(y0, v0, k, gamma, t - h)
        assert (yp - ym) / (2 * h) == pytest.approx(v, rel=1e-6, abs=1e-9)
        ypp = (yp - 2 * y + ym) / (h * h)
        assert ypp == pytest.approx(-gamma * v - k * y, rel=1e-4, abs=1e-6)
    y, v = pso._oscillator(y0, v0, k, gamma, 0.0)
    assert (y, v) == pytest.approx((y0, v0), abs=1e-15)


def test_exact_step_is_the_limit_of_euler_steps():
    x = np.array([0.3, 0.8]); v = np.array([0.05, -0.1])
    xp = np.array([0.5, 0.5]); xg = np.array([0.9, 0.2])
    xe, ve = pso.exact_step(x, v, xp, xg, 0.6, 0.3, 1.0, 0.5, 1.0, 5.0)
    errs = []
    for m in (100, 1000):
        xs, vs = x.copy(), v.copy()
        for _ in range(m):
            xs, vs = pso.euler_step(xs, vs, xp, xg, 0.6, 0.3, 1.0, 0.5, 1.0 / m, 5.0)
        errs.append(np.abs(xs - xe).max())
    assert errs[1] < 0.2 * errs[0] and errs[1] < 1e-3     # first-order convergence


def test_tdamp_one_is_critical():
    cp, cg = 1.0, 0.5
    t = pso.damping_time(1.0, cp, cg)
    k = 0.5 * (cp + cg)
    assert (1.0 / t) ** 2 == pytest.approx(4 * k, rel=1e-14)


def test_euler_orbit_grows_when_its_determinant_exceeds_one():
    """One particle with fixed springs: Eq. 21's recurrence (x, v) -> (x + v dt,
    v (1 - dt/t_damp) + k (c - x) dt) has determinant (1 - dt/t_damp) + k dt^2.
    At App. A.2's constants (dt = 1, mean k = 0.75, t_damp = 5.77) it exceeds
    one and the orbit about the spring centre grows; Locust's exact orbit with
    the same springs decays."""
    cp, cg, dt = 1.0, 0.5, 1.0
    t_damp = pso.damping_time(10.0, cp, cg)
    xi = 0.5
    k = (cp + cg) * xi
    assert (1 - dt / t_damp) + k * dt * dt > 1.0
    c = np.array([0.5])
    for step, grows in ((pso.euler_step, True), (pso.exact_step, False)):
        x, v = np.array([0.51]), np.zeros(1)
        amp0 = abs(x[0] - 0.5)
        amps = []
        for _ in range(40):
            x, v = step(x, v, c, c, xi, xi, cp, cg, dt, t_damp)
            amps.append(abs(x[0] - 0.5) + abs(v[0]))
        assert (max(amps[-8:]) > 10 * amp0) == grows, (step.__name__, amps[-8:])


def test_bests_and_convergence_on_a_bowl():
    c = np.array([0.3, 0.6, 0.25, 0.7, 0.4, 0.55, 0.45])
    bowl = lambda X: np.sum((np.asarray(X) - c) ** 2, axis=1)   # noqa: E731
    d = synthgen.pso_draws(5, 200, 60)
    for form in ("euler", "exact"):
        r = pso.run(bowl, d["x0"], d["xi_p"], d["xi_g"], 60, form=form)
        h = r["history"]
        assert np.all(np.diff(h) <= 0)
        assert r["fg"] == r["fp"].min() and r["fg"] == pytest.approx(bowl(r["xg"][None])[0], rel=1e-14)
        assert r["evals"] == 200 * 61
        if form == "exact":   # the swarm contracts onto the minimum
            assert h[-1] < 1e-6 * h[0], h[-1]
        else:                 # the best still improves, the growing orbits keep the swarm spread out
            assert h[-1] < 0.2 * h[0], h[-1]
