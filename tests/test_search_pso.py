"""The swarm driver (paper_1101_5803_amd.search.SwarmSearch, host logic)
against the particle swarm oracle (oracle/pso.py) on the same seeded draws:
positions, velocities, bests and the best-fitness history, for both orbit
forms, on a bowl and on a function with a wall-bound minimum and an angle
gene that wraps."""
import numpy as np
import pytest

import synthgen
from oracle import pso

search = pytest.importorskip("paper_1101_5803_amd.search")


def _bowl(X):
    c = np.array([0.3, 0.6, 0.25, 0.7, 0.4, 0.55, 0.45])
    return np.sum((np.asarray(X) - c) ** 2, axis=1)


def _wall(X):   # minimum at gene 0 = 1 (on the wall) and gene 2 near 0 (wraps)
    X = np.asarray(X)
    d2 = np.minimum(np.abs(X[:, 2] - 0.02), 1.0 - np.abs(X[:, 2] - 0.02))
    return (1.2 - X[:, 0]) ** 2 + d2 ** 2 + 0.1 * np.sum((X[:, 3:] - 0.5) ** 2, axis=1) + 0.05 * X[:, 1]


@pytest.mark.parametrize("fit", [_bowl, _wall])
@pytest.mark.parametrize("exact", [True, False])
def test_swarm_matches_oracle(fit, exact):
    N, T = 24, 30
    d = synthgen.pso_draws(11, N, T)
    ref = pso.run(fit, d["x0"], d["xi_p"], d["xi_g"], T, form="exact" if exact else "euler")
    s = search.SwarmSearch(fit, d["x0"], search.SwarmConfig(exact=exact))
    for t in range(T):
        s.step(d["xi_p"][t], d["xi_g"][t])
    assert np.allclose(s.X, ref["x"], rtol=0, atol=1e-12)
    assert np.allclose(s.V, ref["v"], rtol=0, atol=1e-12)
    assert np.allclose(s.P, ref["xp"], rtol=0, atol=1e-12)
    assert np.allclose(s.fP, ref["fp"], rtol=1e-12, atol=0)
    assert np.allclose(s.history, ref["history"], rtol=1e-12, atol=0)
    assert s.evals == ref["evals"]
