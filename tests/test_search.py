"""Host GA driver: operators against the oracle GA, monotone progress, checkpoint/resume.

The fitness here is a cheap analytic function on the CPU so that the driver
logic is tested without a GPU; the device fitness is covered in
test_gpu_search.py.
"""
import json
import os

import numpy as np
import pytest

from oracle import ga as oga
import synthgen

search = pytest.importorskip("paper_1101_5803_amd.search")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ferret_defaults.json")


def sphere(U):
    """Quadratic bowl with its minimum inside the unit box (angle genes wrap)."""
    c = np.array([0.3, 0.6, 0.9, 0.2, 0.05, 0.5, 0.5])
    d = U - c
    for g in (2, 4):
        d[:, g] = (d[:, g] + 0.5) % 1.0 - 0.5
    return 1.0 + (d * d).sum(axis=1)


def test_config_from_ferret_defaults():
    cfg = search.GAConfig.from_json(GOLDEN)
    d = json.load(open(GOLDEN))
    assert cfg.xover_strength == d["XOver.strength"] == 0.25
    assert cfg.pmutate == d["mutation.PMutate"] == 0.05
    assert cfg.mutation_scale == d["mutation.scale"] == 0.25


def test_operators_match_oracle_ga():
    P = 64
    X = np.random.default_rng(1).uniform(size=(P, 7))
    dr = synthgen.ga_draws(2, P, 3)
    for g in range(3):
        d = {k: v[g] for k, v in dr.items()}
        Y = search.make_offspring(X, np.arange(P), d["partner"], d["xstrength"], d["mut_mask"], d["mut_step"],
                                  search.GAConfig())
        Yo = oga.offspring(X, d)
        assert np.array_equal(Y, Yo)
        fX, fY = sphere(X), sphere(Y)
        Xn, fn = search.tournament(X, fX, Y, fY, d["perm"])
        Xo, fo = oga.tournament(X, fX, Yo, fY, d["perm"])
        assert np.array_equal(Xn, Xo) and np.array_equal(fn, fo)
        X = Xn


def test_ga_run_matches_oracle_loop_and_improves():
    P, G = 48, 12
    X0 = np.random.default_rng(3).uniform(size=(P, 7))
    dr = synthgen.ga_draws(4, P, G)
    s = search.GeneticSearch(sphere, X0)
    Xo, fo = X0.copy(), sphere(X0)
    for g in range(G):
        d = {k: v[g] for k, v in dr.items()}
        s.step(d)
        Yo = oga.offspring(Xo, d)
        Xo, fo = oga.tournament(Xo, fo, Yo, sphere(Yo), d["perm"])
    assert np.array_equal(s.X, Xo) and np.array_equal(s.fX, fo)
    h = np.array(s.history)
    assert np.all(np.diff(h) <= 0) and h[-1] < h[0]
    assert s.full_solves == P * (G + 1)


def test_checkpoint_resume_is_exact(tmp_path):
    P, G = 32, 6
    X0 = np.random.default_rng(5).uniform(size=(P, 7))
    dr = synthgen.ga_draws(6, P, G)
    one = search.GeneticSearch(sphere, X0)
    for g in range(G):
        one.step({k: v[g] for k, v in dr.items()})
    two = search.GeneticSearch(sphere, X0)
    for g in range(G // 2):
        two.step({k: v[g] for k, v in dr.items()})
    path = str(tmp_path / "ckpt.npz")
    two.save(path)
    three = search.GeneticSearch.resume(path, sphere)
    for g in range(three.generation, G):
        three.step({k: v[g] for k, v in dr.items()})
    assert np.array_equal(one.X, three.X) and np.array_equal(one.fX, three.fX)
    assert one.history == three.history and one.full_solves == three.full_solves
    U1, f1 = one.training_set()
    U3, f3 = three.training_set()
    assert np.array_equal(U1, U3) and np.array_equal(f1, f3)


def test_box_round_trip_and_wrapping():
    box = search.Box(synthgen.PRIOR_LO, synthgen.PRIOR_HI)
    U = np.random.default_rng(7).uniform(size=(10, 7))
    assert np.allclose(box.to_unit(box.to_phys(U)), U, rtol=0, atol=1e-15)
    X = np.full((2, 7), 0.99)
    Y = search.make_offspring(X, np.arange(2), np.array([1, 0]), np.zeros(2), np.zeros((2, 7)),
                              np.full((2, 7), 0.2), search.GAConfig())
    # every gene mutates by +0.05: angle genes wrap to 0.04, the others clip to 1
    assert np.allclose(Y[:, [2, 4]], 0.04) and np.all(Y[:, [0, 1, 3, 5, 6]] == 1.0)


def test_invalid_members_never_win():
    X = np.zeros((3, 7))
    fX = np.array([5.0, 5.0, 5.0])
    Y = np.ones((3, 7))
    fY = np.array([np.inf, 5.0, 4.0])
    Xn, fn = search.tournament(X, fX, Y, fY, np.arange(3))
    assert list(fn) == [5.0, 5.0, 4.0] and np.all(Xn[0] == 0) and np.all(Xn[1] == 0) and np.all(Xn[2] == 1)
