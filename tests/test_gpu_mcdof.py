"""GPU parity of the Monte Carlo degrees of freedom (Sec. 2.5) against the oracle.

The solve's `dof` output (opts mc_noise = bhat) is compared with the oracle
at the GPU's corner lambda, on the same seeded draws bhat, through
gamma = bhat^T bhat - dof (the trace estimate, the part that carries the
computation):
* FP64 path (second system in lockstep with the data system's CG
  coefficients, as the paper does) against oracle.dof.mc_dof, both with CG
  to 1e-12: within 1e-8 relative.  The lockstep vector is a fixed polynomial
  in the operator, so rounding injected at one step is amplified by the
  later factors; 3.8e-9 was seen at lambda = 1e-3 with curvature H.
* FP32 path (second system by its own CG to 1e-7) against
  oracle.dof.mc_dof_solve at 1e-10: within 1e-4 relative.
A member that maps no pixel gets NaN.  The pass leaves every other result of
the solve unchanged (bit for bit), and it is bitwise repeatable.
"""
import os

import numpy as np
import pytest
import torch

import synthgen
from oracle import dof as odof
from oracle import mock, solve

pytestmark = pytest.mark.gpu
DEV = "cuda"
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sl():
    import paper_1101_5803_amd as sl
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sl


def _np(out):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _small_case(reg):
    nx, ny, pix, K = 40, 36, 0.1, 7
    psf = mock.gaussian_psf(K, 2.0)
    w = synthgen.Workload("small", 9, nx, ny, pix, 2, 6, 12, 1.0, K, 2.0, 40.0, reg, (1e-3,), 1e-10, "sersic", 2)
    lens_true = np.array([1.0, 0.75, 0.5, 0.04, 0.3, 0.02, -0.03])
    clean = mock.clean_image(lens_true, synthgen.source_blobs(w), nx, ny, pix, 6, psf)
    sigma = clean.max() / 40.0
    d = clean + sigma * synthgen.noise_unit(w)
    G = synthgen.population(21, 6)
    G[0] = lens_true
    G[4] = [5.0, 1.0, 0.0, 0.0, 0.0, 5.0, 5.0]     # maps nothing onto the grid
    ns = np.array([12, 8, 19, 5, 16, 23], dtype=np.int32)
    return d, sigma, psf, (nx, ny, pix), G, ns


def _check(out, bhat, G, ns, d, sigma, psf, geom, nsub, R, reg, lams, prec, skip=()):
    nx, ny, pix = geom
    n2 = float((bhat ** 2).sum())
    worst = 0.0
    for m in range(len(G)):
        if m in skip:
            assert np.isnan(out["dof"][m]), m
            continue
        k = int(out["k_star"][m])
        pb = solve.Problem(G[m], d, sigma, psf, nx, ny, pix, nsub, int(ns[m]), R, reg)
        if prec == "f64":
            ref = odof.mc_dof(pb, lams[k], bhat, tol=1e-12)
        else:
            ref = odof.mc_dof_solve(pb, lams[k], bhat, tol=1e-10)
        assert ref["status"] == 0
        bound = 1e-8 if prec == "f64" else 1e-4
        g_gpu = n2 - out["dof"][m]
        rel = abs(g_gpu - ref["gamma"]) / abs(ref["gamma"])
        worst = max(worst, rel)
        assert rel <= bound, (m, k, g_gpu, ref["gamma"], rel)
        assert abs(out["dof"][m] - ref["nu"]) <= bound * abs(ref["gamma"])
    return worst


@pytest.mark.parametrize("reg", ["curvature", "identity"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_small_batch_dof_vs_oracle(sl, reg, prec):
    d, sigma, psf, (nx, ny, pix), G, ns = _small_case(reg)
    lams = synthgen.log_grid(1e-3, 1e1, 6)
    bhat = synthgen.mc_draws(9, ny, nx)
    dtype = torch.float64 if prec == "f64" else torch.float32
    solver = sl.Solver(torch.tensor(d, device=DEV), sigma, torch.tensor(psf, device=DEV),
                       sl.Grid(nx, ny, pix, 2), 1.0, reg=reg, dtype=dtype)
    lens = torch.tensor(G, device=DEV)
    nst = torch.tensor(ns, device=DEV)
    tol = 1e-12 if prec == "f64" else 1e-7
    plain = _np(solver.solve_semilinear(lens, nst, lams, tol=tol))
    out = _np(solver.solve_semilinear(lens, nst, lams, tol=tol,
                                      mc_noise=torch.tensor(bhat.reshape(-1), device=DEV)))
    for k in ("chi2", "reg", "iters", "status", "k_star", "corner_status"):
        assert np.array_equal(out[k], plain[k]), k
    worst = _check(out, bhat, G, ns, d, sigma, psf, (nx, ny, pix), 2, 1.0, reg, lams, prec, skip=(4,))
    print(f"{reg} {prec}: worst gamma rel err {worst:.2e}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_c2_member_dof_vs_oracle(sl, prec):
    w = synthgen.C2
    z = np.load(os.path.join(HERE, "data", "c2.npz"))
    bhat = synthgen.mc_draws(w.seed, w.ny, w.nx)
    dtype = torch.float64 if prec == "f64" else torch.float32
    solver = sl.Solver(torch.tensor(z["d"], device=DEV), float(z["sigma"]), torch.tensor(z["psf"], device=DEV),
                       sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width, reg=w.reg, dtype=dtype)
    G = np.atleast_2d(z["lens"])
    ns = np.array([w.ns], dtype=np.int32)
    out = _np(solver.solve_semilinear(torch.tensor(G, device=DEV), torch.tensor(ns, device=DEV), w.lambdas,
                                      tol=1e-12 if prec == "f64" else 1e-7, maxit=20000, max_ns=w.ns,
                                      mc_noise=torch.tensor(bhat.reshape(-1), device=DEV)))
    _check(out, bhat, G, ns, z["d"], float(z["sigma"]), z["psf"], (w.nx, w.ny, w.pix), w.nsub_model, w.half_width,
           w.reg, w.lambdas, prec)
    # the reduced chi^2 at the true lens's corner is close to one (Sec. 2.5, Sec. 4)
    chi2r = out["chi2"][0, int(out["k_star"][0])] / out["dof"][0]
    assert 0.8 < chi2r < 1.3, chi2r


def test_c3_launch_dof_sampled_and_repeatable(sl):
    """The 256-member c3 launch with the Monte Carlo pass: members of the
    smallest, a middle and the largest grids against the oracle, every valid
    member finite with 0 < dof < bhat^T bhat, and two runs identical bit for
    bit."""
    w = synthgen.C3
    z = np.load(os.path.join(HERE, "data", "c2.npz"))
    pop = synthgen.population(w.seed, 256)
    grids = synthgen.member_grids(w.seed, 256)
    bhat = synthgen.mc_draws(w.seed, w.ny, w.nx)
    solver = sl.Solver(torch.tensor(z["d"], device=DEV), float(z["sigma"]), torch.tensor(z["psf"], device=DEV),
                       sl.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width, reg=w.reg, dtype=torch.float32)
    noise = torch.tensor(bhat.reshape(-1), device=DEV)
    lens = torch.tensor(pop, device=DEV)
    nst = torch.tensor(grids, device=DEV)
    a = _np(solver.solve_semilinear(lens, nst, w.lambdas, tol=1e-7, max_ns=96, mc_noise=noise))
    b = _np(solver.solve_semilinear(lens, nst, w.lambdas, tol=1e-7, max_ns=96, mc_noise=noise))
    assert np.array_equal(a["dof"], b["dof"])
    n2 = float((bhat ** 2).sum())   # gamma = bhat^T A xhat >= 0, so 0 < dof <= bhat^T bhat
    assert np.all(np.isfinite(a["dof"])) and np.all((a["dof"] > 0) & (a["dof"] < n2))
    order = np.argsort(grids, kind="stable")
    sample = [int(order[0]), int(order[128]), int(order[-1])]
    _check({k: v[sample] for k, v in a.items() if k != "s_off" and k != "s_corner"}, bhat, pop[sample],
           grids[sample], z["d"], float(z["sigma"]), z["psf"], (w.nx, w.ny, w.pix), w.nsub_model, w.half_width,
           w.reg, w.lambdas, "f32")
