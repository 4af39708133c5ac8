"""GPU parity of the batched solve (sl_solve_semilinear) against the FP64 oracle.

Bars:
* FP64 path, CG to 1e-12 on both sides: chi^2 relative error <= 1e-9 and
  ||ds||/||s|| <= 1e-7 at every lambda.
* FP32 path (FP64 inner products, chi^2, L-curve), CG to 1e-7: chi^2
  relative error <= 1e-5 at every lambda and ||ds||/||s|| <= 1e-4 at the
  L-curve corner (the small-lambda systems are ill-conditioned enough that
  FP32 CG stalls near 1e-7 residual; their solutions are reported, not
  gated).
* The corner is an argmax, so it is unique only where the oracle's own
  corner is stable: the GPU corner must be one of the corners the oracle
  returns when its (reg, chi^2) points are perturbed by relative noise at
  the FP32 path's chi^2 tolerance (1e-5; 64 seeded draws plus the
  unperturbed curve).  For well-separated curvature maxima that set is a
  single index; chi^2 and s are always compared at the GPU's corner.
"""
import os

import numpy as np
import pytest
import torch

import synthgen
from oracle import coracle, lcurve, mock, solve

pytestmark = pytest.mark.gpu
DEV = "cuda"
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def semilin():
    import paper_1101_5803_amd as sl
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sl


def _run(semilin, d, sigma, psf, grid, R, reg, dtype, lens, ns, lambdas, tol, maxit=4000):
    solver = semilin.Solver(torch.tensor(d, device=DEV), sigma, torch.tensor(psf, device=DEV), grid, R,
                            reg=reg, dtype=dtype)
    out = solver.solve_semilinear(torch.tensor(np.atleast_2d(lens), device=DEV),
                                  torch.tensor(np.asarray(ns, dtype=np.int32), device=DEV), lambdas,
                                  tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _corner_set(reg, chi2, rel=1e-5, draws=64):
    """Corners the oracle's L-curve gives under relative noise of size rel."""
    rng = np.random.default_rng(12345)
    ks = {lcurve.corner(reg, chi2)[0]}
    for _ in range(draws):
        ks.add(lcurve.corner(reg * (1 + rel * rng.standard_normal(reg.size)),
                             chi2 * (1 + rel * rng.standard_normal(chi2.size)))[0])
    return ks


def _corner_ok(k_gpu, k_ref, reg, chi2):
    return k_gpu == k_ref or k_gpu in _corner_set(np.asarray(reg), np.asarray(chi2))


def _small_case(psf_kind="gauss", K=7):
    nx, ny, pix = 40, 36, 0.1
    rng = np.random.default_rng(7)
    if psf_kind == "gauss":
        psf = mock.gaussian_psf(K, 2.0)
    else:
        psf = rng.uniform(0.2, 1.0, (K, K))
        psf /= psf.sum()
    w = synthgen.Workload("small", 9, nx, ny, pix, 2, 6, 12, 1.0, K, 2.0, 40.0, "curvature",
                          (1e-3,), 1e-10, "sersic", 2)
    lens_true = np.array([1.0, 0.75, 0.5, 0.04, 0.3, 0.02, -0.03])
    blobs = synthgen.source_blobs(w)
    clean = mock.clean_image(lens_true, blobs, nx, ny, pix, 6, psf)
    sigma = clean.max() / 40.0
    d = clean + sigma * synthgen.noise_unit(w)
    G = synthgen.population(21, 8)
    G[0] = lens_true
    G[5] = [5.0, 1.0, 0.0, 0.0, 0.0, 5.0, 5.0]     # maps nothing onto the grid
    G[6, 1] = 1.0                                     # SIS member
    ns = np.array([12, 8, 19, 5, 16, 11, 2, 23], dtype=np.int32)
    return d, sigma, psf, (nx, ny, pix), G, ns


@pytest.mark.parametrize("reg", ["curvature", "identity"])
@pytest.mark.parametrize("psf_kind", ["gauss", "general"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_small_batched_parity(semilin, reg, psf_kind, prec):
    d, sigma, psf, (nx, ny, pix), G, ns = _small_case(psf_kind)
    lams = synthgen.log_grid(1e-3, 1e1, 6)
    grid = semilin.Grid(nx, ny, pix, 2)
    dtype = torch.float64 if prec == "f64" else torch.float32
    tol = 1e-12 if prec == "f64" else 1e-7
    out = _run(semilin, d, sigma, psf, grid, 1.0, reg, dtype, G, ns, lams, tol)
    ref = coracle.evaluate(G, ns, 1.0, nx, ny, pix, 2, d, sigma, psf, reg, lams, tol=1e-12, want_s=True,
                           threads=8)
    off = out["s_off"]
    assert off[0] == 0 and np.all(np.diff(off) == ns.astype(np.int64) ** 2)
    for m in range(len(G)):
        if m == 5:
            assert np.all(out["status"][m] == semilin._lib.ST_EMPTY)
            assert out["corner_status"][m] == semilin._lib.ST_EMPTY
            np.testing.assert_allclose(out["chi2"][m], (d ** 2).sum() / sigma ** 2, rtol=1e-12)
            assert not out["s_corner"][off[m]:off[m + 1]].any()
            continue
        assert np.all(out["status"][m] == 0), (m, out["status"][m])
        rel = np.abs(out["chi2"][m] - ref["chi2"][m]) / ref["chi2"][m]
        assert rel.max() <= (1e-9 if prec == "f64" else 1e-5), (m, rel)
        k_ref, _ = lcurve.corner(ref["reg"][m], ref["chi2"][m])
        k = int(out["k_star"][m])
        assert _corner_ok(k, k_ref, ref["reg"][m], ref["chi2"][m]), (m, k, k_ref)
        s_ref = ref["s"][m, k, :ns[m] ** 2]
        s_gpu = out["s_corner"][off[m]:off[m + 1]]
        err = np.linalg.norm(s_gpu - s_ref) / np.linalg.norm(s_ref)
        assert err <= (1e-7 if prec == "f64" else 1e-4), (m, err)
        if prec == "f32":
            regrel = np.abs(out["reg"][m] - ref["reg"][m]) / ref["reg"][m]
            assert regrel[k:].max() <= 1e-3, (m, regrel)


@pytest.mark.parametrize("psf_kind", ["gauss", "general"])
def test_small_preconditioned_vs_plain_and_oracle(semilin, psf_kind):
    """Ragged grids n = 2..23 (sine-transform sizes that are not a multiple of
    the 16-wide MFMA tiles, down to n = 2) with lambdas up to 1e3, where the
    FP32 curvature solve takes the spectral preconditioner: the default path
    and plain CG (tuning plain_cg = 1) both match the FP64 oracle, and the
    preconditioner ran (iteration counts differ on some items)."""
    d, sigma, psf, (nx, ny, pix), G, ns = _small_case(psf_kind)
    lams = synthgen.log_grid(1e-2, 1e3, 6)
    solver = semilin.Solver(torch.tensor(d, device=DEV), sigma, torch.tensor(psf, device=DEV),
                            semilin.Grid(nx, ny, pix, 2), 1.0, reg="curvature", dtype=torch.float32)
    lens = torch.tensor(G, device=DEV)
    nst = torch.tensor(ns, device=DEV)
    res = {}
    for name, tun in (("pcg", {}), ("plain", {"plain_cg": 1})):
        out = solver.solve_semilinear(lens, nst, lams, tol=1e-7, maxit=4000, tuning=tun)
        torch.cuda.synchronize()
        res[name] = {k: v.cpu().numpy() for k, v in out.items()}
    ref = coracle.evaluate(G, ns, 1.0, nx, ny, pix, 2, d, sigma, psf, "curvature", lams, tol=1e-12, threads=8)
    live = [m for m in range(len(G)) if m != 5]
    for name in ("pcg", "plain"):
        o = res[name]
        for m in live:
            assert np.all(o["status"][m] == 0), (name, m, o["status"][m])
            rel = np.abs(o["chi2"][m] - ref["chi2"][m]) / ref["chi2"][m]
            assert rel.max() <= 1e-5, (name, m, rel)
    differ = res["pcg"]["iters"][live] != res["plain"]["iters"][live]
    assert differ.any()
    assert res["pcg"]["iters"][live].sum() < res["plain"]["iters"][live].sum()


def test_invalid_members_flagged(semilin):
    d, sigma, psf, (nx, ny, pix), G, ns = _small_case()
    G = G[:4].copy()
    G[1, 1] = 0.0          # q = 0
    G[2, 3] = np.inf
    ns = ns[:4].copy()
    ns[3] = 300            # beyond max_ns
    solver = semilin.Solver(torch.tensor(d, device=DEV), sigma, torch.tensor(psf, device=DEV),
                            semilin.Grid(nx, ny, pix, 2), 1.0)
    out = solver.solve_semilinear(torch.tensor(G, device=DEV), torch.tensor(ns, device=DEV),
                                  [1e-2, 1e-1, 1.0, 10.0], max_ns=32)
    st = out["status"].cpu().numpy()
    assert np.all(st[0] == 0)
    assert np.all(st[1:] == semilin._lib.ST_INVALID)
    assert np.all(np.isnan(out["chi2"].cpu().numpy()[1:]))


def test_host_validation(semilin):
    d, sigma, psf, (nx, ny, pix), G, ns = _small_case()
    solver = semilin.Solver(torch.tensor(d, device=DEV), sigma, torch.tensor(psf, device=DEV),
                            semilin.Grid(nx, ny, pix, 2), 1.0)
    with pytest.raises(semilin._lib.SemilinError, match="ascending"):
        solver.solve_semilinear(torch.tensor(G, device=DEV), torch.tensor(ns, device=DEV), [1.0, 0.5])
    with pytest.raises(semilin._lib.SemilinError, match="maxit"):
        solver.solve_semilinear(torch.tensor(G, device=DEV), torch.tensor(ns, device=DEV), [1.0], maxit=0)


def test_maxit_status(semilin):
    d, sigma, psf, (nx, ny, pix), G, ns = _small_case()
    out = _run(semilin, d, sigma, psf, semilin.Grid(nx, ny, pix, 2), 1.0, "curvature", torch.float32,
               G[:2], ns[:2], [1e-3, 1e-2, 1e-1, 1.0], 1e-7, maxit=3)
    assert np.all(out["status"] == semilin._lib.ST_MAXIT)
    assert np.all(out["iters"] == 3)


def test_c1_plain_fp64(semilin):
    """c1: SIS, H = I, one lambda, FP64 GPU path vs the dense Cholesky oracle."""
    w = synthgen.C1
    z = np.load(os.path.join(os.path.dirname(__file__), "data", "c1.npz"))
    out = _run(semilin, z["d"], float(z["sigma"]), z["psf"], semilin.Grid(w.nx, w.ny, w.pix, w.nsub_model),
               w.half_width, w.reg, torch.float64, z["lens"], [w.ns], w.lambdas, w.tol)
    pb = solve.Problem(z["lens"], z["d"], float(z["sigma"]), z["psf"], w.nx, w.ny, w.pix, w.nsub_model, w.ns,
                       w.half_width, w.reg)
    s_ref = solve.solve_dense(pb, w.lambdas[0])
    err = np.linalg.norm(out["s_corner"] - s_ref) / np.linalg.norm(s_ref)
    assert err <= 1e-8, err
    assert abs(out["chi2"][0, 0] - pb.chi2(s_ref)) <= 1e-10 * pb.chi2(s_ref)
    assert out["k_star"][0] == 0 and out["status"][0, 0] == 0


def _c2_gpu(semilin, dtype, tol):
    w = synthgen.C2
    z = np.load(os.path.join(os.path.dirname(__file__), "data", "c2.npz"))
    return _run(semilin, z["d"], float(z["sigma"]), z["psf"], semilin.Grid(w.nx, w.ny, w.pix, w.nsub_model),
                w.half_width, w.reg, dtype, z["lens"], [w.ns], w.lambdas, tol, maxit=4000)


def test_c2_fp32_vs_oracle(semilin):
    """c2 (128^2 image, 64^2 nodes, 16 lambdas, curvature H): FP32 path."""
    g = np.load(os.path.join(GOLD, "c2_oracle.npz"))
    out = _c2_gpu(semilin, torch.float32, 1e-7)
    assert np.all(out["status"] == 0)
    rel = np.abs(out["chi2"][0] - g["chi2"]) / g["chi2"]
    assert rel.max() <= 1e-5, rel
    k = int(out["k_star"][0])
    assert _corner_ok(k, int(g["k_star"]), g["reg"], g["chi2"])
    err = np.linalg.norm(out["s_corner"] - g["s"][k]) / np.linalg.norm(g["s"][k])
    assert err <= 1e-4, err


def test_c2_fp64_vs_oracle(semilin):
    g = np.load(os.path.join(GOLD, "c2_oracle.npz"))
    out = _c2_gpu(semilin, torch.float64, 1e-10)
    rel = np.abs(out["chi2"][0] - g["chi2"]) / g["chi2"]
    assert rel.max() <= 1e-9, rel
    assert int(out["k_star"][0]) == int(g["k_star"])
    k = int(g["k_star"])
    err = np.linalg.norm(out["s_corner"] - g["s"][k]) / np.linalg.norm(g["s"][k])
    assert err <= 1e-7, err


def test_c3_full_launch_sampled(semilin):
    """c3: 256 members, uneven grids 32..96, one persistent launch; sampled
    members compared with the oracle's results for the same genomes."""
    g = np.load(os.path.join(GOLD, "c3_sample.npz"))
    w = synthgen.C3
    z = np.load(os.path.join(os.path.dirname(__file__), "data", "c2.npz"))
    pop = synthgen.population(w.seed, 256)
    grids = synthgen.member_grids(w.seed, 256)
    out = _run(semilin, z["d"], float(z["sigma"]), z["psf"], semilin.Grid(w.nx, w.ny, w.pix, w.nsub_model),
               w.half_width, w.reg, torch.float32, pop, grids, w.lambdas, 1e-7, maxit=4000)
    off = out["s_off"]
    for j, m in enumerate(g["members"]):
        assert np.all(out["status"][m] == 0)
        rel = np.abs(out["chi2"][m] - g["chi2"][j]) / g["chi2"][j]
        assert rel.max() <= 1e-5, (m, rel)
        k = int(out["k_star"][m])
        assert _corner_ok(k, int(g["k_star"][j]), g["reg"][j], g["chi2"][j]), (m, k)
        if k == int(g["k_star"][j]):
            s_ref = g["s_corner"][j][:grids[m] ** 2]
            err = np.linalg.norm(out["s_corner"][off[m]:off[m + 1]] - s_ref) / np.linalg.norm(s_ref)
            assert err <= 1e-4, (m, err)
    # properties at full size: every member either converged or is flagged
    assert np.all(np.isin(out["status"], [0, 1]))
    assert np.all(out["chi2"] > 0)
    # Tikhonov monotonicity on every member (chi^2 non-decreasing in lambda)
    ok = np.diff(out["chi2"], axis=1) >= -1e-5 * out["chi2"][:, 1:]
    assert ok.mean() > 0.99


def test_c3_preconditioned_matches_plain_cg(semilin):
    """c3 with the spectral preconditioner (default) and with plain CG
    (tuning plain_cg = 1): the same Eq. 7 solutions at every (member, lambda),
    every item converged, and the preconditioner took part of the items (fewer
    CG iterations in total).  The sampled test above compares the default path
    with the oracle; this one carries that bar to all 4096 items."""
    w = synthgen.C3
    z = np.load(os.path.join(os.path.dirname(__file__), "data", "c2.npz"))
    pop = synthgen.population(w.seed, 256)
    grids = synthgen.member_grids(w.seed, 256)
    solver = semilin.Solver(torch.tensor(z["d"], device=DEV), float(z["sigma"]), torch.tensor(z["psf"], device=DEV),
                            semilin.Grid(w.nx, w.ny, w.pix, w.nsub_model), w.half_width, reg=w.reg,
                            dtype=torch.float32)
    lens = torch.tensor(pop, device=DEV)
    ns = torch.tensor(grids, device=DEV)
    res = {}
    for name, tun in (("pcg", {}), ("plain", {"plain_cg": 1})):
        out = solver.solve_semilinear(lens, ns, w.lambdas, tol=1e-7, maxit=4000, max_ns=96, tuning=tun)
        torch.cuda.synchronize()
        res[name] = {k: v.cpu().numpy() for k, v in out.items()}
    a, b = res["pcg"], res["plain"]
    assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
    rel = np.abs(a["chi2"] - b["chi2"]) / b["chi2"]
    assert rel.max() <= 1e-5, rel.max()
    relr = np.abs(a["reg"] - b["reg"]) / b["reg"]
    assert np.median(relr) <= 1e-4, np.median(relr)
    assert a["iters"].sum() < 0.9 * b["iters"].sum(), (a["iters"].sum(), b["iters"].sum())
    # both corners are corners of the same curve up to the FP32 chi^2 tolerance
    same = a["k_star"] == b["k_star"]
    assert same.mean() > 0.95
    for m in np.nonzero(~same)[0]:
        assert a["k_star"][m] in _corner_set(b["reg"][m], b["chi2"][m]) | {int(b["k_star"][m])}, m


def test_c4_full_launch_sampled(semilin):
    """c4: 200x200 image (image frame in global memory), 100x100 nodes, 21x21
    PSF, 24 lambdas; the true lens plus 1024 population members in one launch,
    three sampled against the oracle."""
    g = np.load(os.path.join(GOLD, "c4_sample.npz"))
    w = synthgen.C4
    z = np.load(os.path.join(os.path.dirname(__file__), "data", "c4.npz"))
    pop = synthgen.population(w.seed, 1024)
    lens = np.vstack([g["lens"][:1], pop])
    ns = np.full(lens.shape[0], w.ns, dtype=np.int32)
    out = _run(semilin, z["d"], float(z["sigma"]), z["psf"], semilin.Grid(w.nx, w.ny, w.pix, w.nsub_model),
               w.half_width, w.reg, torch.float32, lens, ns, w.lambdas, w.tol, maxit=4000)
    I = w.ns * w.ns
    for j, m in enumerate(g["members"]):
        row = int(m) + 1   # row 0 is the true lens
        assert np.allclose(lens[row], g["lens"][j])
        assert np.all(out["status"][row] == 0)
        rel = np.abs(out["chi2"][row] - g["chi2"][j]) / g["chi2"][j]
        assert rel.max() <= 1e-5, (m, rel)
        k = int(out["k_star"][row])
        assert _corner_ok(k, int(g["k_star"][j]), g["reg"][j], g["chi2"][j]), (m, k)
        if k == int(g["k_star"][j]):
            off = out["s_off"]
            assert off[row + 1] - off[row] == I
            s = out["s_corner"][off[row]:off[row + 1]]
            err = np.linalg.norm(s - g["s_corner"][j][:I]) / np.linalg.norm(g["s_corner"][j][:I])
            assert err <= 1e-4, (m, err)
    assert np.all(np.isin(out["status"], [0, 1, 2]))
    ok = out["status"] == 0
    assert np.all(out["chi2"][ok] > 0)


def test_max_sizes_normal_equations(semilin):
    """Largest image (256 x 256) and source grid (128 x 128) with a 21 x 21 PSF,
    one member at the smallest grid (2 x 2) and one that maps nothing, in one
    launch.  At this size the oracle is too slow, so the solution is checked
    through properties that hold at any size, with the stand-alone operators
    (themselves oracle-tested) in FP64: the normal-equation residual
    ||(L^T B^T B L + lambda H^T H) s - L^T B^T d|| / ||L^T B^T d|| and chi^2."""
    nx = ny = 256
    pix, R = 0.025, 1.0
    grid = semilin.Grid(nx, ny, pix, 2)
    psf = mock.gaussian_psf(21, 3.0)
    rng = np.random.default_rng(17)
    d = rng.standard_normal((ny, nx))
    sigma = 1.0
    G = np.array([[1.0, 0.7, 0.5, 0.05, 1.0, 0.01, 0.02],
                  [1.1, 0.9, 1.0, 0.02, 0.2, -0.02, 0.0],
                  [20.0, 1.0, 0.0, 0.0, 0.0, 0.0, 30.0]])   # every ray lands ~20" away: maps nothing
    ns = np.array([128, 2, 64], dtype=np.int32)
    lams = [1e-2, 1.0]
    out = _run(semilin, d, sigma, psf, grid, R, "curvature", torch.float32, G, ns, lams, 1e-6, maxit=6000)
    assert np.all(out["status"][:2] == 0), out["status"]
    assert np.all(out["status"][2] == semilin._lib.ST_EMPTY)
    assert np.all(out["k_star"][:2] == 0) and np.all(out["corner_status"][:2] == semilin._lib.ST_LCURVE)
    uv = semilin.lens_trace(torch.tensor(G, device=DEV), grid, ns, R)
    dd = torch.tensor(d, device=DEV)
    pt = torch.tensor(psf, device=DEV)
    off = out["s_off"]
    for m in range(2):
        n = [int(ns[m])]
        s = torch.tensor(out["s_corner"][off[m]:off[m + 1]], device=DEV)
        um = uv[m:m + 1].contiguous()
        by = semilin.apply_B(pt, semilin.apply_L(um, grid, n, s).reshape(1, ny, nx))
        chi2 = float(((by[0] - dd) ** 2).sum()) / sigma ** 2
        assert abs(chi2 - out["chi2"][m, 0]) <= 1e-5 * chi2, (m, chi2, out["chi2"][m, 0])
        b = semilin.apply_LT(um, grid, n, semilin.apply_BT(pt, dd.reshape(1, ny, nx)).reshape(1, -1))
        q = semilin.apply_LT(um, grid, n, semilin.apply_BT(pt, by).reshape(1, -1)) + \
            lams[0] * semilin.apply_HtH("curvature", n, s)
        res = float(torch.linalg.norm(q - b) / torch.linalg.norm(b))
        assert res <= 1e-4, (m, res)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_max_psf_vs_oracle(semilin, prec):
    """The largest PSF (63 x 63, wider than the 40 x 36 image): direct blur path."""
    d, sigma, psf, (nx, ny, pix), G, ns = _small_case("gauss", K=63)
    G, ns = G[:2], ns[:2]
    lams = [1e-2, 1.0]
    dtype = torch.float64 if prec == "f64" else torch.float32
    out = _run(semilin, d, sigma, psf, semilin.Grid(nx, ny, pix, 2), 1.0, "curvature", dtype, G, ns, lams,
               1e-12 if prec == "f64" else 1e-7)
    ref = coracle.evaluate(G, ns, 1.0, nx, ny, pix, 2, d, sigma, psf, "curvature", lams, tol=1e-12, threads=2)
    rel = np.abs(out["chi2"] - ref["chi2"]) / ref["chi2"]
    assert rel.max() <= (1e-9 if prec == "f64" else 1e-5), rel
