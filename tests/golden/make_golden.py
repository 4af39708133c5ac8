"""Write the oracle's reference results for the full-size GPU parity tests.

Calls only the oracle and the seeded input recipes.  Run from the repository
root:  python tests/golden/make_golden.py   (about two minutes on 8 cores)

* c2_oracle.npz  -- the c2 workload (128x128 image, 64x64 nodes, curvature H,
  16 lambdas): per-lambda chi^2, ||H s||^2, solutions, CG iterations, and the
  L-curve corner, from the plain-C FP64 matrix-free CG at tol 1e-10.
* c3_sample.npz  -- three members of the c3 population (first, middle, last)
  scored against the c2 image, same quantities, for sampled checks of the
  256-member launch.
* c4_sample.npz  -- the c4 workload (200x200 image, 100x100 nodes, 21x21 PSF,
  24 lambdas): the true lens and two members of the c4 population, same
  quantities (about ten minutes on 3 cores).
* c3_full.npz    -- all 256 members of the c3 population against the c2
  image: per-lambda chi^2, ||H s||^2, iterations, status, the curvature at
  every knot and the corner k*, and the solution at every index of the
  member's corner set (the corners the L-curve gives under relative 1e-5
  perturbations of its points), packed in FP32; for the three largest grids
  also the corner solution in FP64 (about 30 minutes on 7 cores).

* c2_nsub.npz    -- the c2 lens and image modelled with 1, 3 and 4 subpixels
  per side (the other goldens use 2), 6 lambdas over 1e-3..1e1: chi^2,
  ||H s||^2, iterations, corner and corner solution (about two minutes on
  3 cores).

* c2_radial.npz  -- the c2 lens and image with a non-separable 15x15 PSF
  (synthgen.sinc_moffat_psf: elliptical Moffat times a squared radial sinc),
  so that the solve takes the direct K x K blur: chi^2, ||H s||^2,
  iterations, corner, and the solution at every lambda in FP32 (about a
  minute on 8 cores).

* c2_nearest.npz -- the c2 lens and image with nearest-neighbour source
  interpolation (Sec. 2.1), 6 lambdas over 1e-3..1e1: chi^2, ||H s||^2,
  iterations, corner and corner solution, from the numpy FP64 CG at tol
  1e-10 (about two minutes on 6 cores).

* large_envelope.npz -- the large-scale shape (synthgen.LARGE, Sec. 4):
  the oracle's 40 CGLS iterates with the blur in Fourier space (chi^2,
  carried chi^2, sum s^2, ||s||) and their spread over 24 Monte Carlo
  arithmetic runs at FP32 rounding (about five minutes).

* c2_bicubic.npz -- the same with bicubic source interpolation (Sec. 2.1;
  cubic convolution, Keys a = -1/2, over the 4 x 4 nodes about each
  subpixel's cell, nodes outside the grid zero).

`python tests/golden/make_golden.py c4` writes only c4_sample.npz;
`python tests/golden/make_golden.py c2nearest` writes only c2_nearest.npz;
`python tests/golden/make_golden.py c2bicubic` writes only c2_bicubic.npz;
`python tests/golden/make_golden.py large` writes only large_envelope.npz;
`python tests/golden/make_golden.py c2radial` writes only c2_radial.npz;
`python tests/golden/make_golden.py c3full` writes only c3_full.npz;
`python tests/golden/make_golden.py c2nsub` writes only c2_nsub.npz.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthgen  # noqa: E402
from oracle import coracle, lcurve, mock  # noqa: E402

C3_SAMPLE = (0, 128, 255)
C4_SAMPLE = (0, 511)


def run(lens, ns, w, D, threads):
    out = coracle.evaluate(lens, ns, w.half_width, w.nx, w.ny, w.pix, w.nsub_model, D["d"], D["sigma"],
                           D["psf"], w.reg, w.lambdas, tol=1e-10, want_s=True, threads=threads)
    ks = np.array([lcurve.corner(out["reg"][m], out["chi2"][m])[0] for m in range(len(lens))])
    return out, ks


def c4():
    w = synthgen.C4
    D = mock.workload_data(w)
    pop = synthgen.population(w.seed, 1024)
    lens = np.vstack([np.atleast_2d(D["lens"]), pop[np.array(C4_SAMPLE)]])
    ns = [w.ns] * lens.shape[0]
    out, ks = run(lens, ns, w, D, lens.shape[0])
    np.savez(os.path.join(HERE, "c4_sample.npz"), lens=lens, members=np.array((-1,) + C4_SAMPLE), chi2=out["chi2"],
             reg=out["reg"], iters=out["iters"], k_star=ks, s_corner=np.stack([out["s"][m, ks[m]] for m in
                                                                              range(lens.shape[0])]),
             lambdas=np.array(w.lambdas))


def c3_full(threads=7):
    w = synthgen.C2
    D = mock.workload_data(w)
    M = 256
    pop = synthgen.population(synthgen.C3.seed, M)
    grids = synthgen.member_grids(synthgen.C3.seed, M)
    out = coracle.evaluate(pop, grids, w.half_width, w.nx, w.ny, w.pix, w.nsub_model, D["d"], D["sigma"], D["psf"],
                           w.reg, w.lambdas, tol=1e-10, want_s=True, threads=threads)
    nl = len(w.lambdas)
    ks = np.zeros(M, dtype=np.int32)
    kappa = np.full((M, nl), np.nan)
    sets = np.zeros((M, nl), dtype=bool)
    for m in range(M):
        k, kap = lcurve.corner(out["reg"][m], out["chi2"][m])
        ks[m] = k
        kappa[m] = kap
        for kk in lcurve.corner_set(out["reg"][m], out["chi2"][m]):
            sets[m, kk] = True
    # packed FP32 solutions at every index of every member's corner set
    s_idx, s_pack, s_off = [], [], [0]
    for m in range(M):
        I = int(grids[m]) ** 2
        for kk in np.nonzero(sets[m])[0]:
            s_idx.append((m, kk))
            s_pack.append(out["s"][m, kk, :I].astype(np.float32))
            s_off.append(s_off[-1] + I)
    big = np.argsort(-grids, kind="stable")[:3]
    np.savez_compressed(os.path.join(HERE, "c3_full.npz"), lens=pop, ns=grids, chi2=out["chi2"], reg=out["reg"],
                        iters=out["iters"], status=out["status"], k_star=ks, kappa=kappa, corner_sets=sets,
                        s_index=np.array(s_idx, dtype=np.int32), s_off=np.array(s_off, dtype=np.int64),
                        s_f32=np.concatenate(s_pack), f64_members=big.astype(np.int32),
                        s_f64=np.stack([out["s"][m, ks[m]] for m in big]), lambdas=np.array(w.lambdas), tol=1e-10)


def c2_nsub():
    import concurrent.futures as cf
    w = synthgen.C2
    D = mock.workload_data(w)
    lams = synthgen.log_grid(1e-3, 1e1, 6)
    subs = (1, 3, 4)

    def one(n):
        return coracle.evaluate(np.atleast_2d(D["lens"]), [w.ns], w.half_width, w.nx, w.ny, w.pix, n, D["d"],
                                D["sigma"], D["psf"], w.reg, lams, tol=1e-10, want_s=True, threads=1)

    with cf.ThreadPoolExecutor(3) as ex:
        outs = list(ex.map(one, subs))
    ks = [lcurve.corner(o["reg"][0], o["chi2"][0])[0] for o in outs]
    np.savez_compressed(os.path.join(HERE, "c2_nsub.npz"), nsub=np.array(subs), lambdas=np.array(lams),
                        chi2=np.stack([o["chi2"][0] for o in outs]), reg=np.stack([o["reg"][0] for o in outs]),
                        iters=np.stack([o["iters"][0] for o in outs]), k_star=np.array(ks),
                        s_corner=np.stack([o["s"][0, k] for o, k in zip(outs, ks)]))


def c2_radial():
    import concurrent.futures as cf
    w = synthgen.C2
    D = mock.workload_data(w)
    psf = synthgen.sinc_moffat_psf(w.k_psf)

    def one(lam):
        return coracle.evaluate(np.atleast_2d(D["lens"]), [w.ns], w.half_width, w.nx, w.ny, w.pix, w.nsub_model,
                                D["d"], D["sigma"], psf, w.reg, [lam], tol=1e-10, want_s=True, threads=1)

    with cf.ThreadPoolExecutor(8) as ex:
        outs = list(ex.map(one, w.lambdas))
    chi2 = np.array([o["chi2"][0, 0] for o in outs])
    reg = np.array([o["reg"][0, 0] for o in outs])
    k = lcurve.corner(reg, chi2)[0]
    np.savez_compressed(os.path.join(HERE, "c2_radial.npz"), psf=psf, lambdas=np.array(w.lambdas), chi2=chi2,
                        reg=reg, iters=np.array([o["iters"][0, 0] for o in outs]), k_star=k,
                        s=np.stack([o["s"][0, 0] for o in outs]).astype(np.float32),
                        s_corner=outs[k]["s"][0, 0])


def c2_interp(kind):
    """c2 with another source interpolation: writes c2_<kind>.npz."""
    import concurrent.futures as cf
    from oracle import solve
    w = synthgen.C2
    D = mock.workload_data(w)
    lams = synthgen.log_grid(1e-3, 1e1, 6)
    pb = solve.Problem(D["lens"], D["d"], D["sigma"], D["psf"], w.nx, w.ny, w.pix, w.nsub_model, w.ns,
                       w.half_width, w.reg, kind)

    def one(lam):
        s, it, st = solve.solve_cg(pb, lam, tol=1e-10)
        return s, it, st

    with cf.ThreadPoolExecutor(6) as ex:
        outs = list(ex.map(one, lams))
    chi2 = np.array([pb.chi2(o[0]) for o in outs])
    reg = np.array([pb.regterm(o[0]) for o in outs])
    k = lcurve.corner(reg, chi2)[0]
    np.savez_compressed(os.path.join(HERE, f"c2_{kind}.npz"), lambdas=np.array(lams), chi2=chi2, reg=reg,
                        iters=np.array([o[1] for o in outs]), status=np.array([o[2] for o in outs]), k_star=k,
                        s=np.stack([o[0] for o in outs]))


def large_envelope():
    """Rounding envelope of the FP32 CGLS iterates at the large-scale shape
    (Sec. 4): the oracle's 40 iterates with the blur in Fourier space and
    their spread over 24 Monte Carlo arithmetic runs at FP32 rounding
    (tests/cgls_envelope.py)."""
    sys.path.insert(0, os.path.dirname(HERE))
    import cgls_envelope
    from oracle import solve
    w = synthgen.LARGE
    z = np.load(os.path.join(os.path.dirname(HERE), "data", "large.npz"))
    d = z["d"].astype(np.float64)

    def make(dd):
        return solve.Problem(z["lens"], dd, float(z["sigma"]), z["psf"], w.nx, w.ny, w.pix, w.nsub_model, w.ns,
                             w.half_width, w.reg, blur="fft")
    ref, dev, ds, corners = cgls_envelope.envelope(make, d, "f32", w.k_psf, synthgen.LARGE_ITERS, draws=24)
    np.savez_compressed(os.path.join(HERE, "large_envelope.npz"), chi2=ref["chi2"], chi2_e=ref["chi2_e"],
                        reg=ref["reg"], dev_chi2=dev["chi2"], dev_reg=dev["reg"], ds=ds,
                        corners=np.array(sorted(corners)), s_norm=np.linalg.norm(ref["s"], axis=1))


def main():
    if sys.argv[1:] == ["large"]:
        large_envelope()
        return
    if sys.argv[1:] == ["c2nearest"]:
        c2_interp("nearest")
        return
    if sys.argv[1:] == ["c2bicubic"]:
        c2_interp("bicubic")
        return
    if sys.argv[1:] == ["c2radial"]:
        c2_radial()
        return
    if sys.argv[1:] == ["c2nsub"]:
        c2_nsub()
        return
    if sys.argv[1:] == ["c4"]:
        c4()
        return
    if sys.argv[1:] == ["c3full"]:
        c3_full()
        return
    w = synthgen.C2
    D = mock.workload_data(w)
    out, ks = run(np.atleast_2d(D["lens"]), [w.ns], w, D, 1)
    np.savez(os.path.join(HERE, "c2_oracle.npz"), chi2=out["chi2"][0], reg=out["reg"][0], s=out["s"][0],
             iters=out["iters"][0], k_star=ks[0], lambdas=np.array(w.lambdas))
    pop = synthgen.population(synthgen.C3.seed, 256)
    grids = synthgen.member_grids(synthgen.C3.seed, 256)
    idx = np.array(C3_SAMPLE)
    out, ks = run(pop[idx], grids[idx], w, D, len(idx))
    s_pad = out["s"]
    np.savez(os.path.join(HERE, "c3_sample.npz"), members=idx, lens=pop[idx], ns=grids[idx], chi2=out["chi2"],
             reg=out["reg"], iters=out["iters"], k_star=ks,
             s_corner=np.stack([s_pad[m, ks[m]] for m in range(len(idx))]), lambdas=np.array(w.lambdas))


if __name__ == "__main__":
    main()
