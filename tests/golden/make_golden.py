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

`python tests/golden/make_golden.py c4` writes only c4_sample.npz.
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


def main():
    if sys.argv[1:] == ["c4"]:
        c4()
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
