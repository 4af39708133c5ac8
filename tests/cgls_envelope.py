"""Rounding envelope of the oracle's CGLS iterates (shared by the GPU tests of
the implicit-regularisation solves).

The fixed-iteration CGLS sequence is well conditioned only while it resolves
the large singular values; past that, loss of orthogonality amplifies
rounding, so two correct implementations that round differently drift apart
by far more than the unit roundoff.  A GPU value is therefore judged against
the spread of the oracle run under Monte Carlo arithmetic at the GPU's
rounding level (oracle.implicit's `perturb` hook, Parker, Pierce and Eggert
2000): unit roundoff u (2^-53 in FP64, 2^-24 in FP32) on every updated
vector, u K on the outputs of A and A^T, u sqrt(n) on the FP64 step lengths
(u in FP32), n the longer of the image and the source vectors, and u on the
data.
"""
import numpy as np

from oracle import implicit, lcurve

U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}
FLOOR = {"f64": 1e-13, "f32": 1e-7}
DRAWS = 8


def mca(prec, K, n, rng):
    """Monte Carlo arithmetic at the GPU's rounding level."""
    u = U[prec]
    rel = {"A": u * K, "AT": u * K, "vec": u, "scalar": u if prec == "f32" else u * np.sqrt(n)}

    def perturb(x, kind):
        return x * (1 + rel[kind] * rng.standard_normal(np.shape(x)))
    return perturb


def envelope(make_pb, d, prec, K, n_iter, draws=DRAWS, ref=None):
    """Oracle iterates on d, and their spread over `draws` Monte Carlo arithmetic runs.

    Returns (ref, dev, ds, corners): dev[key] the largest absolute deviation of
    chi^2 (explicit or carried) and of reg over the draws at this or any
    earlier iterate, ds the same for ||s||, corners the corner indices of the
    oracle's curve, of its 1e-5 corner set and of every draw."""
    if ref is None:
        ref = implicit.cgls_iterates(make_pb(d), n_iter)
    rng = np.random.default_rng(77)
    runs = []
    for _ in range(draws):
        pb = make_pb(d * (1 + U[prec] * rng.standard_normal(d.shape)))
        runs.append(implicit.cgls_iterates(pb, n_iter, perturb=mca(prec, K, max(pb.I, d.size), rng)))
    # largest relative deviation over the draws up to each iterate: rounding
    # effects accumulate, and a per-iterate maximum dips where the deviations
    # of all draws happen to change sign together
    rel = {"chi2": np.max([np.maximum(np.abs(r["chi2"] - ref["chi2"]), np.abs(r["chi2_e"] - ref["chi2"]))
                           for r in runs], axis=0) / np.abs(ref["chi2"]),
           "reg": np.max([np.abs(r["reg"] - ref["reg"]) for r in runs], axis=0)
           / np.maximum(np.abs(ref["reg"]), 1e-300)}
    dev = {k: np.maximum.accumulate(v) * np.abs(ref[k]) for k, v in rel.items()}
    sn = np.maximum(np.linalg.norm(ref["s"], axis=1), 1e-300)
    ds = np.maximum.accumulate(np.max([np.linalg.norm(r["s"] - ref["s"], axis=1) for r in runs], axis=0) / sn) * sn
    corners = {lcurve.corner(ref["reg"], ref["chi2"])[0]} | lcurve.corner_set(ref["reg"], ref["chi2"])
    corners |= {lcurve.corner(r["reg"], r["chi2"])[0] for r in runs}
    return ref, dev, ds, corners
