"""Regularised least-squares source solve (FP64 oracle).

Paper: minimise chi^2 (Eq. 4) plus lambda ||H s||^2; the normal equations
with Tikhonov regularisation are (M + lambda H^T H) s = F^T d (Eq. 5-7),
with default solution x0 = 0 (Eq. 13-14); CG-type solvers start from a blank
source (Sec. 2.2); H = I gives the SVD filter-factor form with
phi_i = nu_i^2/(nu_i^2+lambda) (Eqs. 15-18) and gamma = sum mu/(mu+lambda)
(Eq. 19).

Reading: the normal equations are written without the 1/sigma weights,
(L^T B^T B L + lambda H^T H) s = L^T B^T d; with one scalar sigma this only
rescales lambda by sigma^2.  chi^2 = sum_j ((B L s)_j - d_j)^2 / sigma^2 over
all J pixels.  reg = ||H s||^2.

The exact solution of that SPD system is the definition; it is computed two
independent ways: ``solve_dense`` (explicit matrices, Cholesky) and
``solve_cg`` (matrix-free Hestenes-Stiefel CG from s = 0 with the stopping
rule ||r|| <= tol ||b||).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import lens as _lens
from . import operators as _ops

# per-(member, lambda) status codes
ST_OK, ST_MAXIT, ST_EMPTY, ST_BREAKDOWN = 0, 1, 2, 3


@dataclasses.dataclass
class Problem:
    """One lens parameter set scored against one data image."""
    lens: np.ndarray       # genome (7,)
    d: np.ndarray          # data (ny, nx)
    sigma: float
    psf: np.ndarray        # (K, K)
    nx: int
    ny: int
    pix: float
    nsub: int
    ns: int
    half_width: float
    reg: str               # "identity" | "curvature"
    interp: str = "bilinear"   # "bilinear" | "nearest" | "bicubic" (Sec. 2.1)
    blur: str = "direct"       # "direct" (the sums of the definition) | "fft" (Sec. 2.2, same operator)

    def __post_init__(self):
        bx, by = _lens.trace_image(self.lens, self.nx, self.ny, self.pix, self.nsub)
        if self.interp == "bicubic":
            self.table = _ops.bicubic_table(bx, by, self.ns, self.half_width)
        else:
            self.table = _ops.bilinear_table(bx, by, self.ns, self.half_width, nearest=self.interp == "nearest")
        self.I = self.ns * self.ns

    # operators -------------------------------------------------------------
    def L(self, s):
        return _ops.apply_L(self.table, s, self.nsub).reshape(self.ny, self.nx)

    def LT(self, img):
        return _ops.apply_LT(self.table, img, self.I, self.nsub)

    def B(self, img):
        return _ops.apply_B_fft(self.psf, img) if self.blur == "fft" else _ops.apply_B(self.psf, img)

    def BT(self, img):
        return _ops.apply_BT_fft(self.psf, img) if self.blur == "fft" else _ops.apply_BT(self.psf, img)

    def F(self, s):
        return self.B(self.L(s))

    def FT(self, img):
        return self.LT(self.BT(np.asarray(img, dtype=np.float64).reshape(self.ny, self.nx)))

    def normal(self, s, lam):
        return self.FT(self.F(s)) + lam * _ops.apply_HtH(s, self.ns, self.reg)

    def rhs(self):
        return self.FT(self.d)

    # scores ----------------------------------------------------------------
    def chi2(self, s):
        r = self.F(s) - self.d
        return float((r * r).sum() / (self.sigma * self.sigma))

    def regterm(self, s):
        h = _ops.apply_H(s, self.ns, self.reg)
        return float(h @ h)

    # dense matrices ----------------------------------------------------------
    def dense_F(self):
        Lm = _ops.dense_L(self.table, self.I, self.nsub)
        cols = [_ops.apply_B(self.psf, Lm[:, i].reshape(self.ny, self.nx)).reshape(-1)
                for i in range(self.I)]
        return np.stack(cols, axis=1)

    def dense_HtH(self):
        Hm = _ops.dense_H(self.ns, self.reg)
        return Hm.T @ Hm


def solve_dense(pb: Problem, lam: float, Fm=None, G=None):
    """Exact solution via Cholesky of F^T F + lambda H^T H."""
    Fm = pb.dense_F() if Fm is None else Fm
    G = pb.dense_HtH() if G is None else G
    M = Fm.T @ Fm + lam * G
    b = Fm.T @ pb.d.reshape(-1)
    C = np.linalg.cholesky(M)
    z = np.linalg.solve(C, b)
    return np.linalg.solve(C.T, z)


def solve_cg(pb: Problem, lam: float, tol: float = 1e-10, maxit: int | None = None, b=None):
    """Matrix-free CG on the normal equations from s = 0.

    Returns (s, iterations, status).
    """
    I = pb.I
    maxit = max(10 * I, 2000) if maxit is None else maxit
    b = pb.rhs() if b is None else b
    bnorm = float(np.sqrt(b @ b))
    s = np.zeros(I)
    if bnorm == 0.0:
        return s, 0, ST_EMPTY
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    for it in range(maxit):
        if np.sqrt(rr) <= tol * bnorm:
            return s, it, ST_OK
        q = pb.normal(p, lam)
        pq = float(p @ q)
        if not pq > 0.0:
            return s, it, ST_BREAKDOWN
        alpha = rr / pq
        s += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    if np.sqrt(rr) <= tol * bnorm:
        return s, maxit, ST_OK
    return s, maxit, ST_MAXIT


def tikhonov_svd(Fm, d, lam):
    """H = I Tikhonov solution via SVD filter factors (Eqs. 16-18)."""
    U, nu, Vt = np.linalg.svd(Fm, full_matrices=False)
    phi = nu * nu / (nu * nu + lam)
    coef = phi * (U.T @ d.reshape(-1)) / nu
    return Vt.T @ coef


def dof_gamma(Fm, lam):
    """gamma = sum_i mu_i / (mu_i + lambda), mu_i eigenvalues of F^T F (Eq. 19)."""
    mu = np.linalg.eigvalsh(Fm.T @ Fm)
    mu = np.clip(mu, 0.0, None)
    return float((mu / (mu + lam)).sum())


def sweep(pb: Problem, lambdas, tol=1e-10, method="cg", maxit=None):
    """Solve every lambda; returns dict of per-lambda arrays and solutions."""
    nl = len(lambdas)
    out = dict(chi2=np.zeros(nl), reg=np.zeros(nl), iters=np.zeros(nl, dtype=np.int64),
               status=np.zeros(nl, dtype=np.int64), s=np.zeros((nl, pb.I)))
    if method == "dense":
        Fm = pb.dense_F()
        G = pb.dense_HtH()
    b = pb.rhs()
    for k, lam in enumerate(lambdas):
        if method == "dense":
            s, it, st = solve_dense(pb, lam, Fm, G), 0, ST_OK
        else:
            s, it, st = solve_cg(pb, lam, tol=tol, maxit=maxit, b=b)
        out["s"][k] = s
        out["chi2"][k] = pb.chi2(s)
        out["reg"][k] = pb.regterm(s)
        out["iters"][k] = it
        out["status"][k] = st
    return out
