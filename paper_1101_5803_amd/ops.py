"""Python entry points with the C-ABI's names (argument marshalling only).

Each function validates shapes on the host, allocates its outputs with
torch on the input's device, and calls the matching ``sl_*`` entry point
of libsemilin.so on torch's current stream.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib as L

_DT = {torch.float32: L.SL_F32, torch.float64: L.SL_F64}
_REG = {"identity": L.SL_H_IDENTITY, "curvature": L.SL_H_CURVATURE}
_INTERP = {"bilinear": L.SL_INTERP_BILINEAR, "nearest": L.SL_INTERP_NEAREST, "bicubic": L.SL_INTERP_BICUBIC}
TUNING_KEYS = ("wide_window", "lt_csr", "blur_direct", "plain_cg", "pc_theta_pct", "heavy")


@dataclasses.dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    pix: float
    nsub: int

    def c(self):
        return L.ImageGrid(self.nx, self.ny, self.pix, self.nsub)

    @property
    def J(self):
        return self.nx * self.ny


def _dev_check(*ts):
    for t in ts:
        if not (isinstance(t, torch.Tensor) and t.is_cuda):
            raise L.SemilinError("inputs must be CUDA (HIP) tensors")


def lens_trace(lens: torch.Tensor, grid: Grid, ns, half_width: float) -> torch.Tensor:
    """(u, v) grid coordinates of every subpixel, NaN outside; (M, J*n^2, 2) FP64."""
    _dev_check(lens)
    lens = lens.to(torch.float64).contiguous()
    M = lens.shape[0]
    ns = list(ns)
    uv = torch.empty((M, grid.J * grid.nsub ** 2, 2), dtype=torch.float64, device=lens.device)
    g = grid.c()
    L.check(L.lib().sl_lens_trace(L.ptr(lens), M, ctypes.byref(g), L.i32_array(ns), half_width,
                                  L.ptr(uv), L.stream_handle()), "sl_lens_trace")
    return uv


def apply_L(uv: torch.Tensor, grid: Grid, ns, s: torch.Tensor) -> torch.Tensor:
    """Unblurred lensed images (M, J) of packed sources s."""
    _dev_check(uv, s)
    ns = list(ns)
    out = torch.empty((len(ns), grid.J), dtype=s.dtype, device=s.device)
    g = grid.c()
    L.check(L.lib().sl_apply_L(_DT[s.dtype], L.ptr(uv), len(ns), ctypes.byref(g), L.i32_array(ns),
                               L.ptr(s.contiguous()), L.ptr(out), L.stream_handle()), "sl_apply_L")
    return out


def apply_LT(uv: torch.Tensor, grid: Grid, ns, img: torch.Tensor) -> torch.Tensor:
    """Packed L^T of images (M, J)."""
    _dev_check(uv, img)
    ns = list(ns)
    out = torch.empty(int(sum(n * n for n in ns)), dtype=img.dtype, device=img.device)
    g = grid.c()
    L.check(L.lib().sl_apply_LT(_DT[img.dtype], L.ptr(uv), len(ns), ctypes.byref(g), L.i32_array(ns),
                                L.ptr(img.contiguous()), L.ptr(out), L.stream_handle()), "sl_apply_LT")
    return out


def apply_LT_ordered(uv: torch.Tensor, grid: Grid, ns, img: torch.Tensor) -> torch.Tensor:
    """Packed L^T of images (M, J) summed in a fixed order (bitwise reproducible)."""
    _dev_check(uv, img)
    ns = list(ns)
    out = torch.empty(int(sum(n * n for n in ns)), dtype=img.dtype, device=img.device)
    g = grid.c()
    nsa = L.i32_array(ns)
    need = int(L.lib().sl_apply_LT_ordered_workspace_size(ctypes.byref(g), nsa, len(ns)))
    if need == 0:
        raise L.SemilinError(L.lib().sl_last_error().decode())
    ws = torch.empty(need, dtype=torch.uint8, device=img.device)
    L.check(L.lib().sl_apply_LT_ordered(_DT[img.dtype], L.ptr(uv), len(ns), ctypes.byref(g), nsa,
                                        L.ptr(img.contiguous()), L.ptr(out), L.ptr(ws), need, L.stream_handle()),
            "sl_apply_LT_ordered")
    return out


def _blur(name, psf, x):
    _dev_check(psf, x)
    psf = psf.to(torch.float64).contiguous()
    x = x.contiguous()
    ny, nx = x.shape[-2:]
    n = x.numel() // (nx * ny)
    out = torch.empty_like(x)
    L.check(getattr(L.lib(), name)(_DT[x.dtype], nx, ny, n, L.ptr(psf), psf.shape[0], L.ptr(x), L.ptr(out),
                                   L.stream_handle()), name)
    return out


def apply_B(psf: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """PSF convolution (zero padding, same size) of images (..., ny, nx)."""
    return _blur("sl_apply_B", psf, x)


def apply_BT(psf: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Correlation with the PSF: the transpose of apply_B."""
    return _blur("sl_apply_BT", psf, x)


def fft_blur(psf: torch.Tensor, x: torch.Tensor, transpose: bool = False, workspace: torch.Tensor | None = None):
    """apply_B (or, transpose, apply_BT) of one image (ny, nx) computed in Fourier space (sl_fft_blur),
    for PSFs up to 129 x 129."""
    _dev_check(psf, x)
    psf = psf.to(torch.float64).contiguous()
    x = x.contiguous()
    if x.dim() != 2:
        raise L.SemilinError("fft_blur takes one image (ny, nx)")
    ny, nx = x.shape
    dt = _DT[x.dtype]
    need = L.lib().sl_fft_blur_workspace_size(dt, nx, ny, psf.shape[0])
    if need == 0:
        raise L.SemilinError(L.lib().sl_last_error().decode())
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(int(need), dtype=torch.uint8, device=x.device)
    out = torch.empty_like(x)
    L.check(L.lib().sl_fft_blur(dt, int(bool(transpose)), nx, ny, L.ptr(psf), psf.shape[0], L.ptr(x), L.ptr(out),
                                L.ptr(workspace), workspace.numel(), L.stream_handle()), "sl_fft_blur")
    return out


def apply_HtH(reg: str, ns, s: torch.Tensor) -> torch.Tensor:
    _dev_check(s)
    ns = list(ns)
    out = torch.empty_like(s)
    L.check(L.lib().sl_apply_HtH(_DT[s.dtype], _REG[reg], len(ns), L.i32_array(ns), L.ptr(s.contiguous()),
                                 L.ptr(out), L.stream_handle()), "sl_apply_HtH")
    return out


def profile_enable(on: bool = True) -> None:
    """Record HIP events around every persistent solve kernel (clears the record)."""
    L.check(L.lib().sl_profile_enable(1 if on else 0), "sl_profile_enable")


def profile_solve_ms():
    """(summed milliseconds, launches) of the recorded solve kernels; synchronises."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int32(0)
    L.check(L.lib().sl_profile_solve_ms(ctypes.byref(ms), ctypes.byref(n)), "sl_profile_solve_ms")
    return float(ms.value), int(n.value)


def lcurve_corner(reg, chi2):
    """Host L-curve corner: returns (k_star, kappa ndarray)."""
    reg = np.ascontiguousarray(reg, dtype=np.float64)
    chi2 = np.ascontiguousarray(chi2, dtype=np.float64)
    n = reg.size
    k = ctypes.c_int32(0)
    kap = np.zeros(n)
    dp = ctypes.POINTER(ctypes.c_double)
    L.check(L.lib().sl_lcurve_corner(reg.ctypes.data_as(dp), chi2.ctypes.data_as(dp), n, ctypes.byref(k),
                                     kap.ctypes.data_as(dp)), "sl_lcurve_corner")
    return int(k.value), kap


class Plan:
    """A captured solve (sl_plan_*): launch() replays it on torch's current stream."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep   # buffers whose addresses the graph holds
        self.out = keep[3]

    def launch(self):
        if not self._h:
            raise L.SemilinError("plan destroyed")
        L.check(L.lib().sl_plan_launch(self._h, L.stream_handle()), "sl_plan_launch")
        return self.out

    def close(self):
        if self._h:
            torch.cuda.synchronize()
            L.check(L.lib().sl_plan_destroy(self._h), "sl_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Batched semilinear solve against one data image (sl_solve_semilinear).

    Holds the problem description and a workspace tensor sized for
    (max_ns, n_members, n_lambda); the workspace is allocated by torch once
    and grown on demand.
    """

    def __init__(self, d: torch.Tensor, sigma: float, psf: torch.Tensor, grid: Grid, half_width: float,
                 reg: str = "curvature", dtype: torch.dtype = torch.float32, interp: str = "bilinear"):
        _dev_check(d, psf)
        self.d = d.to(torch.float64).contiguous().reshape(-1)
        self.psf = psf.to(torch.float64).contiguous()
        if self.d.numel() != grid.J:
            raise L.SemilinError("data image does not match the grid")
        self.grid = grid
        self.sigma = float(sigma)
        self.half_width = float(half_width)
        self.reg = reg
        self.dtype = dtype
        self.device = d.device
        self._ws = None
        self._cws = None   # workspace of chi2_sources
        self._lws = None   # workspace of solve_large
        # launch hint: a PSF whose second singular value is not negligible is not rank 1, so the solve
        # launches only the direct blur form (the device's own rank-1 test decides every other case)
        sv = np.linalg.svd(self.psf.cpu().numpy(), compute_uv=False)
        general = int(sv.size > 1 and sv[1] > 1e-8 * sv[0])
        self._pb = L.Problem(grid.c(), ctypes.c_void_p(self.d.data_ptr()), self.sigma,
                             ctypes.c_void_p(self.psf.data_ptr()), self.psf.shape[0], self.half_width,
                             _REG[reg], _DT[dtype], general, _INTERP[interp])

    def workspace_bytes(self, max_ns: int, n_members: int, n_lambda: int) -> int:
        n = L.lib().sl_solve_workspace_size(ctypes.byref(self._pb), max_ns, n_members, n_lambda)
        if n == 0:
            raise L.SemilinError(L.lib().sl_last_error().decode())
        return int(n)

    def workspace(self, max_ns, n_members, n_lambda):
        need = self.workspace_bytes(max_ns, n_members, n_lambda)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def alloc_result(self, ns_total: int, n_members: int, n_lambda: int):
        dev = self.device
        return dict(
            s_corner=torch.empty(max(ns_total, 1), dtype=torch.float64, device=dev),
            s_off=torch.empty(n_members + 1, dtype=torch.int64, device=dev),
            chi2=torch.empty((n_members, n_lambda), dtype=torch.float64, device=dev),
            reg=torch.empty((n_members, n_lambda), dtype=torch.float64, device=dev),
            iters=torch.empty((n_members, n_lambda), dtype=torch.int32, device=dev),
            status=torch.empty((n_members, n_lambda), dtype=torch.int32, device=dev),
            k_star=torch.empty(n_members, dtype=torch.int32, device=dev),
            corner_status=torch.empty(n_members, dtype=torch.int32, device=dev),
            dof=torch.empty(n_members, dtype=torch.float64, device=dev),
        )

    def member_info(self, max_ns: int, n_members: int, n_lambda: int) -> np.ndarray:
        """(n_members, 10) int32 table {ns, I, M, r0, r1, c0, c1, status, Lt layout, LDS frame} of the last solve."""
        info = np.zeros((n_members, 10), dtype=np.int32)
        L.check(L.lib().sl_solve_member_info(ctypes.byref(self._pb), max_ns, n_members, n_lambda, L.ptr(self._ws),
                                             info.ctypes.data_as(ctypes.c_void_p)), "sl_solve_member_info")
        return info

    def _args(self, lens, ns, lambdas, tol, maxit, max_ns, out, tuning, mc_noise=None):
        _dev_check(lens, ns)
        if lens.dtype != torch.float64 or ns.dtype != torch.int32 or not lens.is_contiguous() \
                or not ns.is_contiguous():
            raise L.SemilinError("lens must be contiguous float64 (M, 7) and ns contiguous int32 (M,)")
        M = lens.shape[0]
        lam = [float(x) for x in lambdas]
        if max_ns is None:
            max_ns = int(ns.max().item())
        ws = self.workspace(max_ns, M, len(lam))
        if out is None:
            out = self.alloc_result(M * max_ns * max_ns, M, len(lam))
        res = L.Result(*[ctypes.c_void_p(out[k].data_ptr()) for k in
                         ("s_corner", "s_off", "chi2", "reg", "iters", "status", "k_star", "corner_status", "dof")])
        tun = None
        if tuning is not None:
            tun = L.Tuning(*[int(tuning.get(k, 0)) for k in TUNING_KEYS])
        noise = None
        if mc_noise is not None:
            _dev_check(mc_noise)
            if mc_noise.dtype != torch.float64 or not mc_noise.is_contiguous() or mc_noise.numel() != self.grid.J:
                raise L.SemilinError("mc_noise must be a contiguous float64 device tensor of ny*nx draws")
            noise = ctypes.c_void_p(mc_noise.data_ptr())
        opts = L.SolveOpts(float(tol), int(maxit), ctypes.pointer(tun) if tun is not None else None, noise)
        return M, lam, int(max_ns), ws, out, res, opts, tun

    def solve_semilinear(self, lens: torch.Tensor, ns: torch.Tensor, lambdas, tol=1e-7, maxit=4000,
                         max_ns: int | None = None, out=None, tuning: dict | None = None,
                         mc_noise: torch.Tensor | None = None):
        """Run the batched solve; returns the result dict of device tensors.

        lens (M, 7) FP64 and ns (M,) int32 on the device; lambdas a host
        sequence.  ``max_ns`` bounds ns (defaults to ns.max(), which syncs).
        ``tuning`` (dict with keys wide_window, lt_csr, blur_direct, plain_cg)
        forces a kernel variant; None takes the autotuner's choice, if any.
        plain_cg = 1 turns the spectral preconditioner of the FP32 curvature
        solve off.  ``mc_noise`` (ny*nx FP64 Gaussian draws on the device)
        adds the Monte Carlo degrees of freedom at each corner to out["dof"].
        """
        lens = lens.to(torch.float64).contiguous()
        ns = ns.to(torch.int32).contiguous()
        M, lam, max_ns, ws, out, res, opts, _tun = self._args(lens, ns, lambdas, tol, maxit, max_ns, out, tuning,
                                                              mc_noise)
        L.check(L.lib().sl_solve_semilinear(ctypes.byref(self._pb), L.ptr(lens), L.ptr(ns), max_ns, M,
                                            L.f64_array(lam), len(lam), ctypes.byref(opts), L.ptr(ws),
                                            ws.numel(), ctypes.byref(res), L.stream_handle()),
                "sl_solve_semilinear")
        return out

    def solve_implicit(self, lens: torch.Tensor, ns: torch.Tensor, n_iter: int = 40, max_ns: int | None = None,
                       out=None, mc_noise: torch.Tensor | None = None):
        """Implicit regularisation (sl_solve_implicit): n_iter CGLS iterations per member with no lambda and the
        L-curve over the iterates; out["chi2"], out["reg"] are (M, n_iter), k_star the corner iterate index.
        ``mc_noise`` (FP64 solves only: ny*nx FP64 Gaussian draws on the device) adds the lockstep Monte Carlo
        degrees-of-freedom system; out["dof"][m] is then its estimate at the member's corner iterate."""
        lens = lens.to(torch.float64).contiguous()
        ns = ns.to(torch.int32).contiguous()
        M, lam, max_ns, ws, out, res, opts, _tun = self._args(lens, ns, list(range(1, n_iter + 1)), 0.0, 1, max_ns,
                                                              out, None, mc_noise)
        L.check(L.lib().sl_solve_implicit(ctypes.byref(self._pb), L.ptr(lens), L.ptr(ns), max_ns, M, int(n_iter),
                                          ctypes.byref(opts), L.ptr(ws), ws.numel(), ctypes.byref(res),
                                          L.stream_handle()), "sl_solve_implicit")
        return out

    def solve_large(self, lens, ns: int, n_iter: int = 40, out=None):
        """One lens on a large image (sl_solve_large): n_iter CGLS iterations with the blur in Fourier space,
        the L-curve over the iterates; the result dict of solve_implicit with one member."""
        lens = torch.as_tensor(lens, dtype=torch.float64, device=self.device).contiguous().reshape(-1)
        if lens.numel() != 7:
            raise L.SemilinError("lens must hold the 7 lens parameters")
        need = L.lib().sl_solve_large_workspace_size(ctypes.byref(self._pb), int(ns), int(n_iter))
        if need == 0:
            raise L.SemilinError(L.lib().sl_last_error().decode())
        if self._lws is None or self._lws.numel() < need:
            self._lws = torch.empty(int(need), dtype=torch.uint8, device=self.device)
        if out is None:
            out = self.alloc_result(ns * ns, 1, n_iter)
        res = L.Result(*[ctypes.c_void_p(out[k].data_ptr()) for k in
                         ("s_corner", "s_off", "chi2", "reg", "iters", "status", "k_star", "corner_status", "dof")])
        L.check(L.lib().sl_solve_large(ctypes.byref(self._pb), L.ptr(lens), int(ns), int(n_iter), L.ptr(self._lws),
                                       self._lws.numel(), ctypes.byref(res), L.stream_handle()), "sl_solve_large")
        return out

    def chi2_sources(self, lens, ns: int, sources: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Image chi^2 of candidate sources for one lens (sl_chi2_sources): sources is a contiguous
        float64 device tensor (P, ns*ns); returns (P,) float64 on the device."""
        _dev_check(sources)
        lens = torch.as_tensor(lens, dtype=torch.float64, device=self.device).contiguous().reshape(-1)
        if lens.numel() != 7:
            raise L.SemilinError("lens must hold the 7 lens parameters")
        if sources.dtype != torch.float64 or not sources.is_contiguous() or sources.dim() != 2 \
                or sources.shape[1] != ns * ns:
            raise L.SemilinError("sources must be a contiguous float64 device tensor (P, ns*ns)")
        P = sources.shape[0]
        if out is None:
            out = torch.empty(P, dtype=torch.float64, device=self.device)
        need = L.lib().sl_chi2_sources_workspace_size(ctypes.byref(self._pb), int(ns))
        if need == 0:
            raise L.SemilinError(L.lib().sl_last_error().decode())
        if self._cws is None or self._cws.numel() < need:
            self._cws = torch.empty(int(need), dtype=torch.uint8, device=self.device)
        L.check(L.lib().sl_chi2_sources(ctypes.byref(self._pb), L.ptr(lens), int(ns), L.ptr(sources), P,
                                        L.ptr(self._cws), self._cws.numel(), L.ptr(out), L.stream_handle()),
                "sl_chi2_sources")
        return out

    def autotune(self, lens: torch.Tensor, ns: torch.Tensor, lambdas, tol=1e-7, maxit=4000,
                 max_ns: int | None = None, out=None):
        """Time every kernel variant on this problem (synchronous); returns (best dict, ms per variant, out).

        Later solves of the same signature with tuning=None use the best variant.
        """
        lens = lens.to(torch.float64).contiguous()
        ns = ns.to(torch.int32).contiguous()
        M, lam, max_ns, ws, out, res, opts, _tun = self._args(lens, ns, lambdas, tol, maxit, max_ns, out, None)
        best = L.Tuning()
        ms = (ctypes.c_double * L.N_VARIANTS)()
        L.check(L.lib().sl_solve_autotune(ctypes.byref(self._pb), L.ptr(lens), L.ptr(ns), max_ns, M,
                                          L.f64_array(lam), len(lam), ctypes.byref(opts), L.ptr(ws), ws.numel(),
                                          ctypes.byref(res), L.stream_handle(), ctypes.byref(best), ms),
                "sl_solve_autotune")
        return ({k: getattr(best, k) for k in TUNING_KEYS}, list(ms), out)

    def plan(self, lens: torch.Tensor, ns: torch.Tensor, lambdas, tol=1e-7, maxit=4000,
             max_ns: int | None = None, out=None, tuning: dict | None = None) -> "Plan":
        """Capture the solve on these buffers into a HIP graph (sl_plan_create).

        lens and ns must be contiguous device tensors of the right dtypes: the
        graph keeps their addresses, and each replay reads their contents.
        """
        M, lam, max_ns, ws, out, res, opts, _tun = self._args(lens, ns, lambdas, tol, maxit, max_ns, out, tuning)
        h = ctypes.c_void_p()
        L.check(L.lib().sl_plan_create(ctypes.byref(self._pb), L.ptr(lens), L.ptr(ns), max_ns, M, L.f64_array(lam),
                                       len(lam), ctypes.byref(opts), L.ptr(ws), ws.numel(), ctypes.byref(res),
                                       ctypes.byref(h)), "sl_plan_create")
        return Plan(h, keep=(lens, ns, ws, out, self))


# ---------------------------------------------------------------- surrogate MLP
MLP_SHAPES = [((7, 256), (256,)), ((256, 256), (256,)), ((256, 1), (1,))]
_mlp_ws = {}


def mlp_pack(weights, device=None) -> torch.Tensor:
    """[(W0, b0), (W1, b1), (W2, b2)] (W[in][out]) -> packed FP32 parameter vector."""
    parts = []
    for (W, b), (sw, sb) in zip(weights, MLP_SHAPES):
        W = torch.as_tensor(np.asarray(W, dtype=np.float32)).reshape(sw)
        b = torch.as_tensor(np.asarray(b, dtype=np.float32)).reshape(sb)
        parts += [W.reshape(-1), b.reshape(-1)]
    v = torch.cat(parts)
    assert v.numel() == L.MLP_NPARAM
    return v.to(device) if device is not None else v


def mlp_unpack(vec) -> list:
    """Packed parameter vector -> [(W0, b0), (W1, b1), (W2, b2)] as FP64 numpy arrays."""
    v = vec.detach().cpu().to(torch.float64).numpy() if isinstance(vec, torch.Tensor) else np.asarray(vec)
    out, o = [], 0
    for sw, sb in MLP_SHAPES:
        nw, nb = sw[0] * sw[1], sb[0]
        out.append((v[o:o + nw].reshape(sw), v[o + nw:o + nw + nb]))
        o += nw + nb
    return out


def _mlp_workspace(batch: int, device) -> torch.Tensor:
    need = int(L.lib().sl_mlp_workspace_size(int(batch)))
    if need == 0:
        raise L.SemilinError(L.lib().sl_last_error().decode())
    key = str(device)
    ws = _mlp_ws.get(key)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
        _mlp_ws[key] = ws
    return ws


def _mlp_check(params, x):
    _dev_check(params, x)
    if params.dtype != torch.float32 or params.numel() != L.MLP_NPARAM or not params.is_contiguous():
        raise L.SemilinError(f"params must be a contiguous float32 vector of {L.MLP_NPARAM}")
    if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != 7:
        raise L.SemilinError("x must be float32 of shape (batch, 7)")


def mlp_forward(params: torch.Tensor, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Surrogate predictions y (batch,) FP32 for inputs x (batch, 7)."""
    _mlp_check(params, x)
    x = x.contiguous()
    B = x.shape[0]
    y = out if out is not None else torch.empty(B, dtype=torch.float32, device=x.device)
    ws = _mlp_workspace(B, x.device)
    L.check(L.lib().sl_mlp_forward(L.ptr(params), L.ptr(x), B, L.ptr(y), L.ptr(ws), L.stream_handle()),
            "sl_mlp_forward")
    return y


def mlp_forward_noalloc(params: torch.Tensor, x: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """mlp_forward through sl_mlp_forward_noalloc: the library allocates nothing (its scratch is a static
    device array); the caller passes the output buffer.  Overlapping calls on one GPU race."""
    _mlp_check(params, x)
    _dev_check(out)
    x = x.contiguous()
    B = x.shape[0]
    if out.dtype != torch.float32 or out.numel() < B or not out.is_contiguous():
        raise L.SemilinError("out must be a contiguous float32 tensor of at least batch elements")
    L.check(L.lib().sl_mlp_forward_noalloc(L.ptr(params), L.ptr(x), B, L.ptr(out), L.stream_handle()),
            "sl_mlp_forward_noalloc")
    return out


def mlp_train_step(params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, x: torch.Tensor, y: torch.Tensor,
                   lr: float, t: int, grads: torch.Tensor | None = None, loss: torch.Tensor | None = None) -> None:
    """One in-place Adam step of params (and moments m, v) on the batch's MSE."""
    _mlp_check(params, x)
    _dev_check(m, v, y)
    x = x.contiguous()
    y = y.to(torch.float32).contiguous()
    B = x.shape[0]
    if y.numel() != B:
        raise L.SemilinError("y must hold one target per row of x")
    ws = _mlp_workspace(B, x.device)
    L.check(L.lib().sl_mlp_train_step(L.ptr(params), L.ptr(m), L.ptr(v), L.ptr(x), L.ptr(y), B, float(lr), int(t),
                                      L.ptr(grads), L.ptr(loss), L.ptr(ws), L.stream_handle()),
            "sl_mlp_train_step")
