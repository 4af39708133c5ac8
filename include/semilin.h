/*
 * semilin.h -- C ABI of the MI355X (gfx950) matrix-free semilinear lens solver.
 *
 * The library scores lens parameter sets the way Rogers & Fiege (2011) do:
 * image pixels, split into n x n subpixels, are traced to the source plane
 * through an analytic lens (thin-lens mapping, Sec. 2 Eq. 1; SIE deflection,
 * Sec. 2.3 Eqs. 10-11; SIS, Sec. 4; plus uniform external shear, which the
 * paper does not use); a pixelated source s is interpolated bilinearly at the
 * traced positions and averaged over subpixels (L, Sec. 2.1-2.2), blurred by
 * the PSF (B, Sec. 2.2); the regularised normal equations
 *     (L^T B^T B L + lambda H^T H) s = L^T B^T d          (Eq. 7, Eq. 13-14, x0 = 0)
 * are solved by conjugate gradients from a blank source (Sec. 2.2) for every
 * lambda of a grid; chi^2 (Eq. 4) and ||H s||^2 form the L-curve whose point
 * of maximum curvature (Sec. 2.6, Eq. 20) gives the lens's fitness.
 *
 * Conventions shared by every call:
 *  - lengths in arcsec, angles in radians, arrays row-major;
 *  - image pixel (r, c), index j = r*nx + c, has centre
 *    ((c-(nx-1)/2) pix, (r-(ny-1)/2) pix); its subpixel k = sr*nsub + sc sits
 *    at offset (((sc+1/2)/nsub - 1/2) pix, ((sr+1/2)/nsub - 1/2) pix);
 *  - a member's source grid has ns x ns nodes at (-R + c h, -R + r h),
 *    h = 2R/(ns-1), node i = r*ns + c; packed source vectors of several
 *    members are concatenated in member order (member m starts at
 *    sum_{m'<m} ns_{m'}^2);
 *  - a subpixel traced to grid coordinates (u, v) is inside iff
 *    0 <= u, v <= ns-1; it then spreads bilinear weights, each divided by
 *    nsub^2, over the 4 nodes of cell (min(floor v, ns-2), min(floor u, ns-2));
 *    outside subpixels contribute nothing;
 *  - B is the zero-padded "same"-size convolution with a K x K PSF (K odd)
 *    centred at (K-1)/2; B^T is the matching correlation;
 *  - H is the identity or the stacked Dirichlet second differences along x
 *    and along y (one row per node per axis);
 *  - lens genome = 7 doubles (theta_E, q, pa, gamma, gamma_pa, x0, y0):
 *    Einstein radius, axis ratio in (0,1], mass major-axis angle from +x,
 *    external shear strength and angle, lens centre.
 *
 * Ownership: every array is allocated by the caller.  "device" arrays live
 * in GPU memory of the current HIP device; "host" arrays in host memory and
 * are only read during the call.  The library allocates no memory the caller
 * sees; the solver's scratch comes from a caller workspace sized by
 * sl_solve_workspace_size().  Calls are asynchronous on `stream` (a
 * hipStream_t; NULL = default stream) unless stated otherwise; kernel faults
 * surface at the next synchronisation.
 *
 * Errors: SL_OK (0) on success; SL_EINVAL (-1) for a bad host-side argument,
 * detected before any launch; SL_EHIP (-2) for a HIP runtime error; SL_ENOIMPL
 * (-3) for a size beyond the compiled limits.  sl_last_error() returns a
 * thread-local message about the last non-zero return.  Per-member problems
 * that live in device data (a bad genome, a source grid out of range, a lens
 * that maps no ray onto the grid, CG hitting maxit) are reported through the
 * per-(member, lambda) status array, never through the return code.
 */
#ifndef SEMILIN_H
#define SEMILIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SL_OK = 0, SL_EINVAL = -1, SL_EHIP = -2, SL_ENOIMPL = -3 };
enum { SL_INTERP_BILINEAR = 0, SL_INTERP_NEAREST = 1, SL_INTERP_BICUBIC = 2 };
enum { SL_F32 = 0, SL_F64 = 1 };                  /* arithmetic of the bulk work */
enum { SL_H_IDENTITY = 0, SL_H_CURVATURE = 1 };   /* regularisation operator H */

/* per-(member, lambda) status */
enum {
  SL_ST_OK = 0,        /* ||r|| <= tol ||b|| reached */
  SL_ST_MAXIT = 1,     /* stopped at maxit; results written from the last iterate */
  SL_ST_EMPTY = 2,     /* no subpixel maps onto the grid: b = 0, s = 0 */
  SL_ST_BREAKDOWN = 3, /* <p, A p> <= 0 (loss of positive definiteness) */
  SL_ST_INVALID = 4,   /* bad genome (non-finite, q outside (0,1], theta_E < 0) or ns out of range */
  SL_ST_LCURVE = 5     /* (k_star status) fewer than 4 distinct L-curve points; k* = 0 */
};

#define SL_MAX_LAMBDA 64   /* longest lambda grid */
#define SL_MAX_PSF 63      /* largest PSF side K */
#define SL_MAX_NSUB 4      /* largest subpixel count per side */

typedef struct {
  int nx, ny;     /* image columns and rows */
  double pix;     /* arcsec per pixel */
  int nsub;       /* n: subpixels per pixel side (1..SL_MAX_NSUB) */
} sl_image_grid;

/*
 * Lens tracing (Sec. 2 Eq. 1, Eqs. 10-11, Sec. 2.2 subpixels).
 * lens: device double[n_members*7] genomes.  ns: host int32[n_members]
 * source-grid sides (>= 2).  uv: device double[n_members][ny*nx*nsub^2][2],
 * the grid coordinates (u, v) = ((beta_x+R)/h, (beta_y+R)/h) of every
 * subpixel, written NaN for subpixels outside the grid.  Computed in FP64.
 */
int sl_lens_trace(const double* lens, int n_members, const sl_image_grid* img,
                  const int32_t* ns, double half_width, double* uv, void* stream);

/*
 * L: unblurred lensed image of packed sources (Sec. 2.1, Sec. 2.2).
 * dtype SL_F32 -> s, img_out are float; SL_F64 -> double.
 * uv: as written by sl_lens_trace.  s: device packed sources.
 * img_out: device [n_members][ny*nx], overwritten.
 */
int sl_apply_L(int dtype, const double* uv, int n_members, const sl_image_grid* img,
               const int32_t* ns, const void* s, void* img_out, void* stream);

/*
 * L^T: exact transpose of sl_apply_L (Sec. 2.2).  img_in: device
 * [n_members][ny*nx]; s_out: device packed sources, overwritten.
 * Accumulates with atomics, so the summation order is not fixed
 * (sl_apply_LT_ordered below is the reproducible form).
 */
int sl_apply_LT(int dtype, const double* uv, int n_members, const sl_image_grid* img,
                const int32_t* ns, const void* img_in, void* s_out, void* stream);

/*
 * L^T in a fixed summation order: the same operator as sl_apply_LT, with
 * every node's terms added in ascending (pixel, subpixel, corner) order --
 * the order of a sequential scatter over the image -- so the result is
 * bitwise reproducible.  The terms of each node are found by a counting sort
 * in `workspace` (device, 4-byte aligned, at least
 * sl_apply_LT_ordered_workspace_size(img, ns, n_members) bytes; contents
 * need not be initialised; calls sharing it must not overlap).  Other
 * arguments as sl_apply_LT.  The workspace-size query returns 0 for invalid
 * arguments.
 */
size_t sl_apply_LT_ordered_workspace_size(const sl_image_grid* img, const int32_t* ns, int n_members);
int sl_apply_LT_ordered(int dtype, const double* uv, int n_members, const sl_image_grid* img,
                        const int32_t* ns, const void* img_in, void* s_out, void* workspace,
                        size_t workspace_bytes, void* stream);

/*
 * B and B^T on n_images images of ny x nx (Sec. 2.2; zero padding).
 * psf: device double[k*k], k odd <= SL_MAX_PSF.  in/out: device, distinct.
 */
int sl_apply_B(int dtype, int nx, int ny, int n_images, const double* psf, int k,
               const void* in, void* out, void* stream);
int sl_apply_BT(int dtype, int nx, int ny, int n_images, const double* psf, int k,
                const void* in, void* out, void* stream);

/*
 * H^T H on packed sources (Eq. 7).  reg: SL_H_IDENTITY or SL_H_CURVATURE.
 */
int sl_apply_HtH(int dtype, int reg, int n_members, const int32_t* ns, const void* s, void* out,
                 void* stream);

typedef struct {
  sl_image_grid img;
  const double* d;     /* device double[ny*nx]: data image */
  double sigma;        /* noise standard deviation (one value for all pixels) */
  const double* psf;   /* device double[k*k], sums to one */
  int k;               /* PSF side, odd, <= SL_MAX_PSF */
  double half_width;   /* R: every member's grid spans +-R */
  int reg;             /* SL_H_IDENTITY | SL_H_CURVATURE */
  int dtype;           /* SL_F32: FP32 bulk, FP64 inner products / chi^2 / L-curve;
                          SL_F64: FP64 throughout */
  int psf_general;     /* 0: the solve tests the PSF for rank 1 on the device and launches
                          the banded and the direct form of each persistent kernel, the one
                          that does not apply returning at entry; 1: the caller states that
                          the PSF is not rank 1, and only the direct form is launched (as
                          with sl_tuning.blur_direct; correct for any PSF, slower for a
                          separable one) */
  int interp;          /* source interpolation in L (Sec. 2.1): SL_INTERP_BILINEAR (the four
                          nodes around a subpixel, weighted), SL_INTERP_NEAREST (the
                          nearest node, weight 1; a fraction of exactly 1/2 rounds up), or
                          SL_INTERP_BICUBIC (cubic convolution, Keys a = -1/2, over the
                          4 x 4 nodes about the subpixel's cell; nodes outside the grid
                          are zero; L then has up to 16 n^2 entries per pixel, the
                          transposed operator four times the bilinear storage, and the
                          solve takes the direct blur form as with psf_general = 1) */
} sl_problem;

/*
 * Kernel variant of the batched solve.  Every variant computes the same
 * quantities; they differ only in the order of floating-point sums, so their
 * results agree to rounding.  All zero is the default variant.
 */
typedef struct {
  int wide_window;     /* 1: banded blur window one compiled size above the minimum */
  int lt_csr;          /* 1: transposed trace operator in CSR rows instead of sliced ELL */
  int blur_direct;     /* 1: direct K x K blur even when the PSF is separable */
  int plain_cg;        /* 1: plain CG even where the spectral preconditioner applies (see
                          sl_solve_semilinear); not part of the autotuner's search */
  int pc_theta_pct;    /* preconditioner threshold theta in percent: items with
                          lambda >= theta c take it (see sl_solve_semilinear); 0: 15 */
  int heavy;           /* count of each member's smallest lambdas queued ahead of the
                          other lambdas (their solves take the most iterations); 0: 4 */
} sl_tuning;

typedef struct {
  double tol;          /* stop when ||r|| <= tol ||b|| */
  int maxit;           /* iteration cap per (member, lambda) */
  const sl_tuning* tuning; /* nullable: NULL takes the autotuner's choice for this problem
                              signature when sl_solve_autotune has made one in this
                              process, else the default variant */
  const double* mc_noise;  /* nullable; device double[ny*nx]: the zero-mean, unit-variance
                              Gaussian draws bhat of the Monte Carlo estimate of the effective
                              degrees of freedom (Sec. 2.5).  When given, the solve also writes
                              sl_result.dof (see sl_solve_semilinear). */
} sl_solve_opts;

typedef struct {
  double* s_corner;    /* device double[sum_m ns_m^2]: solution at each member's corner */
  int64_t* s_off;      /* device int64[n_members+1]: start of each member in s_corner */
  double* chi2;        /* device double[n_members*n_lambda] */
  double* reg;         /* device double[n_members*n_lambda]: ||H s||^2 */
  int32_t* iters;      /* device int32[n_members*n_lambda] */
  int32_t* status;     /* device int32[n_members*n_lambda], SL_ST_* */
  int32_t* k_star;     /* device int32[n_members]: L-curve corner index */
  int32_t* corner_status; /* device int32[n_members]: SL_ST_OK, _EMPTY, _INVALID or _LCURVE; or
                              SL_ST_MAXIT / SL_ST_BREAKDOWN when some lambda of the member's curve
                              did not converge (k_star is still its curve's corner) */
  double* dof;         /* device double[n_members], written when opts->mc_noise is given (else
                          unused, may be NULL): the Monte Carlo degrees of freedom nu at the
                          corner lambda (Sec. 2.5); NaN for a member without a solve */
} sl_result;

/*
 * Workspace bytes for sl_solve_semilinear with these sizes.  max_ns bounds
 * every member's ns.  Returns 0 for invalid sizes (see sl_last_error()).
 */
size_t sl_solve_workspace_size(const sl_problem* pb, int max_ns, int n_members, int n_lambda);

/*
 * Batched regularised solve and L-curve corner of n_members lens sets
 * against one data image (Sec. 2.1-2.6, Sec. 3: the fitness of the outer
 * optimiser).  Every (member, lambda) pair is one conjugate-gradient solve
 * of Eq. 7 from s = 0, stopped when ||b - A s|| <= tol ||b||; all pairs run
 * in one persistent launch.  With SL_F32 and curvature H, a pair whose
 * lambda >= 0.15 c (and whose n x n grid fits beside the blur frame in LDS)
 * is solved by preconditioned CG with M = c I + lambda H^T H, applied exactly
 * through the orthonormal 2-D sine transform that diagonalises H^T H (H^T H
 * = D^2 (x) I + I (x) D^2 with D the second-difference matrix).  c is a
 * per-member estimate of the data term's scale, sum_i w_i b_i^2 / sum_i b_i^2
 * with w = L^T 1 (the bilinear weight each node receives from the image
 * pixels, L averaging the nsub^2 subpixels of a pixel).  The result is
 * the same Eq. 7 solution to the stopping tolerance; sl_tuning.plain_cg = 1
 * solves every pair with plain CG.
 *   lens:    device double[n_members*7]
 *   ns:      device int32[n_members], each in [2, max_ns]
 *   lambdas: host double[n_lambda], strictly ascending, positive, n_lambda <= SL_MAX_LAMBDA
 *   workspace: device, >= sl_solve_workspace_size(pb, max_ns, n_members, n_lambda) bytes,
 *              256-byte aligned; contents need not be initialised
 * Results go to `out`.  With n_lambda < 4 the corner is index 0
 * (corner_status SL_ST_LCURVE when n_lambda is 2 or 3).
 *
 * Monte Carlo degrees of freedom (Sec. 2.5; opts->mc_noise = bhat): after
 * the corners are known, a second system (A^T A + lambda H^T H) x = A^T bhat
 * (A = B L) is solved at every member's corner lambda, and
 * dof[m] = bhat^T (bhat - A xhat), computed as bhat^T bhat - <A^T bhat, xhat>
 * in FP64.  SL_F64: as the paper does, the corner lambda's data system is
 * solved again by plain CG from s = 0 and the second system is advanced in
 * lockstep with the data system's coefficients alpha_k, beta_k (about two
 * solves per member).  SL_F32: that fixed-coefficient recurrence amplifies
 * FP32 rounding without bound on long solves, so the second system is solved
 * by its own CG to the same relative tolerance (one solve per member); both
 * converge to the same xhat.  The expectation of dof over bhat is J - gamma,
 * gamma the trace of the influence matrix (Eq. 19 for H = I), so
 * chi2[m][k_star] / dof[m] is the reduced chi^2.
 */
int sl_solve_semilinear(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns,
                        int n_members, const double* lambdas, int n_lambda,
                        const sl_solve_opts* opt, void* workspace, size_t workspace_bytes,
                        sl_result* out, void* stream);

/*
 * Implicit regularisation by the iteration count (Sec. 2.4, Sec. 2.6, and
 * the fitness of Sec. 3): no lambda; for every member, n_iter CGLS
 * iterations on min ||A s - d|| (A = B L) from s = 0, each applying A once
 * and A^T once, and after iteration k (k = 1..n_iter)
 * chi^2 = ||d - A s_k||^2 / sigma^2 (from the image residual, carried as a
 * vector) and the zeroth-order measure sum_i s_k,i^2 (whatever pb->reg
 * says).  The L-curve over the iterates gives k_star (index k - 1 of the
 * corner iterate) and the member's fitness chi2[m][k_star]; s_corner holds
 * that iterate.  Arguments and outputs as sl_solve_semilinear with
 * n_lambda = n_iter: chi2, reg, iters (= k), status are [n_members][n_iter];
 * workspace from sl_solve_workspace_size(pb, max_ns, n_members, n_iter).
 * n_iter in [4, SL_MAX_LAMBDA]; opts->tol is not used (the count stops the
 * iteration).  After a breakdown (A p = 0) the remaining iterates repeat
 * the last one with status SL_ST_BREAKDOWN.
 *
 * Monte Carlo degrees of freedom (Sec. 2.5, as the paper runs it inside
 * CGLS; opts->mc_noise = bhat, SL_F64 only, else SL_EINVAL): a second system
 * with data bhat is advanced with the data system's step lengths alpha_k,
 * beta_k, and dof[m] = bhat^T (bhat - A xhat_k*) at the corner iterate
 * (computed as bhat^T bhat - <A^T bhat, xhat> in FP64).  Its expectation over
 * bhat is J minus the sum of the CGLS filter factors after k* iterations.
 * The fixed-coefficient recurrence amplifies rounding of the step lengths
 * geometrically with k; FP32 rounding already spoils it within a few
 * iterations, hence FP64 only.  About twice the work of the solve alone.
 */
int sl_solve_implicit(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns,
                      int n_members, int n_iter, const sl_solve_opts* opt, void* workspace,
                      size_t workspace_bytes, sl_result* out, void* stream);

/*
 * Image chi^2 of candidate sources for one lens: the fitness of the final
 * source-refinement search (Sec. 3.2), which holds the best lens fixed and
 * treats every source node as a free, bounded parameter.  For each source
 * s_p (p < n_sources), chi2[p] = ||B L s_p - d||^2 / sigma^2 over all J
 * pixels (Eq. 4), with L and B as in the solve (pixels that do not map keep
 * their data).  One lens, one grid: the solve's trace and tables are built
 * once per call, then the candidates run in one persistent launch.  FP32
 * bulk with an FP64 residual sum (SL_F32) or FP64 throughout (SL_F64).
 *   lens:    device double[7], the lens parameters
 *   ns:      source grid side, in [2, 128]
 *   sources: device double[n_sources][ns*ns], row-major nodes as in s_corner
 *   chi2:    device double[n_sources]; NaN for an invalid lens, sum d^2 /
 *            sigma^2 when no pixel maps
 *   workspace: device, >= sl_chi2_sources_workspace_size(pb, ns) bytes,
 *            256-byte aligned
 * Asynchronous on `stream`; SL_EINVAL for bad host-side arguments.
 */
size_t sl_chi2_sources_workspace_size(const sl_problem* pb, int ns);
int sl_chi2_sources(const sl_problem* pb, const double* lens, int ns, const double* sources,
                    int n_sources, void* workspace, size_t workspace_bytes, double* chi2,
                    void* stream);

/*
 * Blur in Fourier space (Sec. 2.2: the paper convolves with the PSF there),
 * for wide PSFs: the operator of sl_apply_B (transpose = 0) or sl_apply_BT
 * (transpose = 1) on one ny x nx image, computed with 2-D FFTs on an
 * Ny x Nx frame of powers of two with Ny >= ny + (k-1)/2 and
 * Nx >= nx + (k-1)/2, on which the circular convolution equals the
 * zero-padded one.  dtype SL_F32 (in/out float, FP32 transforms) or SL_F64.
 * psf: device double[k*k], k odd <= 129; nx, ny <= 2048 and Nx, Ny <= 4096.
 * in/out: device, distinct.  workspace: device, 256-byte aligned, at least
 * sl_fft_blur_workspace_size(dtype, nx, ny, k) bytes, contents need not be
 * initialised (the query returns 0 for invalid arguments).
 */
size_t sl_fft_blur_workspace_size(int dtype, int nx, int ny, int k);
int sl_fft_blur(int dtype, int transpose, int nx, int ny, const double* psf, int k, const void* in,
                void* out, void* workspace, size_t workspace_bytes, void* stream);

/*
 * One large problem with implicit regularisation, the paper's large-scale
 * test (Sec. 4: a 640 x 640 image, a 512 x 512 source grid, a 65 x 65 PSF,
 * 40 CGLS iterations): one lens (device double[7]), images up to
 * 2048 x 2048, ns up to 1024, PSF side k odd up to 129 (pb->k may exceed
 * SL_MAX_PSF here), B and B^T applied in Fourier space: with pb->dtype
 * SL_F32 and k <= 65 by overlap-save on 96 x 128 tiles (32 x 64 owned
 * pixels each, a 32-pixel halo), otherwise on the padded frame of
 * sl_fft_blur; both the linear convolution of Eq. 4 up to rounding.  L^T is
 * a gather over a node-major table built and sorted on the device (each
 * node's terms summed in ascending pixel order: bitwise reproducible).  The
 * iteration, its outputs and statuses are those of sl_solve_implicit for
 * one member: n_iter CGLS iterations (1..SL_MAX_LAMBDA) from s = 0, after
 * iteration k chi2[k] = ||d - A s_k||^2 / sigma^2 from the carried residual
 * and reg[k] = sum_i s_k,i^2, k_star the L-curve corner over the iterates,
 * s_corner (double[ns*ns]) that iterate, s_off = {0, ns*ns}; chi2, reg,
 * iters, status hold n_iter entries.  pb->reg and pb->psf_general are not
 * used; pb->interp selects L as in the batched solve.  No Monte Carlo
 * degrees of freedom (out->dof is not written).  workspace: device,
 * 256-byte aligned, at least sl_solve_large_workspace_size(pb, ns, n_iter)
 * bytes (0 for invalid arguments); calls sharing it must not overlap.
 */
size_t sl_solve_large_workspace_size(const sl_problem* pb, int ns, int n_iter);
int sl_solve_large(const sl_problem* pb, const double* lens, int ns, int n_iter, void* workspace,
                   size_t workspace_bytes, sl_result* out, void* stream);
/*
 * Autotuner: a staged search over the solve's settings.  Variants 0..7 are
 * the structural switches (wide_window, lt_csr, blur_direct as the bits of
 * the index) at the default threshold and queue order; variants 8..11 set
 * pc_theta_pct to 5, 10, 25, 40 on the best of 0..7 (FP32 with curvature H
 * only: elsewhere the preconditioner never runs); variants 12..15 set heavy
 * to 2, 3, 6, 8 on the best of 0..11.  Each variant runs once untimed and
 * twice timed with HIP events on `stream` (the faster counts).  The fastest
 * is recorded for this problem signature (dtype, image size, subpixels, PSF
 * size, regulariser, max_ns, n_members, n_lambda) in a process-wide table
 * that later calls with opt->tuning == NULL consult.  Synchronous.  With the
 * environment variable SL_AUTOTUNE_VERBOSE=1 it prints one line per variant
 * to stderr as that variant is timed.
 * Arguments are those of sl_solve_semilinear; on return `out` holds the best
 * variant's results, *best (nullable) its settings and ms (nullable, host
 * double[SL_N_VARIANTS]) each variant's time, or -1 for a variant that does
 * not exist for this PSF size and dtype or was skipped.
 */
#define SL_N_VARIANTS 16
int sl_solve_autotune(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns,
                      int n_members, const double* lambdas, int n_lambda,
                      const sl_solve_opts* opt, void* workspace, size_t workspace_bytes,
                      sl_result* out, void* stream, sl_tuning* best, double* ms);

/*
 * Graph plan: the launches of one sl_solve_semilinear call (same
 * arguments; the variant is resolved at creation) captured once into a HIP
 * graph on a private stream.  sl_plan_launch replays it on `stream`; each
 * replay re-reads the device inputs (lens, ns, data, PSF) that the pointers
 * given at creation hold at that time, so a caller updates the lens buffer in
 * place between replays.  The pointers, sizes and lambdas are fixed for the
 * plan's lifetime; the workspace and result buffers must outlive it and
 * replays that share them must not overlap.  No replay allocates.
 */
typedef struct sl_plan sl_plan;
int sl_plan_create(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns,
                   int n_members, const double* lambdas, int n_lambda,
                   const sl_solve_opts* opt, void* workspace, size_t workspace_bytes,
                   const sl_result* out, sl_plan** plan);
int sl_plan_launch(sl_plan* plan, void* stream);
int sl_plan_destroy(sl_plan* plan);

/*
 * Per-member table of the last sl_solve_semilinear that used `workspace`
 * (synchronous: waits for the device).  info_host: host int32[n_members][10]
 * = {ns, I, M (pixels that map onto the grid), r0, r1, c0, c1 (their
 * bounding box), status, Lt (layout of the transposed operator: 0 CSR rows,
 * 1 sliced ELL, 2 sliced ELL with paired 16-bit offsets), frame (1: the
 * member's image frame lives in LDS, 0: in global memory)}; the last two
 * are -1 for a member whose status is not SL_ST_OK.  Sizes must match that
 * call.
 */
int sl_solve_member_info(const sl_problem* pb, int max_ns, int n_members, int n_lambda,
                         const void* workspace, int32_t* info_host);

/*
 * Kernel timing for measurement: while enabled, every sl_solve_semilinear
 * records HIP events around its CG phase (k_split and the persistent CG
 * kernels, preconditioned and plain) on the call's stream.
 * sl_profile_enable(1) clears the record; sl_profile_solve_ms() waits for the
 * recorded events and returns the summed milliseconds and launch count.
 */
int sl_profile_enable(int on);
int sl_profile_solve_ms(double* ms_total, int32_t* launches);

/*
 * L-curve corner (Sec. 2.6, Eq. 20) on the host, synchronous: points
 * (log10 reg_k, log10 chi2_k) are parameterised by chord length, points whose
 * step is <= 1e-12 of the total are dropped, not-a-knot cubic splines are
 * fitted to both coordinates and the curvature
 * |x'y'' - y'x''| / (x'^2 + y'^2)^(3/2) is evaluated at the knots;
 * *k_star = argmax (ties within 1e-12 relative go to the smaller index).
 * kappa (nullable) receives n curvatures, NaN at dropped points.
 * Returns SL_EINVAL when n < 4, a value is not positive and finite, or fewer
 * than 4 distinct points remain.
 */
int sl_lcurve_corner(const double* reg, const double* chi2, int n, int32_t* k_star, double* kappa);

/* ---------------------------------------------------------------------------
 * Surrogate MLP 7 -> 256 -> 256 -> 1 with GELU in its erf form,
 * gelu(z) = z Phi(z).  It is not part of the paper's method: a learned
 * pre-screen that predicts ln chi^2 at the L-curve corner from the seven lens
 * parameters, so that a genetic search (Appendix A.1) can send only its most
 * promising offspring to the full solve.
 *
 * Parameters live in one device float buffer of SL_MLP_NPARAM floats in the
 * order W0[7][256], b0[256], W1[256][256], b1[256], W2[256][1], b2[1]
 * (W[in][out], row-major).  Adam moments m, v use the same layout.
 * Numerics: FP32 master weights.  Products take BF16 copies (round to nearest
 * even) of the weights W0, W1, W2 and of every layer input (x, h1, h2) and
 * accumulate in FP32; biases stay FP32.  The forward 256 x 256 product uses
 * the BF16 matrix cores; the backward products keep the gradient signals in
 * FP32 and treat the BF16 rounding of an activation as the identity.
 * Every sum has a fixed order: results are bitwise reproducible.
 * All calls are asynchronous on `stream`; argument errors return SL_EINVAL
 * before any launch.
 * ------------------------------------------------------------------------- */
#define SL_MLP_IN 7
#define SL_MLP_HID 256
#define SL_MLP_NPARAM (7 * 256 + 256 + 256 * 256 + 256 + 256 + 1)
#define SL_MLP_MAX_BATCH (1 << 20)

/*
 * Bytes of device workspace that a call with this batch size needs (BF16
 * and FP32 transposed copies of W1, activations, GELU derivatives and partial
 * sums of the training step).  Returns 0, with sl_last_error set, for a
 * batch outside [0, SL_MLP_MAX_BATCH].  The caller allocates it; calls that
 * share a workspace must not overlap in time.
 */
size_t sl_mlp_workspace_size(int batch);

/*
 * Forward pass: y[b] = MLP(x[b]) for 0 <= b < batch (1 <= batch <=
 * SL_MLP_MAX_BATCH).  params: device float[SL_MLP_NPARAM]; x: device
 * float[batch][7]; y: device float[batch]; workspace: device buffer of at
 * least sl_mlp_workspace_size(batch) bytes (256-byte aligned).
 */
int sl_mlp_forward(const float* params, const float* x, int batch, float* y, void* workspace,
                   void* stream);

/*
 * sl_mlp_forward without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same results as sl_mlp_forward, bit
 * for bit.  Its scratch (the BF16 and FP32 transposed copies of W1,
 * 384 KiB, whatever the batch) is a static device array of the library,
 * one per GPU, held until the process ends; the call allocates nothing.
 * Every call on a GPU shares that GPU's array, so calls that overlap in
 * time on one GPU (two streams, two threads) race and must be serialised by
 * the caller.  batch in [1, SL_MLP_MAX_BATCH], else SL_EINVAL.
 */
int sl_mlp_forward_noalloc(const float* params, const float* x, int batch, float* y, void* stream);

/*
 * One Adam step on the mean squared error L = (1/B) sum_b (y_hat_b - y_b)^2:
 * forward, backward (same BF16 roundings), then with g = dL/dparams
 *   m = 0.9 m + 0.1 g;  v = 0.999 v + 0.001 g^2;
 *   p -= lr (m / (1 - 0.9^t)) / (sqrt(v / (1 - 0.999^t)) + 1e-8)
 * for step number t >= 1 and lr > 0.  params, adam_m, adam_v: device
 * float[SL_MLP_NPARAM], updated in place; x: device float[batch][7]; y:
 * device float[batch] targets.  grads_out (nullable): device
 * float[SL_MLP_NPARAM] receives g; loss_out (nullable): device float[1]
 * receives L of the batch before the update.  workspace as for
 * sl_mlp_forward.
 */
int sl_mlp_train_step(float* params, float* adam_m, float* adam_v, const float* x, const float* y,
                      int batch, float lr, int t, float* grads_out, float* loss_out,
                      void* workspace, void* stream);

/* Thread-local message describing the last non-zero return. */
const char* sl_last_error(void);

/* Library version string. */
const char* sl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SEMILIN_H */
