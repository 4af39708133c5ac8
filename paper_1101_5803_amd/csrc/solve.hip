// Batched matrix-free regularised source solve (Rogers & Fiege 2011, Sec. 2.1-2.6).
//
// One call scores n_members lens parameter sets against one data image:
//   k_setup   (1 block)          member offsets, XCD-sorted work queues, PSF
//                                factorisation (rank-1 test, 1-D taps, the
//                                banded B^T B coefficients and their image-edge
//                                corrections), sum of d^2
//   k_prep    (1 block/member)   FP64 subpixel trace (Eq. 1, Eqs. 10-11) of
//                                every pixel, compaction of the pixels that map
//                                onto the grid (Sec. 2.2: the others get no
//                                intensity), their bounding box, and the
//                                right-hand side b = L^T B^T d in FP64
//   k_solve   (persistent, 1 block/CU)  each block pulls (member, lambda) items
//                                and runs CG on (L^T B^T B L + lambda H^T H) s = b
//                                from s = 0 (Eq. 7, Eq. 13-14, Sec. 2.2); the
//                                iterate s and residual r in global memory (each
//                                element touched only by its owner thread), p
//                                and q = A p in LDS, the image-space intermediate
//                                in an LDS frame over the mapped bounding box;
//                                ends with chi^2 (Eq. 4) and ||H s||^2 in FP64
//   k_split   (1 block)          moves the items that take the spectral
//                                preconditioner to their own queues (FP32,
//                                curvature H); k_solve<.., true> runs them as
//                                preconditioned CG on a side stream, beside
//                                the plain k_solve
//   k_corner  (1 block/member)   L-curve corner (Sec. 2.6, Eq. 20) in FP64 and
//                                the corner solution copy
//
// B^T B for a rank-1 PSF P = g_y g_x^T factorises as (C_y^T C_y) (x) (C_x^T C_x)
// with C the truncated 1-D "same" convolutions; each factor is a symmetric
// banded matrix equal to the autocorrelation of the 1-D taps except in the
// ck x ck corners next to the image edges, so B^T B y is two in-place banded
// passes over the frame (rows, then columns) with (4ck+1) taps plus a small
// correction for outputs within ck of the image edge.  A PSF that is not
// rank-1 takes the direct K x K path with an image-space buffer in global memory.
#include <algorithm>
#include <array>
#include <map>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "common.h"

namespace sl {

constexpr int kNT = 1024;     // threads per FP32 solve block (kNTof below)
constexpr int kWaves = kNT / kWave;
// Threads per solve block by bulk type: FP64 blocks run 512 threads, which
// leaves 256 VGPRs per lane and no spills; FP32 keeps 1024, whose extra waves
// hide the gathers' latency better than an unspilled 512-thread block does.
template <typename T>
constexpr int kNTof = sizeof(T) == 8 ? 512 : kNT;
constexpr int kSegR = 4;       // outputs per lane in a banded pass
constexpr int kUpd = 4;        // CG vector-update chunk (nodes per thread)
// The spectral preconditioner pays for its four n x n transforms only where
// lambda H^T H dominates the spectrum: it is used when lambda >= kPcTheta c.
constexpr int kPcThetaPct = 15;   // default theta = 0.15 (sl_tuning.pc_theta_pct = 0)
constexpr int kFillW = 16;     // waves that fill the transposed operator in parallel (k_prep's 1024 threads)
constexpr int kHeavy = 4;      // default count of smallest lambdas of each member queued ahead of the rest
constexpr int kMaxCK = 31;

struct alignas(16) MemberInfo {
  int ns, I, M, r0, r1, c0, c1, status;   // M: interleaved table slots (>= mapped pixels)
  long long off;   // start in packed vectors
  int Mtrue;       // pixels with at least one subpixel on the grid
  int sell;        // transposed operator: CSR (0), sliced-ELL (1), sliced-ELL with paired 16-bit offsets (2)
  float pc_c;      // scale c of the spectral preconditioner (see k_prep)
  int lds_frame;   // 1: the member's image frame fits in LDS beside p and q; 0: global frame
  int pad_[2];
};

// Device constants written by k_setup (one copy per workspace).
struct alignas(16) Consts {
  int qhead[8];
  int qcount[8];
  int pqhead[8];    // queues of the preconditioned items (filled by k_split)
  int pqcount[8];
  int sep;          // PSF is rank-1
  int mchead;       // next member of the Monte Carlo degrees-of-freedom pass
  int imhead;       // next member of the implicit-regularisation solve
  int pad0;
  double sum_d2;
  double sum_n2;    // sum of the squared Monte Carlo draws
};

struct Layout {
  size_t consts, lam, taps_d, taps_f, minfo, queues, pqueues, pix, cell, fx, fy, b, bh, dofk, ltc, s_all, gframe, gz, rbuf, mcbuf, ibuf,
      lt_ptr, lt_perm,
      lt_ent,
      total;
  long long lt_cap;
  int qcap, n_wg, I_max, J, n2, gframe_elems, slot_cap;
};

// Offsets (elements) inside the taps arrays, for a PSF of side K (ck = (K-1)/2).
struct TapIdx {
  int gx, gy, ax, ay, elx, erx, ely, ery, psf, total;
  __host__ __device__ TapIdx(int K) {
    const int ck = (K - 1) / 2;
    const int na = 4 * kMaxCK + 1;     // autocorrelation padded to the largest window
    gx = 0;
    gy = gx + K;
    ax = gy + K;
    ay = ax + na;
    elx = ay + na;
    erx = elx + ck * ck;
    ely = erx + ck * ck;
    ery = ely + ck * ck;
    psf = ery + ck * ck;
    total = psf + K * K;
  }
};

// One entry of the transposed lens operator: L^T w at a node is the sum of
// w[off] * weight over the node's entries (off = frame offset of the pixel).
template <typename T>
struct alignas(2 * sizeof(T) > 8 ? 16 : 8) LtEntry {
  int off;
  T w;
};

// ------------------------------------------------------------------ parameters
struct SolveArgs {
  int nx, ny, nsub, n2, K, ck, ckt, reg, n_members, n_lambda, max_ns, maxit, lds_frame_cap;
  int q_off, red_off, pc_off, frame_off;   // byte offsets in dynamic LDS
  int gframe_elems;                // per-block global frame size (elements)
  int slot_cap;                    // trace-table slots per member (J + 64)
  double pix, R, sigma, tol;
  double* lamv;                    // workspace copy of the lambda grid
  const double* lens;
  const int32_t* ns;
  const double* d;
  const double* psf;
  // results
  double* s_corner;
  int64_t* s_off;
  double* chi2;
  double* regv;
  int32_t* iters;
  int32_t* status;
  int32_t* k_star;
  int32_t* corner_status;
  // workspace
  Consts* consts;
  double* taps_d;
  void* taps_t;   // taps in the bulk type
  MemberInfo* minfo;
  int* queues;
  int* pqueues;     // [8][qcap] items of the preconditioned solve
  int qcap;
  int32_t* pix_list;
  int32_t* cell;
  void* fx;
  void* fy;
  double* b;
  void* s_all;
  void* gframe;
  void* gz;
  void* rbuf;       // per-block CG residual
  int32_t* lt_ptr;  // [member][I_max + 65] slice (or row) starts of the transposed operator
  int32_t* lt_perm; // [member][I_max] nodes in slice order, packed (row << 16 | col)
  void* lt_ent;     // [member][lt_cap] LtEntry<T>
  long long lt_cap; // entries per member
  int I_max;
  int force_csr;    // variant: transposed operator as CSR rows
  int force_direct; // direct K x K blur only (variant, the hint that the PSF is not rank 1, or bicubic L)
  int psf_general;  // the caller's hint: the PSF is not rank 1
  int interp;       // SL_INTERP_BILINEAR | NEAREST (the fractions k_prep stores) | BICUBIC
  int prep_tags;    // k_prep has one LDS int per node after its 8 I_max + 768 bytes (conflict tags)
  int implicit;     // implicit regularisation: n_lambda unregularised CG iterations (k_implicit)
  int heavy;        // smallest lambdas of each member queued ahead of the rest
  float pc_theta;   // items with lambda >= pc_theta c take the spectral preconditioner
  int plain_cg;     // variant: no spectral preconditioner
  // Monte Carlo degrees of freedom (Sec. 2.5), when mcn is not NULL
  const double* mcn; // [ny*nx] Gaussian draws bhat
  double* dofv;      // [n_members] result: bhat^T (bhat - A xhat) at the corner
  double* bh;        // [member][I_max] A^T bhat (FP64)
  double* dofk;      // [member][n_lambda] implicit solve: the estimate after each iterate
  int* ltc;          // [member][I_max][kFillW] per-wave fill cursors of the transposed operator
  void* mcbuf;       // [n_wg][5][I_max] r, xhat, rhat, phat, saved p of the pass
  void* ibuf;        // [n_wg][J] image residual e = d - A s of the implicit-regularisation solve
};

// ------------------------------------------------------------------ block scan
// Exclusive prefix count of `flag` over the block; returns this thread's
// offset and writes the block total to *total.  `scratch` >= 16 ints.
__device__ __forceinline__ int block_excl_count(bool flag, int* scratch, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long bal = __ballot(flag);
  const int in_wave = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  if (lane == 0) scratch[wid] = __popcll(bal);
  __syncthreads();
  int before = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const int c = scratch[i];
    if (i < wid) before += c;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return before + in_wave;
}

// ------------------------------------------------------------------ k_setup
struct LamList {
  double v[SL_MAX_LAMBDA];
};

template <typename T>
__global__ void __launch_bounds__(1024) k_setup(SolveArgs a, LamList lams) {
  // the tap table is built by thread 0 in LDS from the PSF staged there (in
  // global memory every read of its loops waited on the stores before it) and
  // copied out by all threads
  extern __shared__ __align__(16) unsigned char smem_setup[];
  double* tsh = reinterpret_cast<double*>(smem_setup);
  __shared__ double red[32];
  if (threadIdx.x < a.n_lambda) a.lamv[threadIdx.x] = lams.v[threadIdx.x];
  __shared__ int counts[4097];
  const int tid = threadIdx.x;
  const int M = a.n_members, K = a.K, ck = a.ck;
  // the PSF staged in LDS beside the tap table, by all threads
  double* psh = tsh + TapIdx(SL_MAX_PSF).total;
  for (int i = tid; i < K * K; i += blockDim.x) psh[i] = a.psf[i];
  __syncthreads();
  // offsets of packed solutions; invalid ns contribute nothing
  if (tid == 0) {
    long long off = 0;
    for (int m = 0; m < M; ++m) {
      const int ns = a.ns[m];
      const bool ok = ns >= 2 && ns <= a.max_ns;
      a.s_off[m] = off;
      a.minfo[m].ns = ok ? ns : 0;
      a.minfo[m].I = ok ? ns * ns : 0;
      a.minfo[m].off = off;
      off += ok ? (long long)ns * ns : 0;
    }
    a.s_off[M] = off;
  }
  // counting sort of members by descending ns -> XCD queues round-robin
  for (int i = tid; i <= 4096; i += blockDim.x) counts[i] = 0;
  __syncthreads();
  if (tid == 0) {
    for (int m = 0; m < M; ++m) {
      const int ns = a.ns[m];
      counts[(ns >= 2 && ns <= a.max_ns) ? ns : 0]++;
    }
    int start = 0;   // exclusive prefix in descending ns order (keys are at most max_ns)
    for (int v = a.max_ns < 4096 ? a.max_ns : 4096; v >= 0; --v) {
      const int c = counts[v];
      counts[v] = start;
      start += c;
    }
    // rank r -> queue r % 8; the sort is stable in member index.  Within a
    // queue the `heavy` smallest lambdas of every member come first (their
    // solves take the most CG iterations, so starting them early shortens
    // the tail of the launch), then the other lambdas; both parts keep the
    // members in order, so the blocks of an XCD share few members at a time
    // and their tables stay in its L2.
    for (int m = 0; m < M; ++m) {
      const int ns = a.ns[m];
      const int key = (ns >= 2 && ns <= a.max_ns) ? ns : 0;
      const int r = counts[key]++;
      const int q = r & 7, t = r >> 3;
      const int nmq = (M - q + 7) / 8;   // members in queue q
      const int H = a.n_lambda < a.heavy ? a.n_lambda : a.heavy;
      for (int k = 0; k < a.n_lambda; ++k)
        a.queues[q * a.qcap + (k < H ? t * H + k : nmq * H + t * (a.n_lambda - H) + (k - H))] = m * a.n_lambda + k;
    }
    for (int q = 0; q < 8; ++q) {
      // members with rank r = q + 8 t fill queue q densely
      const int nm = (M > q) ? (M - q + 7) / 8 : 0;
      a.consts->qcount[q] = nm * a.n_lambda;
      a.consts->qhead[q] = 0;
      a.consts->pqcount[q] = 0;
      a.consts->pqhead[q] = 0;
    }
    // PSF: rank-1 test and factorisation P[a][b] = gy[a] * gx[b]
    const TapIdx ti(K);
    int am = 0, bm = 0;
    double pmax = 0.0;
    for (int i = 0; i < K * K; ++i)
      if (fabs(psh[i]) > pmax) {
        pmax = fabs(psh[i]);
        am = i / K;
        bm = i % K;
      }
    double* tp = tsh;
    for (int i = 0; i < ti.total; ++i) tp[i] = 0.0;
    for (int i = 0; i < K * K; ++i) tp[ti.psf + i] = psh[i];
    int sep = pmax > 0.0;
    if (sep) {
      for (int x = 0; x < K; ++x) {
        tp[ti.gy + x] = psh[x * K + bm];
        tp[ti.gx + x] = psh[am * K + x] / psh[am * K + bm];
      }
      for (int x = 0; x < K && sep; ++x)
        for (int y = 0; y < K; ++y)
          if (fabs(psh[x * K + y] - tp[ti.gy + x] * tp[ti.gx + y]) > 1e-12 * pmax) {
            sep = 0;
            break;
          }
    }
    // the banded path needs the kernel's window to cover +-2ck
    if (ck > a.ckt || a.force_direct) sep = 0;
    a.consts->sep = sep;
    if (sep) {
      // autocorrelations a[d] = sum_i g[i] g[i-d], stored at index d + 2*kMaxCK
      for (int dd = -(K - 1); dd <= K - 1; ++dd) {
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < K; ++i) {
          const int j = i - dd;
          if (j < 0 || j >= K) continue;
          sx += tp[ti.gx + i] * tp[ti.gx + j];
          sy += tp[ti.gy + i] * tp[ti.gy + j];
        }
        tp[ti.ax + dd + 2 * kMaxCK] = sx;
        tp[ti.ay + dd + 2 * kMaxCK] = sy;
      }
      // edge corrections: the truncated 1-D convolution C has (C^T C)[c][c']
      // = a[c'-c] - sum over intermediate indices k outside the image
      for (int p = 0; p < ck; ++p)
        for (int q = 0; q < ck; ++q) {
          double lx = 0.0, ly = 0.0, rx = 0.0, ry = 0.0;
          for (int k = -ck; k < 0; ++k) {
            const int i1 = k - p + ck, i2 = k - q + ck;
            if (i1 >= 0 && i1 < K && i2 >= 0 && i2 < K) {
              lx += tp[ti.gx + i1] * tp[ti.gx + i2];
              ly += tp[ti.gy + i1] * tp[ti.gy + i2];
            }
          }
          // right edge: outputs c = n - ck + p, inputs c' = n - ck + q, k = n + kk
          for (int kk = 0; kk < ck; ++kk) {
            const int i1 = kk + 2 * ck - p, i2 = kk + 2 * ck - q;   // k - c + ck, k - c' + ck
            if (i1 >= 0 && i1 < K && i2 >= 0 && i2 < K) {
              rx += tp[ti.gx + i1] * tp[ti.gx + i2];
              ry += tp[ti.gy + i1] * tp[ti.gy + i2];
            }
          }
          tp[ti.elx + p * ck + q] = lx;
          tp[ti.ely + p * ck + q] = ly;
          tp[ti.erx + p * ck + q] = rx;
          tp[ti.ery + p * ck + q] = ry;
        }
    }
  }
  __syncthreads();
  {
    const TapIdx ti(K);
    T* tt = reinterpret_cast<T*>(a.taps_t);
    for (int i = tid; i < ti.total; i += blockDim.x) {
      a.taps_d[i] = tsh[i];
      tt[i] = (T)tsh[i];
    }
  }
  // sums of d^2 and of the Monte Carlo draws squared, in FP64
  double acc = 0.0, accn = 0.0;
  const int J = a.nx * a.ny;
  for (int j = tid; j < J; j += blockDim.x) {
    acc += a.d[j] * a.d[j];
    if (a.mcn) accn += a.mcn[j] * a.mcn[j];
  }
  acc = block_sum(acc, red);
  accn = block_sum(accn, red);
  if (tid == 0) {
    a.consts->sum_d2 = acc;
    a.consts->sum_n2 = accn;
    a.consts->mchead = 0;
    a.consts->imhead = 0;
  }
}

// ------------------------------------------------------------------ k_prep
template <typename T>
__device__ void prep_member(const SolveArgs& a, int m, MemberInfo mi, const double* gl, int* bbox, int* scan,
                            double* bacc);

template <typename T>
__global__ void __launch_bounds__(1024) k_prep(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* bacc = reinterpret_cast<double*>(smem);
  __shared__ int scan[32];
  __shared__ int bbox[4];
  __shared__ double g[7];
  const int m = blockIdx.x, tid = threadIdx.x;
  const int nx = a.nx, ny = a.ny, J = nx * ny, nsub = a.nsub, n2 = a.n2;
  MemberInfo mi = a.minfo[m];
  if (tid < 7) g[tid] = a.lens[7L * m + tid];
  if (tid == 0) {
    bbox[0] = INT_MAX;
    bbox[1] = INT_MIN;
    bbox[2] = INT_MAX;
    bbox[3] = INT_MIN;
  }
  __syncthreads();
  double gl[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) gl[i] = g[i];
  // the same for every thread; readfirstlane makes that visible to the compiler,
  // so the branch around the barriers below is a scalar (block-uniform) branch
  const int valid = __builtin_amdgcn_readfirstlane((int)(mi.ns >= 2 && lens_valid(gl)));
  if (!valid) {
    if (tid == 0) {
      mi.M = 0;
      mi.Mtrue = 0;
      mi.status = SL_ST_INVALID;
      mi.r0 = mi.c0 = 0;
      mi.r1 = mi.c1 = -1;
      a.minfo[m] = mi;
    }
  } else {
    prep_member<T>(a, m, mi, gl, bbox, scan, bacc);
  }
}

// Cubic convolution kernel (Keys 1981, a = -1/2) at distance d >= 0 from a
// node; the tap at offset o (-1..2) from a cell's first node lies at
// distance |f - o| for the fraction f in [0, 1].
template <typename F>
__device__ __forceinline__ F keys_w(F d) {
  return d <= F(1) ? (F(1.5) * d - F(2.5)) * d * d + F(1)
                   : (d < F(2) ? ((F(-0.5) * d + F(2.5)) * d - F(4)) * d + F(2) : F(0));
}

// Pair q (q < 16 n^2) of mapped slot t under bicubic interpolation: subpixel
// q / 16, tap q % 16 = 4 (j + 1) + (i + 1) at row offset j and column offset
// i from the cell's first node; node -1 for an off-grid subpixel or a tap
// outside the grid (the source is zero there).  The weight includes the
// 1/n^2 subpixel average.  Pairs are not merged: a node can occur at several
// q of one pixel, each q adding its own entry.
template <typename T>
__device__ __forceinline__ void bicubic_pair(int t, int q, int ns, int n2, const int32_t* cellp, const T* fxp,
                                             const T* fyp, int& node, double& w) {
  const int k = q >> 4, j = (q >> 2) & 3, i = q & 3;
  const int c = cellp[(long)t * n2 + k];
  node = -1;
  w = 0.0;
  if (c < 0) return;
  const int r = c / ns + j - 1, col = c % ns + i - 1;
  if (r < 0 || r >= ns || col < 0 || col >= ns) return;
  const double fx = (double)fxp[(long)t * n2 + k], fy = (double)fyp[(long)t * n2 + k];
  node = r * ns + col;
  w = keys_w(fabs(fy - (j - 1))) * keys_w(fabs(fx - (i - 1))) / n2;
}

// Trace, compaction and right-hand side of one valid member (all threads).
// Unique (node, weight) pairs of the subpixels of mapped slot t, weights
// including the 1/n^2 subpixel average; returns the pair count (<= 4 n^2).
template <typename T>
__device__ int pixel_pairs(int t, int ns, int n2, const int32_t* cellp, const T* fxp, const T* fyp, int* node,
                           double* wt) {
  int cnt = 0;
  const double inv = 1.0 / n2;
  for (int k = 0; k < n2; ++k) {
    const int c = cellp[(long)t * n2 + k];
    if (c < 0) continue;
    const double fx = (double)fxp[(long)t * n2 + k], fy = (double)fyp[(long)t * n2 + k];
    const int nd[4] = {c, c + 1, c + ns, c + ns + 1};
    const double ww[4] = {(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy};
    for (int q = 0; q < 4; ++q) {
      int f = 0;
      while (f < cnt && node[f] != nd[q]) ++f;
      if (f == cnt) {
        node[cnt] = nd[q];
        wt[cnt] = 0.0;
        ++cnt;
      }
      wt[f] += ww[q] * inv;
    }
  }
  return cnt;
}

// pixel_pairs for 2 x 2 subpixels with everything in registers: the 16
// (subpixel, corner) pairs in the same order, a pair whose node already
// occurred folds its weight into the first occurrence (same summation order
// as pixel_pairs); folded pairs get node -1.
template <typename T>
__device__ __forceinline__ void pixel_pairs4(int t, int ns, const int32_t* cellp, const T* fxp, const T* fyp,
                                             int (&node)[16], double (&wt)[16]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = cellp[(long)t * 4 + k];
    const double fx = (double)fxp[(long)t * 4 + k], fy = (double)fyp[(long)t * 4 + k];
    const bool in = c >= 0;
    node[4 * k + 0] = in ? c : -1;
    node[4 * k + 1] = in ? c + 1 : -1;
    node[4 * k + 2] = in ? c + ns : -1;
    node[4 * k + 3] = in ? c + ns + 1 : -1;
    wt[4 * k + 0] = (1 - fx) * (1 - fy) * 0.25;
    wt[4 * k + 1] = fx * (1 - fy) * 0.25;
    wt[4 * k + 2] = (1 - fx) * fy * 0.25;
    wt[4 * k + 3] = fx * fy * 0.25;
  }
#pragma unroll
  for (int i = 1; i < 16; ++i) {
    bool folded = node[i] < 0;
#pragma unroll
    for (int j = 0; j < i; ++j) {
      const bool hit = !folded && node[j] == node[i];
      wt[j] += hit ? wt[i] : 0.0;
      folded = folded || hit;
    }
    if (folded) node[i] = -1;
  }
}

// Rank of this lane among the lanes of its wave that hold the same key
// (key >= 0), and their count.  With an LDS tag array (one int per key), a
// step in which no two lanes share a key is recognised in one store/load
// round trip: every lane writes its lane id at its key and reads it back, and
// a lane that reads another id shares its key.  Whether some lane does is the
// same whichever store won, so the outcome, and every summation order built
// on it, is the same on every run.  Only when keys are shared are the ranks
// counted lane by lane (64 readlane steps).
__device__ __forceinline__ void lane_rank(int key, int* tag, int& rank, int& total) {
  const int lane = threadIdx.x & 63;
  if (tag) {
    if (key >= 0) tag[key] = lane;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int seen = key >= 0 ? reinterpret_cast<volatile int*>(tag)[key] : lane;
    const int clash = __builtin_amdgcn_readfirstlane((int)(__ballot(seen != lane) != 0ull));
    // every lane has read its tag before a later step writes the array again
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (!clash) {
      rank = 0;
      total = 1;
      return;
    }
  }
  rank = 0;
  total = 0;
  for (int l = 0; l < 64; ++l) {   // uniform lane index: v_readlane
    const int kl = __builtin_amdgcn_readlane(key, l);
    if (kl == key) {
      ++total;
      if (l < lane) ++rank;
    }
  }
}

// Quarter-octave bucket of a row length (0 for empty rows): rows in one
// bucket differ by less than 19%.
__device__ __forceinline__ int len_bucket(int c) {
  if (c <= 0) return 0;
  const int msb = 31 - __clz(c);
  const int frac = msb >= 2 ? (c >> (msb - 2)) & 3 : (c << (2 - msb)) & 3;
  return 4 * msb + frac + 1;
}

// Node-major form of L^T for one member, sliced-ELL with rows sorted by length
// (SELL-C-sigma with C = 64, one slice per wave): nodes are ordered by
// descending length bucket (stable in node index) into perm[] = packed
// (row << 16 | col); entry j of the node at position p sits at
// ptr[p/64] + 64 j + p%64, every slice padded to its longest row with
// entries (offset 0, weight 0) -- offset 0 is a frame halo element, always
// zero.  Entries of a node are filled in a fixed order, so the per-node sum
// is the same on every run.  Falls back to plain CSR in node order (ptr = row
// starts) when the padded form exceeds the capacity; returns 1 for
// sliced-ELL, 0 for CSR.  lds: LDS ints (>= 2 I + 64 + 128).
template <typename T>
__device__ int build_transpose(const SolveArgs& a, int m, int ns, int slots, const int* bbox, int* scan, int* lds,
                               const int32_t* pix, const int32_t* cellp, const T* fxp, const T* fyp, int* tag) {
  const int tid = threadIdx.x, n2 = a.n2, I = ns * ns;
  const int halo = 2 * a.ckt;
  const int pitch = (bbox[3] - bbox[2] + 1 + 2 * halo) | 1;
  const int ngroups = (I + 63) / 64;
  int* cnt = lds;                       // [I + 64] row lengths, later fill cursors
  int* ipos = lds + I + 64;             // [I] sorted position of every node
  int* hist = ipos + I;                 // [128] bucket histogram
  int32_t* rp = a.lt_ptr + (long)m * (a.I_max + 65);
  int32_t* perm = a.lt_perm + (long)m * a.I_max;
  LtEntry<T>* ent = reinterpret_cast<LtEntry<T>*>(a.lt_ent) + (long)m * a.lt_cap;
  int node[4 * SL_MAX_NSUB * SL_MAX_NSUB];
  double wt[4 * SL_MAX_NSUB * SL_MAX_NSUB];
  __shared__ int totals[2];
  for (int i = tid; i < I + 64; i += blockDim.x) cnt[i] = 0;
  for (int i = tid; i < 128; i += blockDim.x) hist[i] = 0;
  if (tid == 0) totals[0] = totals[1] = 0;
  __syncthreads();
  const bool cubic = a.interp == SL_INTERP_BICUBIC;
  if (cubic) {
    for (int t = tid; t < slots; t += blockDim.x) {
      if (pix[t] < 0) continue;
      for (int q = 0; q < 16 * n2; ++q) {
        int nd;
        double ww;
        bicubic_pair(t, q, ns, n2, cellp, fxp, fyp, nd, ww);
        if (nd >= 0) atomicAdd(&cnt[nd], 1);
      }
    }
  } else if (n2 == 4) {
    for (int t = tid; t < slots; t += blockDim.x) {
      if (pix[t] < 0) continue;
      int nd[16];
      double ww[16];
      pixel_pairs4(t, ns, cellp, fxp, fyp, nd, ww);
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (nd[q] >= 0) atomicAdd(&cnt[nd[q]], 1);
    }
  } else {
    for (int t = tid; t < slots; t += blockDim.x) {
      if (pix[t] < 0) continue;
      const int np = pixel_pairs(t, ns, n2, cellp, fxp, fyp, node, wt);
      for (int q = 0; q < np; ++q) atomicAdd(&cnt[node[q]], 1);
    }
  }
  __syncthreads();
  for (int i = tid; i < I; i += blockDim.x) atomicAdd(&hist[len_bucket(cnt[i])], 1);
  __syncthreads();
  if (tid == 0) {   // descending buckets -> start positions
    int run = 0;
    for (int b = 127; b >= 0; --b) {
      const int c = hist[b];
      hist[b] = run;
      run += c;
    }
  }
  __syncthreads();
  // stable placement in node order: one wave per bucket pass keeps it deterministic.
  // Only this wave touches hist[] here, and one wave's LDS accesses complete in
  // order, so wavefront-scope fences (compiler ordering, no wait on the global
  // stores) around the wave barrier order its LDS read-modify-writes.
  if (tid < 64) {
    for (int i0 = 0; i0 < I; i0 += 64) {
      const int i = i0 + tid;
      const int b = i < I ? len_bucket(cnt[i]) : -1;
      // rank of the lane among lower lanes with the same bucket, and the bucket's count
      int before = 0, total = 0;
      for (int l = 0; l < 64; ++l) {   // uniform lane index: v_readlane, no LDS round trip
        const int bl = __builtin_amdgcn_readlane(b, l);
        if (bl == b) {
          ++total;
          if (l < tid) ++before;
        }
      }
      const int p = i < I ? hist[b] + before : 0;
      if (i < I) {
        ipos[i] = p;
        perm[p] = ((i / ns) << 16) | (i % ns);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // the bucket's last lane advances it past this group's nodes
      if (i < I && before == total - 1) hist[b] = p + 1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  // FP32 members whose frame fits in LDS (frame offsets below 2^16) store the
  // sliced-ELL entries in pairs: slices of even length, one dword holding the
  // 16-bit offsets of entries 2k and 2k + 1 of a lane and one float2 their
  // weights (6 bytes per entry instead of 8)
  const int fh = bbox[1] - bbox[0] + 1, fw = bbox[3] - bbox[2] + 1;
  const int pair_ok = __builtin_amdgcn_readfirstlane(
      (int)(sizeof(T) == 4 && (long)(fh + 4 * a.ckt + kSegR) * ((fw + 4 * a.ckt) | 1) <= a.lds_frame_cap &&
            a.lds_frame_cap <= 65536));
  // slice lengths (rows sorted by length: little padding) and the plain total
  for (int g = tid; g < ngroups; g += blockDim.x) {
    int mx = 0;
    for (int l = 0; l < 64 && 64 * g + l < I; ++l) {
      const int i = (perm[64 * g + l] >> 16) * ns + (perm[64 * g + l] & 0xFFFF);
      mx = max(mx, cnt[i]);
    }
    if (pair_ok) mx = (mx + 1) & ~1;
    atomicAdd(&totals[0], 64 * mx);
  }
  __syncthreads();
  const int sell = __builtin_amdgcn_readfirstlane((int)(!a.force_csr && (long long)totals[0] <= a.lt_cap));
  const int paired = sell && pair_ok;
  // exclusive scan over units: slices (padded sizes) for sliced-ELL, rows for CSR
  const int nunits = sell ? ngroups : I;
  const int chunk = (nunits + blockDim.x - 1) / blockDim.x;
  const int u0 = min(nunits, tid * chunk), u1 = min(nunits, u0 + chunk);
  auto unit_size = [&](int u) {
    if (!sell) return cnt[u];
    int mx = 0;
    for (int l = 0; l < 64 && 64 * u + l < I; ++l) {
      const int i = (perm[64 * u + l] >> 16) * ns + (perm[64 * u + l] & 0xFFFF);
      mx = max(mx, cnt[i]);
    }
    if (paired) mx = (mx + 1) & ~1;
    return 64 * mx;
  };
  int local = 0;
  for (int u = u0; u < u1; ++u) local += unit_size(u);
  const int lane = tid & 63, wid = tid >> 6;
  int incl = local;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) scan[wid] = incl;
  __syncthreads();
  int before = 0;
  for (int i = 0; i < wid; ++i) before += scan[i];
  int run = before + incl - local;
  for (int u = u0; u < u1; ++u) {
    rp[u] = run;
    run += unit_size(u);
  }
  if (tid == blockDim.x - 1) rp[nunits] = run;
  __syncthreads();
  // padding entries: offset 0 (a halo corner of the frame, always zero), weight 0
  const int E = rp[ngroups];   // sliced-ELL entries (a multiple of 128 when paired)
  unsigned short* off16 = reinterpret_cast<unsigned short*>(ent);
  float* w32 = reinterpret_cast<float*>(off16 + E);
  if (paired)
    for (int e = tid; e < 3 * (E >> 1); e += blockDim.x) reinterpret_cast<unsigned*>(ent)[e] = 0u;
  else if (sell)
    for (int e = tid; e < E; e += blockDim.x) {
      ent[e].off = 0;
      ent[e].w = (T)0;
    }
  // entry base of every node: ipos[] becomes the index of its first entry
  for (int i = tid; i < I; i += blockDim.x) {
    const int p = ipos[i];
    ipos[i] = sell ? rp[p >> 6] + (p & 63) : rp[i];
    cnt[i] = 0;   // fill cursors
  }
  __syncthreads();
  const int estep = sell ? 64 : 1;
  // Fill in a fixed order without sorting.  The entries of a node are
  // ordered by (slot group of 64, pair q, lane): lanes holding the same node
  // take consecutive positions in lane order (a pixel's pairs have distinct
  // nodes), the same on every run.
  //
  // 2 x 2 subpixels: the kFillW waves fill in parallel, wave w taking the
  // contiguous range of slot groups [w G / kFillW, (w + 1) G / kFillW).  A
  // first pass counts each node's entries per wave (global atomics into the
  // member's cursor table), an exclusive scan over the waves gives wave w the
  // position after the entries of the groups before its range, and then each
  // wave walks its groups as one wave would.  So the order, and every sum
  // built on it, is the order of a single wave walking all groups.  The
  // waves share the LDS conflict tags: a clash seen through another wave's
  // tag only sends a step down the exact counting path.
  if (n2 == 4 && !cubic) {
    const int G = (slots + 63) / 64;
    const int w = tid >> 6, lane = tid & 63;
    const int g0 = (w * G) / kFillW, g1 = ((w + 1) * G) / kFillW;
    int* cw = a.ltc + (long)m * a.I_max * kFillW;   // [node][wave]
    for (int e = tid; e < I * kFillW; e += blockDim.x) cw[e] = 0;
    __syncthreads();
    for (int g = g0; g < g1; ++g) {   // counts per (node, wave)
      const int t = g * 64 + lane;
      if (t < slots && pix[t] >= 0) {
        int nd[16];
        double ww[16];
        pixel_pairs4(t, ns, cellp, fxp, fyp, nd, ww);
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (nd[q] >= 0) atomicAdd(&cw[nd[q] * kFillW + w], 1);
      }
    }
    __syncthreads();
    for (int i = tid; i < I; i += blockDim.x) {   // exclusive scan over the waves; cnt[i] keeps the total
      int run = 0;
      for (int v = 0; v < kFillW; ++v) {
        const int c = __hip_atomic_load(&cw[i * kFillW + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&cw[i * kFillW + v], run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        run += c;
      }
      cnt[i] = run;
    }
    __syncthreads();
    for (int g = g0; g < g1; ++g) {   // uniform per wave
      const int t = g * 64 + lane;
      int nd[16];
      double ww[16];
      int off = 0;
      const int rc = t < slots ? pix[t] : -1;
      if (rc >= 0) {
        off = ((rc >> 16) - bbox[0] + halo) * pitch + ((rc & 0xFFFF) - bbox[2] + halo);
        pixel_pairs4(t, ns, cellp, fxp, fyp, nd, ww);
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) nd[q] = -1;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int key = nd[q];
        if (!__builtin_amdgcn_readfirstlane((int)(__ballot(key >= 0) != 0ull))) continue;   // uniform
        int rank, total;
        lane_rank(key, tag, rank, total);
        int* cur = key >= 0 ? &cw[key * kFillW + w] : nullptr;
        const int j = key >= 0 ? __hip_atomic_load(cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + rank : 0;
        // every lane has read its cursor before the last lane of a node advances it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (key >= 0 && rank == total - 1)
          __hip_atomic_store(cur, j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the advance is complete before this wave's next step reads the cursors
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (key >= 0 && j < cnt[key]) {   // j < cnt[key] always holds; the test keeps every write in the node's rows
          if (paired) {
            const long ps = ((long)(ipos[key] & ~63) >> 1) + 64L * (j >> 1) + (ipos[key] & 63);
            off16[2 * ps + (j & 1)] = (unsigned short)off;
            w32[2 * ps + (j & 1)] = (float)ww[q];
          } else {
            const long e = (long)ipos[key] + (long)estep * j;
            ent[e].off = off;
            ent[e].w = (T)ww[q];
          }
        }
      }
    }
  } else if (tid < 64) {
    const int lane = tid;
    for (int t0 = 0; t0 < slots; t0 += 64) {
      const int t = t0 + lane;
      int np = 0, off = 0;
      if (t < slots) {
        const int rc = pix[t];
        if (rc >= 0) {
          off = ((rc >> 16) - bbox[0] + halo) * pitch + ((rc & 0xFFFF) - bbox[2] + halo);
          np = cubic ? 16 * n2 : pixel_pairs(t, ns, n2, cellp, fxp, fyp, node, wt);
        }
      }
      int npmax = np;
      for (int o = 32; o > 0; o >>= 1) npmax = max(npmax, __shfl_xor(npmax, o, 64));
      for (int q = 0; q < npmax; ++q) {
        int key = -1;
        double wq = 0.0;
        if (q < np) {
          if (cubic) {
            bicubic_pair(t, q, ns, n2, cellp, fxp, fyp, key, wq);
          } else {
            key = node[q];
            wq = wt[q];
          }
        }
        int rank, total;
        lane_rank(key, tag, rank, total);
        const int j = key >= 0 ? cnt[key] + rank : 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (key >= 0 && rank == total - 1) cnt[key] = j + 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (key >= 0) {
          if (paired) {
            const long ps = ((long)(ipos[key] & ~63) >> 1) + 64L * (j >> 1) + (ipos[key] & 63);
            off16[2 * ps + (j & 1)] = (unsigned short)off;
            w32[2 * ps + (j & 1)] = (float)wq;
          } else {
            const long e = (long)ipos[key] + (long)estep * j;
            ent[e].off = off;
            ent[e].w = (T)wq;
          }
        }
      }
    }
  }
  __syncthreads();
  return paired ? 2 : sell;
}

// bacc[key] += val on the lanes of one wave with key >= 0; lanes that share
// a key add in lane order (they take turns by their rank among the lanes
// with that key), so every node's sum has the same order on every run.
__device__ __forceinline__ void wave_ordered_add(double* bacc, int* tag, int key, double val) {
  if (!__builtin_amdgcn_readfirstlane((int)(__ballot(key >= 0) != 0ull))) return;   // uniform
  int rank, total;
  lane_rank(key, tag, rank, total);
  (void)total;
  for (int r = 0; __ballot(key >= 0 && rank >= r) != 0ull; ++r) {
    if (key >= 0 && rank == r) bacc[key] += val;
    // this round's LDS writes precede the next round's reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// (B^T img)[pixel of slot t] for every slot (0 for empty slots), FP64, by all
// threads of the block, into vbuf[slots] (global memory of this member).
__device__ void correlate_slots(const SolveArgs& a, const double* img, int slots, const int32_t* pix,
                                double* vbuf) {
  const int nx = a.nx, ny = a.ny, K = a.K, ck = a.ck;
  for (int t = threadIdx.x; t < slots; t += blockDim.x) {
    const int rc = pix[t];
    double v = 0.0;
    if (rc >= 0) {
      const int r = rc >> 16, c = rc & 0xFFFF;
      for (int aa = 0; aa < K; ++aa) {
        const int rr = r + aa - ck;
        if (rr < 0 || rr >= ny) continue;
        for (int bb = 0; bb < K; ++bb) {
          const int cc = c + bb - ck;
          if (cc < 0 || cc >= nx) continue;
          v += a.psf[aa * K + bb] * img[rr * nx + cc];
        }
      }
    }
    vbuf[t] = v;
  }
}

// Right-hand side b = L^T B^T img in FP64 (Eq. 7: img = d) into bacc[I] (zeroed), by
// one wave, from v = B^T img at the mapped pixels (vbuf, correlate_slots): it
// walks the slots 64 at a time and spreads each lane's value over its
// pixel's (node, weight) pairs, pair by pair, through wave_ordered_add.  The
// order of every node's terms is therefore (slot group, pair, lane), the
// same on every run.  `slots` is a multiple of 64.
template <typename T>
__device__ void rhs_fixed_order(const SolveArgs& a, const double* vbuf, int ns, int slots, const int32_t* pix,
                                const int32_t* cellp, const T* fxp, const T* fyp, double* bacc, int* tag) {
  const int lane = threadIdx.x & 63;
  const int n2 = a.n2;
  for (int t0 = 0; t0 < slots; t0 += 64) {
    const int t = t0 + lane;
    const int rc = pix[t];
    const double v = vbuf[t];
    if (a.interp == SL_INTERP_BICUBIC) {
      for (int q = 0; q < 16 * n2; ++q) {
        int nd = -1;
        double w = 0.0;
        if (rc >= 0) bicubic_pair(t, q, ns, n2, cellp, fxp, fyp, nd, w);
        wave_ordered_add(bacc, tag, nd, w * v);
      }
    } else if (n2 == 4) {
      int nd[16];
      double ww[16];
      if (rc >= 0) {
        pixel_pairs4(t, ns, cellp, fxp, fyp, nd, ww);
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          nd[q] = -1;
          ww[q] = 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) wave_ordered_add(bacc, tag, nd[q], ww[q] * v);
    } else {
      int node[4 * SL_MAX_NSUB * SL_MAX_NSUB];
      double wt[4 * SL_MAX_NSUB * SL_MAX_NSUB];
      const int np = rc >= 0 ? pixel_pairs(t, ns, n2, cellp, fxp, fyp, node, wt) : 0;
      int npmax = np;
      for (int o = 32; o > 0; o >>= 1) npmax = max(npmax, __shfl_xor(npmax, o, 64));
      for (int q = 0; q < npmax; ++q) wave_ordered_add(bacc, tag, q < np ? node[q] : -1, q < np ? wt[q] * v : 0.0);
    }
  }
}

template <typename T>
__device__ void prep_member(const SolveArgs& a, int m, MemberInfo mi, const double* gl, int* bbox, int* scan,
                            double* bacc) {
  const int tid = threadIdx.x;
  const int nx = a.nx, ny = a.ny, J = nx * ny, nsub = a.nsub, n2 = a.n2;
  const Lens L = make_lens(gl);
  const int ns = mi.ns;
  const double h = 2.0 * a.R / (ns - 1);
  int32_t* pix = a.pix_list + (long)m * a.slot_cap;
  int32_t* cellp = a.cell + (long)m * a.slot_cap * n2;
  T* fxp = reinterpret_cast<T*>(a.fx) + (long)m * a.slot_cap * n2;
  T* fyp = reinterpret_cast<T*>(a.fy) + (long)m * a.slot_cap * n2;
  // pass 1: count the pixels with at least one subpixel on the grid, and their bounding box
  int count = 0;
  for (int j0 = 0; j0 < J; j0 += blockDim.x) {
    const int j = j0 + tid;
    const int r = j / nx, c = j % nx;
    bool mapped = false;
    if (j < J) {
      for (int k = 0; k < n2; ++k) {
        double x, y, bx, by, fx, fy;
        int cell;
        subpixel_xy(r, c, k / nsub, k % nsub, nx, ny, a.pix, nsub, x, y);
        lens_map(L, x, y, bx, by);
        mapped |= grid_cell((bx + a.R) / h, (by + a.R) / h, ns, cell, fx, fy);
      }
    }
    if (mapped) {
      atomicMin(&bbox[0], r);
      atomicMax(&bbox[1], r);
      atomicMin(&bbox[2], c);
      atomicMax(&bbox[3], c);
    }
    int tot;
    (void)block_excl_count(mapped, scan, &tot);
    count += tot;
  }
  // The table is interleaved: compacted entry pos goes to slot (pos % S) * 64 + pos / S,
  // so the 64 lanes of a wave take pixels spread over the whole mapped region and
  // their L^T atomics rarely hit the same source node; slots past the last entry
  // hold -1.
  const int Mtrue = __builtin_amdgcn_readfirstlane(count);   // block-uniform: branches below enclose barriers
  const int S = (Mtrue + 63) / 64;
  const int slots = 64 * S;
  int base = 0;
  for (int j0 = 0; j0 < J; j0 += blockDim.x) {
    const int j = j0 + tid;
    const int r = j / nx, c = j % nx;
    bool mapped = false;
    if (j < J) {
      for (int k = 0; k < n2; ++k) {
        double x, y, bx, by, fx, fy;
        int cell;
        subpixel_xy(r, c, k / nsub, k % nsub, nx, ny, a.pix, nsub, x, y);
        lens_map(L, x, y, bx, by);
        mapped |= grid_cell((bx + a.R) / h, (by + a.R) / h, ns, cell, fx, fy);
      }
    }
    int tot;
    const int pos = base + block_excl_count(mapped, scan, &tot);
    if (mapped) {
      const int slot = (pos % S) * 64 + pos / S;
      pix[slot] = (r << 16) | c;   // packed row/column of the mapped pixel
      for (int k = 0; k < n2; ++k) {
        double x, y, bx, by, fx = 0.0, fy = 0.0;
        int cell = -1;
        subpixel_xy(r, c, k / nsub, k % nsub, nx, ny, a.pix, nsub, x, y);
        lens_map(L, x, y, bx, by);
        if (!grid_cell((bx + a.R) / h, (by + a.R) / h, ns, cell, fx, fy)) {
          cell = -1;
          fx = fy = 0.0;
        } else if (a.interp == SL_INTERP_NEAREST) {   // the nearest of the cell's four nodes, weight 1
          fx = fx >= 0.5 ? 1.0 : 0.0;
          fy = fy >= 0.5 ? 1.0 : 0.0;
        }
        cellp[(long)slot * n2 + k] = cell;
        fxp[(long)slot * n2 + k] = (T)fx;
        fyp[(long)slot * n2 + k] = (T)fy;
      }
    }
    base += tot;
  }
  for (int sl_ = tid; sl_ < slots; sl_ += blockDim.x) {
    if ((sl_ % 64) * S + sl_ / 64 >= Mtrue) {
      pix[sl_] = -1;
      for (int k = 0; k < n2; ++k) {
        cellp[(long)sl_ * n2 + k] = -1;
        fxp[(long)sl_ * n2 + k] = (T)0;
        fyp[(long)sl_ * n2 + k] = (T)0;
      }
    }
  }
  __syncthreads();
  const int Mm = slots;
  // right-hand side b = L^T B^T d (FP64): B^T d at the mapped pixels by every
  // thread, then the scatter over the nodes in a fixed order by wave 0.  The
  // per-slot values go to this member's L^T entry region, which
  // build_transpose fills only later (it holds >= 8 slot_cap bytes).
  const int I = ns * ns;
  double* vbuf = reinterpret_cast<double*>(reinterpret_cast<LtEntry<T>*>(a.lt_ent) + (long)m * a.lt_cap);
  // conflict tags of lane_rank, past the accumulator and the transpose build's arrays
  int* tag = a.prep_tags ? reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(bacc) + 8L * a.I_max + 768)
                         : nullptr;
  for (int i = tid; i < I; i += blockDim.x) bacc[i] = 0.0;
  correlate_slots(a, a.d, Mm, pix, vbuf);
  __syncthreads();
  if (tid < 64) rhs_fixed_order<T>(a, vbuf, ns, Mm, pix, cellp, fxp, fyp, bacc, tag);
  __syncthreads();
  const double inv_n2 = 1.0 / n2;
  // scale of the spectral preconditioner: c = sum_i cov_i b_i^2 / sum_i b_i^2
  // with cov = L^T 1 (the bilinear weight each node receives), a cheap
  // stand-in for the Rayleigh quotient <b, L^T B^T B L b> / <b, b>
  {
    __shared__ double pcred[32];
    double num = 0.0, den = 0.0;
    for (int t = tid; t < Mm; t += blockDim.x) {
      if (pix[t] < 0) continue;
      if (a.interp == SL_INTERP_BICUBIC) {
        for (int q = 0; q < 16 * n2; ++q) {
          int nd;
          double w;
          bicubic_pair(t, q, ns, n2, cellp, fxp, fyp, nd, w);
          if (nd >= 0) num += w * bacc[nd] * bacc[nd];
        }
        continue;
      }
      for (int k = 0; k < n2; ++k) {
        const int cell = cellp[(long)t * n2 + k];
        if (cell < 0) continue;
        const double fx = (double)fxp[(long)t * n2 + k], fy = (double)fyp[(long)t * n2 + k];
        const double b0 = bacc[cell], b1 = bacc[cell + 1], b2 = bacc[cell + ns], b3 = bacc[cell + ns + 1];
        num += ((1 - fx) * (1 - fy) * b0 * b0 + fx * (1 - fy) * b1 * b1 + (1 - fx) * fy * b2 * b2 +
                fx * fy * b3 * b3) * inv_n2;
      }
    }
    for (int i = tid; i < I; i += blockDim.x) den += bacc[i] * bacc[i];
    block_sum2(num, den, pcred);
    if (tid == 0) mi.pc_c = den > 0.0 ? (float)(num / den) : 0.0f;
  }
  double* bm = a.b + (long)m * a.I_max;
  for (int i = tid; i < I; i += blockDim.x) bm[i] = bacc[i];
  __syncthreads();
  if (a.mcn) {   // A^T bhat of the Monte Carlo degrees of freedom, in the same fixed order
    for (int i = tid; i < I; i += blockDim.x) bacc[i] = 0.0;
    correlate_slots(a, a.mcn, Mm, pix, vbuf);
    __syncthreads();
    if (tid < 64) rhs_fixed_order<T>(a, vbuf, ns, Mm, pix, cellp, fxp, fyp, bacc, tag);
    __syncthreads();
    double* bhm = a.bh + (long)m * a.I_max;
    for (int i = tid; i < I; i += blockDim.x) bhm[i] = bacc[i];
    __syncthreads();
  }
  int sell = 0;
  if (Mtrue > 0)
    sell = build_transpose<T>(a, m, ns, Mm, bbox, scan, reinterpret_cast<int*>(bacc), pix, cellp, fxp, fyp, tag);
  if (tid == 0) {
    const int fh = Mtrue > 0 ? bbox[1] - bbox[0] + 1 : 0, fw = Mtrue > 0 ? bbox[3] - bbox[2] + 1 : 0;
    mi.lds_frame = (long)(fh + 4 * a.ckt + kSegR) * ((fw + 4 * a.ckt) | 1) <= a.lds_frame_cap;
    mi.sell = sell;
    mi.M = Mm;
    mi.Mtrue = Mtrue;
    mi.status = Mtrue > 0 ? SL_ST_OK : SL_ST_EMPTY;
    mi.r0 = Mtrue > 0 ? bbox[0] : 0;
    mi.r1 = Mtrue > 0 ? bbox[1] : -1;
    mi.c0 = Mtrue > 0 ? bbox[2] : 0;
    mi.c1 = Mtrue > 0 ? bbox[3] : -1;
    a.minfo[m] = mi;
  }
}

// ------------------------------------------------------------------ banded pass
// In-place pass out(p) = sum_{|d|<=2ck} a[|d|] in(p+d) - edge corrections along
// `nlines` lines of length `len` of the frame interior.  The frame carries a
// zero halo of 2*CKT elements on every side, so windows need no bounds tests.
// `F0` points at interior element (0, 0).  ROW: element (line, p) at
// F0[line*pitch + p]; else F0[p*pitch + line].  Every line is handled by the
// lanes of one wave within one step, so all reads of a line precede its
// writes.  acoef[d + 2*kMaxCK] = a[d].
template <typename T, int CKT, bool ROW>
__device__ __forceinline__ void banded_pass(T* __restrict__ F0, int pitch, int nlines, int len,
                                            int img_off, int img_len, int ck,
                                            const T* __restrict__ acoef, const T* __restrict__ EL,
                                            const T* __restrict__ ER) {
  constexpr int W = kSegR + 4 * CKT;
  constexpr int NH = 2 * CKT;
  T ac[NH + 1];
#pragma unroll
  for (int x = 0; x <= NH; ++x) ac[x] = acoef[2 * kMaxCK + x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int S = (len + kSegR - 1) / kSegR;
  const int LPW = 64 / S;
  // consecutive lanes walk consecutive lines (odd pitch / unit stride: no LDS
  // bank conflicts); the segments of one line stay in one wave step
  const int sub_line = lane % LPW, seg = lane / LPW;
  const int p0 = seg * kSegR;
  const int step = ROW ? 1 : pitch;          // distance between positions
  const int lstride = ROW ? pitch : 1;       // distance between lines
  const bool edges = img_off < ck || img_off + len > img_len - ck;
  for (int l0 = wv * LPW; l0 < nlines; l0 += (kNTof<T> / kWave) * LPW) {   // same trip count for the whole wave
    const int line = l0 + sub_line;
    const bool active = seg < S && line < nlines;
    const T* src = F0 + (active ? line * lstride + (p0 - NH) * step : 0);
    T win[W];
#pragma unroll
    for (int x = 0; x < W; ++x) win[x] = active ? src[x * step] : (T)0;
    T out[kSegR];
#pragma unroll
    for (int o = 0; o < kSegR; ++o) {
      T acc = ac[0] * win[o + NH];
#pragma unroll
      for (int d = 1; d <= NH; ++d) acc += ac[d] * (win[o + NH - d] + win[o + NH + d]);
      out[o] = acc;
    }
    if (active && edges) {
      // outputs within ck of the image border: subtract the part of the
      // autocorrelation that runs through intermediate pixels outside the image
#pragma unroll
      for (int o = 0; o < kSegR; ++o) {
        const int gpos = img_off + p0 + o;
        if (gpos < ck) {
          T corr = 0;
          for (int q = 0; q < ck; ++q) {
            const int pp = q - img_off;
            if (pp >= 0 && pp < len) corr += EL[gpos * ck + q] * F0[line * lstride + pp * step];
          }
          out[o] -= corr;
        }
        if (gpos >= img_len - ck) {
          const int pr = gpos - (img_len - ck);
          T corr = 0;
          for (int q = 0; q < ck; ++q) {
            const int pp = img_len - ck + q - img_off;
            if (pp >= 0 && pp < len) corr += ER[pr * ck + q] * F0[line * lstride + pp * step];
          }
          out[o] -= corr;
        }
      }
    }
    // every lane of the wave has read its window (and edge inputs) before any
    // lane overwrites the line: keep the compiler from sinking loads below here
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (active) {
      T* dst = F0 + line * lstride + p0 * step;
#pragma unroll
      for (int o = 0; o < kSegR; ++o)
        if (p0 + o < len) dst[o * step] = out[o];
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------------ k_solve
template <typename T>
__device__ __forceinline__ T lds_node(const T* P, int ns, int r, int c) {
  return (r < 0 || c < 0 || r >= ns || c >= ns) ? (T)0 : P[r * ns + c];
}

// H^T H p at node (r, c): D2 (x) I + I (x) D2 with the 1-D Dirichlet D2
// (rows [5,-4,1], [-4,6,-4,1], [1,-4,6,-4,1], ...).
template <typename T>
__device__ __forceinline__ T hth_node(const T* P, int ns, int r, int c) {
  const T ctr = P[r * ns + c];
  const T dgx = (T)(6 - (c == 0) - (c == ns - 1));
  const T dgy = (T)(6 - (r == 0) - (r == ns - 1));
  const T n1 = lds_node(P, ns, r, c - 1) + lds_node(P, ns, r, c + 1) + lds_node(P, ns, r - 1, c) +
               lds_node(P, ns, r + 1, c);
  const T n2 = lds_node(P, ns, r, c - 2) + lds_node(P, ns, r, c + 2) + lds_node(P, ns, r - 2, c) +
               lds_node(P, ns, r + 2, c);
  return (dgx + dgy) * ctr - (T)4 * n1 + n2;
}

template <typename T>
__device__ __forceinline__ double reg_node(const T* P, int ns, int r, int c, int reg) {
  const double ctr = (double)P[r * ns + c];
  if (reg == SL_H_IDENTITY) return ctr * ctr;
  const double dx = (double)lds_node(P, ns, r, c - 1) - 2.0 * ctr + (double)lds_node(P, ns, r, c + 1);
  const double dy = (double)lds_node(P, ns, r - 1, c) - 2.0 * ctr + (double)lds_node(P, ns, r + 1, c);
  return dx * dx + dy * dy;
}

// Block-wide FP64 sum with one barrier; consecutive calls must alternate `buf`
// (0/1) and be separated by at least one other barrier before a buffer is reused.
template <int NW = kWaves>
__device__ __forceinline__ double block_sum1(double v, double* scratch, int buf) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  double* sc = scratch + 16 * buf;
  if (lane == 0) sc[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += sc[i];
  return t;
}

// ---------------------------------------------------------------- spectral preconditioner
// H^T H = D^2 (x) I + I (x) D^2 with D = tridiag(1, -2, 1) (Dirichlet second
// differences on an n x n grid).  The orthonormal sine transform S,
// S_jk = sqrt(2/(n+1)) sin(pi (j+1)(k+1) / (n+1)) (symmetric, S S = I),
// diagonalises D: D = S diag(-4 sin^2(pi (k+1) / (2(n+1)))) S, so
// M = c I + lambda H^T H = (S (x) S) diag(c + lambda (mu_j + mu_k)) (S (x) S)
// with mu_k the eigenvalues of D^2, and M^-1 x is two 2-D transforms and a
// division.  With x an n x n array X, (S (x) S) x = S X S.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// C = S B (n x n, row-major B in LDS) on the FP32 matrix cores, stored
// row-major (trans = 0) or transposed (trans = 1); with `scale`, element
// (j, k) is divided by c + lambda (mu_j + mu_k).  S comes from the table
// tab[m] = sqrt(2/(n+1)) sin(pi m / (n+1)), m = (j+1)(k+1) mod 2(n+1).
// Each wave takes 16 x 48 output strips (three 16 x 16 tiles sharing the S
// operand, three independent accumulator chains); the operands of the next
// k-step are loaded before the current step's MFMAs.
// v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element r is C[4 (l/16) + r][l%16].
__device__ __forceinline__ void sine_mul(const float* tab, const float* mu, int n, const float* B, float* C, int trans, int scale,
                         float c, float lam) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lc = lane & 15, lq = lane >> 4;
  const int nt = (n + 15) >> 4, ng = (nt + 2) / 3, nn2 = 2 * (n + 1);
  for (int strip = wv; strip < nt * ng; strip += kWaves) {
    const int i0 = (strip / ng) << 4, jg = (strip % ng) * 48;
    const int i = i0 + lc;
    const int j0 = jg + lc, j1 = j0 + 16, j2 = j0 + 32;
    f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0, acc2 = acc0;
    int mi = ((i + 1) * (lq + 1)) % nn2;          // table index of S[i][t], t = t0 + lq
    const int step = (4 * (i + 1)) % nn2;
    float av = (i < n && lq < n) ? tab[mi] : 0.0f;
    float b0 = (lq < n && j0 < n) ? B[lq * n + j0] : 0.0f;
    float b1 = (lq < n && j1 < n) ? B[lq * n + j1] : 0.0f;
    float b2 = (lq < n && j2 < n) ? B[lq * n + j2] : 0.0f;
    for (int t0 = 0; t0 < n; t0 += 4) {
      mi += step;
      if (mi >= nn2) mi -= nn2;
      const int tn = t0 + 4 + lq;
      const float avn = (i < n && tn < n) ? tab[mi] : 0.0f;
      const float b0n = (tn < n && j0 < n) ? B[tn * n + j0] : 0.0f;
      const float b1n = (tn < n && j1 < n) ? B[tn * n + j1] : 0.0f;
      const float b2n = (tn < n && j2 < n) ? B[tn * n + j2] : 0.0f;
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b1, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b2, acc2, 0, 0, 0);
      av = avn;
      b0 = b0n;
      b1 = b1n;
      b2 = b2n;
    }
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const f32x4 acc = g == 0 ? acc0 : (g == 1 ? acc1 : acc2);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * lq + r, col = jg + 16 * g + lc;
        if (row < n && col < n) {
          float v = acc[r];
          if (scale) v = v / (c + lam * (mu[row] + mu[col]));
          if (trans)
            C[col * n + row] = v;
          else
            C[row * n + col] = v;
        }
      }
    }
  }
}

// One preconditioned-CG direction update, all threads of the block:
// z = M^-1 r (r from r_g, the n x n scratch T in the frame, X = the Q region),
// rz_new = <r, z>, p = z + beta p with beta = rz_new / rz_old (0 when
// `restart`), and the scratch zeroed again.  Returns rz_new.  Kept out of
// line so that its registers do not add to the CG loop's pressure.
__device__ __attribute__((noinline)) double pc_apply(float* P, float* X, float* Tb, const float* tab,
                                                     const float* mu, int n, const float* r_g, float c, float lam,
                                                     double rz_old, int restart, double* red) {
  const int tid = threadIdx.x, nn = n * n;
  for (int i = tid; i < nn; i += kNT) X[(i % n) * n + i / n] = r_g[i];   // X^T
  __syncthreads();
  // every product is S B; the stored transposes make the next B row-major
  sine_mul(tab, mu, n, X, Tb, 1, 0, 0.0f, 0.0f);     // (S X^T)^T = X S
  __syncthreads();
  sine_mul(tab, mu, n, Tb, X, 0, 1, c, lam);         // Y = S X S over the eigenvalues of M
  __syncthreads();
  sine_mul(tab, mu, n, X, Tb, 1, 0, 0.0f, 0.0f);     // (S Y)^T
  __syncthreads();
  sine_mul(tab, mu, n, Tb, X, 1, 0, 0.0f, 0.0f);     // (S (S Y)^T)^T = S Y S = z, node order
  __syncthreads();
  double rzn = 0.0;
  for (int i = tid; i < nn; i += kNT) rzn += (double)r_g[i] * (double)X[i];
  rzn = block_sum1(rzn, red, 2);
  const float beta = restart ? 0.0f : (float)(rzn / rz_old);
  for (int i = tid; i < nn; i += kNT) P[i] = X[i] + beta * P[i];
  for (int e = tid; e < nn; e += kNT) Tb[e] = 0.0f;   // the scratch lies in the frame
  return rzn;
}

// Bicubic value of the n x n subpixels of mapped pixel t: for each subpixel
// the 4 x 4 nodes about its cell, weighted by the cubic convolution kernel in
// x and y, nodes outside the grid left out.
template <typename T>
__device__ __forceinline__ T pixel_gather_cubic(const T* X, int ns, int n2, int t, const int32_t* cellp,
                                                const T* fxp, const T* fyp) {
  T acc = 0;
#pragma unroll 1
  for (int k = 0; k < n2; ++k) {
    const int c = cellp[(long)t * n2 + k];
    if (c < 0) continue;
    const T fx = fxp[(long)t * n2 + k], fy = fyp[(long)t * n2 + k];
    const int r = c / ns, col = c % ns;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      const int rr = r + j - 1;
      if (rr < 0 || rr >= ns) continue;
      T row = 0;
#pragma unroll 1
      for (int i = 0; i < 4; ++i) {
        const int cc = col + i - 1;
        if (cc >= 0 && cc < ns) row += keys_w(fabs(fx - (T)(i - 1))) * X[rr * ns + cc];
      }
      acc += keys_w(fabs(fy - (T)(j - 1))) * row;
    }
  }
  return acc;
}

// Interpolated value of the n x n subpixels of mapped pixel t: sum_k w_k . x[cell_k..]
// (bilinear weights, or the nearest node's weight 1; bicubic when `cubic`)
template <typename T>
__device__ __forceinline__ T pixel_gather(const T* X, int ns, int n2, int t, const int32_t* cellp, const T* fxp,
                                          const T* fyp, bool cubic) {
  if (cubic) return pixel_gather_cubic(X, ns, n2, t, cellp, fxp, fyp);
  T acc = 0;
  if (n2 == 4) {
    const int4 c4 = reinterpret_cast<const int4*>(cellp)[t];
    T fx[4], fy[4];
    if constexpr (sizeof(T) == 4) {
      const float4 a4 = reinterpret_cast<const float4*>(fxp)[t];
      const float4 b4 = reinterpret_cast<const float4*>(fyp)[t];
      fx[0] = a4.x; fx[1] = a4.y; fx[2] = a4.z; fx[3] = a4.w;
      fy[0] = b4.x; fy[1] = b4.y; fy[2] = b4.z; fy[3] = b4.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        fx[k] = fxp[4L * t + k];
        fy[k] = fyp[4L * t + k];
      }
    }
    const int cl[4] = {c4.x, c4.y, c4.z, c4.w};
    // branch-free: an off-grid subpixel (cell -1) reads node 0 and adds zero
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = max(cl[k], 0);
      const T v = (1 - fy[k]) * ((1 - fx[k]) * X[c] + fx[k] * X[c + 1]) +
                  fy[k] * ((1 - fx[k]) * X[c + ns] + fx[k] * X[c + ns + 1]);
      acc += cl[k] >= 0 ? v : (T)0;
    }
    return acc;
  }
  for (int k = 0; k < n2; ++k) {
    const int c = cellp[(long)t * n2 + k];
    if (c < 0) continue;
    const T fx = fxp[(long)t * n2 + k], fy = fyp[(long)t * n2 + k];
    acc += (1 - fy) * ((1 - fx) * X[c] + fx * X[c + 1]) + fy * ((1 - fx) * X[c + ns] + fx * X[c + ns + 1]);
  }
  return acc;
}

// Invalid or empty member: s = 0, chi^2 = sum d^2 / sigma^2 (no barriers).
template <typename T>
__device__ void trivial_item(const SolveArgs& a, const MemberInfo& mi, int m, int kl) {
  const long out_idx = (long)m * a.n_lambda + kl;
  T* s_dst = reinterpret_cast<T*>(a.s_all) + out_idx * a.I_max;
  for (int i = threadIdx.x; i < mi.I; i += kNTof<T>) s_dst[i] = (T)0;
  if (threadIdx.x == 0) {
    a.chi2[out_idx] = mi.status == SL_ST_INVALID ? NAN : a.consts->sum_d2 / (a.sigma * a.sigma);
    a.regv[out_idx] = mi.status == SL_ST_INVALID ? NAN : 0.0;
    a.iters[out_idx] = 0;
    a.status[out_idx] = mi.status;
  }
}

// One CG solve of a valid member.  Every branch that encloses a barrier
// depends only on block-uniform values made scalar with readfirstlane.
// LDS: P = search direction p, Q = A p accumulator, the image frame (LDSF)
// and reduction scratch.  The iterate s (in its output slot) and the
// residual r live in global memory, read and written by their owner thread.
// The operands of one item's regularised normal operator (see apply_normal).
template <typename T>
struct OpView {
  const int32_t* pix;        // mapped-pixel slots: packed (row << 16 | col), -1 past the end
  const int32_t* cellp;      // [slot][n^2] bilinear cell of each subpixel, -1 off the grid
  const T* fxp;
  const T* fyp;
  T* F;                      // image frame with its zero halo (LDS or global)
  T* F0;                     // frame interior (0, 0) = image pixel (r0, c0)
  T* Z;                      // per-block image buffer of the direct blur (z = B y on the dilated box)
  T* W;                      // per-block image buffer of the direct blur (B^T z on the bounding box)
  const T* taps;
  const int32_t* lt_rp;      // transposed operator: slice (or row) starts
  const LtEntry<T>* lt_e;    //                      entries
  const int32_t* perm;       //                      nodes in slice order
  int ns, I, M, r0, c0, h, w, pitch, fo, n2, nx, ny, K, ck, sell, Dr0, Dc0, Dh, Dw;
  bool sep, ident;
  T inv_n2, lamT;
  bool cubic;                // bicubic L (16 nodes per subpixel); else bilinear or nearest
};

// y = L p into the frame: every mapped pixel is written once (assignment, so
// the frame outside the mapped pixels keeps whatever it held, zero unless a
// banded pass wrote it).  Two pixels per thread and step so that their table
// loads are in flight together.
// The bicubic form, out of line: its 16 taps per subpixel stay out of the
// register budget of the persistent kernels that inline the other forms.
template <typename T, int NT>
__device__ __attribute__((noinline)) void gather_L_cubic(const int32_t* pix, const int32_t* cellp, const T* fxp,
                                                        const T* fyp, T* F0, const T* P, int M, int ns, int n2,
                                                        int pitch, int fo, T inv_n2) {
  for (int t = threadIdx.x; t < M; t += NT) {
    const int rc = pix[t];
    if (rc >= 0) F0[(rc >> 16) * pitch + (rc & 0xFFFF) + fo] = pixel_gather_cubic(P, ns, n2, t, cellp, fxp, fyp) * inv_n2;
  }
}

// CUBIC = false compiles the bicubic branch out (the banded-blur kernels: a
// bicubic problem always takes the direct form).
template <typename T, int NT, bool CUBIC = true>
__device__ __forceinline__ void gather_L(const OpView<T>& o, const T* __restrict__ P) {
  const int32_t* pix = o.pix;
  T* const F0 = o.F0;
  const int M = o.M, ns = o.ns, n2 = o.n2, pitch = o.pitch, fo = o.fo;
  const T inv_n2 = o.inv_n2;
  if constexpr (CUBIC) {
    if (o.cubic) {
      gather_L_cubic<T, NT>(pix, o.cellp, o.fxp, o.fyp, F0, P, M, ns, n2, pitch, fo, inv_n2);
      return;
    }
  }
  for (int t = threadIdx.x; t < M; t += 2 * NT) {
    const int t2 = t + NT;
    const int rc = pix[t];
    const int rc2 = t2 < M ? pix[t2] : -1;
    const T v1 = pixel_gather(P, ns, n2, t, o.cellp, o.fxp, o.fyp, false);
    const T v2 = t2 < M ? pixel_gather(P, ns, n2, t2, o.cellp, o.fxp, o.fyp, false) : (T)0;
    if (rc >= 0) F0[(rc >> 16) * pitch + (rc & 0xFFFF) + fo] = v1 * inv_n2;
    if (rc2 >= 0) F0[(rc2 >> 16) * pitch + (rc2 & 0xFFFF) + fo] = v2 * inv_n2;
  }
}

// z = B y over the dilated box (Dh x Dw, row-major) from the frame, whose
// entries off the mapped pixels are zero.  Returns this thread's part of
// ||z||^2.
template <typename T, int CKT, int NT>
__device__ __forceinline__ double blur_box(const OpView<T>& o, T* __restrict__ Z) {
  const T* const F0 = o.F0;
  const T* taps = o.taps;
  const TapIdx ti(o.K);
  const int K = o.K, ck = o.ck, r0 = o.r0, c0 = o.c0, h = o.h, w = o.w, pitch = o.pitch;
  const int Dr0 = o.Dr0, Dc0 = o.Dc0, Dh = o.Dh, Dw = o.Dw;
  double zz = 0.0;
  for (int e = threadIdx.x; e < Dh * Dw; e += NT) {
    const int rr_ = Dr0 + e / Dw, cc_ = Dc0 + e % Dw;
    T acc = 0;
    if (ck <= CKT) {
      // every tap of an output in the dilated region lands in the bounding
      // box or its zero halo (2 CKT >= 2 ck on each side): no bounds tests
      const T* yrow = F0 + (rr_ + ck - r0) * pitch + (cc_ + ck - c0);
      const T* tp = taps + ti.psf;
      for (int aa = 0; aa < K; ++aa) {
        const T* y = yrow - aa * pitch;
        for (int bb = 0; bb < K; ++bb) acc += tp[aa * K + bb] * y[-bb];
      }
    } else {   // PSFs wider than the widest compiled window: the halo is narrower than ck
      for (int aa = 0; aa < K; ++aa) {
        const int yr = rr_ - aa + ck - r0;
        if (yr < 0 || yr >= h) continue;
        for (int bb = 0; bb < K; ++bb) {
          const int yc = cc_ - bb + ck - c0;
          if (yc < 0 || yc >= w) continue;
          acc += taps[ti.psf + aa * K + bb] * F0[yr * pitch + yc];
        }
      }
    }
    Z[e] = acc;
    zz += (double)acc * (double)acc;
  }
  return zz;
}

// w = B^T z at the mapped pixels, into the frame; z lives on the dilated box.
template <typename T, int NT>
__device__ __forceinline__ void blur_T_mapped(const OpView<T>& o, const T* __restrict__ Z) {
  const int32_t* pix = o.pix;
  T* const F0 = o.F0;
  const T* taps = o.taps;
  const TapIdx ti(o.K);
  const int K = o.K, ck = o.ck, pitch = o.pitch, fo = o.fo, M = o.M;
  const int Dr0 = o.Dr0, Dc0 = o.Dc0, Dh = o.Dh, Dw = o.Dw;
  for (int t = threadIdx.x; t < M; t += NT) {
    if (pix[t] < 0) continue;
    const int rr_ = pix[t] >> 16, cc_ = pix[t] & 0xFFFF;
    T acc = 0;
    for (int aa = 0; aa < K; ++aa) {
      const int zr = rr_ + aa - ck - Dr0;
      if (zr < 0 || zr >= Dh) continue;
      for (int bb = 0; bb < K; ++bb) {
        const int zc = cc_ + bb - ck - Dc0;
        if (zc < 0 || zc >= Dw) continue;
        acc += taps[ti.psf + aa * K + bb] * Z[zr * Dw + zc];
      }
    }
    F0[rr_ * pitch + cc_ + fo] = acc;
  }
}

// q = L^T w + lambda H^T H p gathered per node from the transposed operator
// (no atomics, fixed order), stored in Q.  Returns this thread's part of
// <p, q>.  With GRAD, q = L^T w alone (no P term) and the return value is
// this thread's part of ||q||^2.
template <typename T, int NT, bool GRAD>
__device__ __forceinline__ double gather_LT(const OpView<T>& o, const T* __restrict__ P, T* __restrict__ Q) {
  const int tid = threadIdx.x;
  const T* const F = o.F;
  const int32_t* lt_rp = o.lt_rp;
  const LtEntry<T>* lt_e = o.lt_e;
  const int32_t* perm = o.perm;
  const int ns = o.ns, I = o.I, sell = o.sell;
  const bool ident = o.ident;
  const T lamT = o.lamT;
  double pq = 0.0;
  if (sell) {
    // sliced-ELL in length-sorted node order: wave w takes slices w, w + 16, ...;
    // the slice bounds are wave-uniform (scalar loads) and every lane of a
    // slice has `len` entries (padding reads the zero halo), eight in flight
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nslices = (I + 63) >> 6;
    const int lt_E = lt_rp[nslices];   // sliced-ELL entries of the member
    for (int sl = wid; sl < nslices; sl += NT / 64) {
      const int idx = sl * 64 + lane;
      const int b0 = lt_rp[sl];
      const int len = (lt_rp[sl + 1] - b0) >> 6;
      const int pk = idx < I ? perm[idx] : 0;
      T acc = 0;
      if (sizeof(T) == 4 && sell == 2) {
        // paired entries (even `len`, entries summed in the same order)
        const unsigned* op = reinterpret_cast<const unsigned*>(lt_e) + (b0 >> 1) + lane;
        const float2* wq = reinterpret_cast<const float2*>(reinterpret_cast<const unsigned*>(lt_e) + (lt_E >> 1)) +
                           (b0 >> 1) + lane;
        const int npair = len >> 1;
        int j = 0;
        for (; j + 7 < npair; j += 8) {   // sixteen entries in flight
          unsigned ov[8];
          float2 wv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            ov[u] = op[64L * (j + u)];
            wv[u] = wq[64L * (j + u)];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            acc += (T)wv[u].x * F[ov[u] & 0xFFFFu];
            acc += (T)wv[u].y * F[ov[u] >> 16];
          }
        }
        for (; j < npair; ++j) {
          const unsigned o0 = op[64L * j];
          const float2 w0 = wq[64L * j];
          acc += (T)w0.x * F[o0 & 0xFFFFu];
          acc += (T)w0.y * F[o0 >> 16];
        }
      } else {
        const LtEntry<T>* ep = lt_e + b0 + lane;
        int j = 0;
        for (; j + 7 < len; j += 8) {
          LtEntry<T> x[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) x[u] = ep[64L * (j + u)];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc += x[u].w * F[x[u].off];
        }
        for (; j < len; ++j) {
          const LtEntry<T> x0 = ep[64L * j];
          acc += x0.w * F[x0.off];
        }
      }
      if (idx < I) {
        const int rn_ = pk >> 16, cn_ = pk & 0xFFFF, i = rn_ * ns + cn_;
        if (GRAD) {
          Q[i] = acc;
          pq += (double)acc * (double)acc;
        } else {
          const T pv = P[i];
          const T qv = acc + lamT * (ident ? pv : hth_node(P, ns, rn_, cn_));
          Q[i] = qv;
          pq += (double)pv * (double)qv;
        }
      }
    }
  } else {
    for (int i = tid; i < I; i += NT) {
      T acc = 0;
      const int e0 = lt_rp[i], e1 = lt_rp[i + 1];
      for (int e = e0; e < e1; ++e) acc += lt_e[e].w * F[lt_e[e].off];
      if (GRAD) {
        Q[i] = acc;
        pq += (double)acc * (double)acc;
      } else {
        const int rn_ = i / ns, cn_ = i - rn_ * ns;
        const T pv = P[i];
        const T qv = acc + lamT * (ident ? pv : hth_node(P, ns, rn_, cn_));
        Q[i] = qv;
        pq += (double)pv * (double)qv;
      }
    }
  }
  return pq;
}

// Register-tiled direct K x K forms, for a PSF of exactly KT = 2 CKT + 1
// taps per side.  Each thread computes eight consecutive outputs of one row
// from a window of KT + 7 values per input row, so that one load serves up
// to eight products; consecutive lanes take consecutive rows, so with the
// odd frame pitch their LDS reads fall in distinct banks.  The last tile of a
// row starts at width - 8: tiles overlap there and write the same values
// twice.  Each output sums its taps in the order of the per-output forms
// (row of the PSF outer, column inner), so the results are the same.
// Usable when ck == CKT and both the box and the dilated box are at least 8
// wide (tiled_ok).
template <typename T, int CKT>
__device__ __forceinline__ bool tiled_ok(const OpView<T>& o) {
  return o.ck == CKT && o.w >= 8 && o.Dw >= 8;
}

// z = B y over the dilated box into Z (Dh x Dw, row-major), y in the frame
// with its zero halo.  Returns this thread's part of ||z||^2 (each output
// counted once).
template <typename T, int CKT, int NT>
__device__ __forceinline__ double blur_box_t8(const OpView<T>& o, T* __restrict__ Z) {
  constexpr int KT = 2 * CKT + 1, NV = KT + 7;
  const int Dh = o.Dh, Dw = o.Dw, pitch = o.pitch;
  const T* tp = o.taps + TapIdx(KT).psf;
  // output (r, c) of the dilated box reads base[(r - aa) * pitch + (c - bb)]
  const T* base = o.F0 + (o.Dr0 + CKT - o.r0) * pitch + (o.Dc0 + CKT - o.c0);
  const int nct = (Dw + 7) >> 3;
  double zz = 0.0;
  for (int t = threadIdx.x; t < Dh * nct; t += NT) {
    const int r = t % Dh;
    const int cn = (t / Dh) * 8;          // nominal tile start
    const int c = min(cn, Dw - 8);
    T acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0;
    for (int aa = 0; aa < KT; ++aa) {
      const T* row = base + (r - aa) * pitch + c - (KT - 1);
      T v[NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) v[j] = row[j];
      const T* ta = tp + aa * KT;
#pragma unroll
      for (int bb = 0; bb < KT; ++bb) {
        const T tv = ta[bb];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] += tv * v[i - bb + KT - 1];
      }
    }
    T* zo = Z + r * Dw + c;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      zo[i] = acc[i];
      if (c + i >= cn) zz += (double)acc[i] * (double)acc[i];
    }
  }
  return zz;
}

// w = B^T z over the bounding box (h x w) into W (row-major, pitch w), z
// staged in the frame over the dilated box with zeros beyond it.
template <typename T, int CKT, int NT>
__device__ __forceinline__ void blurT_box_t8(const OpView<T>& o, T* __restrict__ W) {
  constexpr int KT = 2 * CKT + 1, NV = KT + 7;
  const int h = o.h, w = o.w, pitch = o.pitch;
  const T* tp = o.taps + TapIdx(KT).psf;
  // output (r, c) of the box reads base[(r + aa) * pitch + (c + bb)]
  const T* base = o.F0 - CKT * pitch - CKT;
  const int nct = (w + 7) >> 3;
  for (int t = threadIdx.x; t < h * nct; t += NT) {
    const int r = t % h;
    const int c = min((t / h) * 8, w - 8);
    T acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0;
    for (int aa = 0; aa < KT; ++aa) {
      const T* row = base + (r + aa) * pitch + c;
      T v[NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) v[j] = row[j];
      const T* ta = tp + aa * KT;
#pragma unroll
      for (int bb = 0; bb < KT; ++bb) {
        const T tv = ta[bb];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] += tv * v[i + bb];
      }
    }
    T* wo = W + r * w + c;
#pragma unroll
    for (int i = 0; i < 8; ++i) wo[i] = acc[i];
  }
}

// frame over the dilated box = Z (Dh x Dw, row-major)
template <typename T, int NT>
__device__ __forceinline__ void stage_dilated(const OpView<T>& o, const T* __restrict__ Z) {
  const int Dw = o.Dw, pitch = o.pitch;
  T* const D0 = o.F0 + (o.Dr0 - o.r0) * pitch + (o.Dc0 - o.c0);
  for (int e = threadIdx.x; e < o.Dh * Dw; e += NT) D0[(e / Dw) * pitch + e % Dw] = Z[e];
}

// frame over the bounding box = W (h x w, row-major)
template <typename T, int NT>
__device__ __forceinline__ void stage_box(const OpView<T>& o, const T* __restrict__ W) {
  const int w = o.w, pitch = o.pitch;
  for (int e = threadIdx.x; e < o.h * w; e += NT) o.F0[(e / w) * pitch + e % w] = W[e];
}

// Frame = B^T z at (at least) the mapped pixels, z on the dilated box in Zs.
// The tiled form writes the whole dilated box (z there, B^T z over the
// bounding box), so afterwards the rows of the dilated box must be zeroed
// before the next L gather (clear_rows); the per-output form writes the
// mapped pixels only.  Ends with a barrier.
template <typename T, int CKT, int NT>
__device__ __forceinline__ void adjoint_blur(const OpView<T>& o, const T* __restrict__ Zs) {
  if (tiled_ok<T, CKT>(o)) {   // uniform: scalar member values
    stage_dilated<T, NT>(o, Zs);
    __syncthreads();
    blurT_box_t8<T, CKT, NT>(o, o.W);
    __syncthreads();
    stage_box<T, NT>(o, o.W);
  } else {
    blur_T_mapped<T, NT>(o, Zs);
  }
  __syncthreads();
}

// z = B y over the dilated box into Z; returns this thread's part of ||z||^2.
template <typename T, int CKT, int NT>
__device__ __forceinline__ double forward_blur(const OpView<T>& o, T* __restrict__ Z) {
  if (tiled_ok<T, CKT>(o)) return blur_box_t8<T, CKT, NT>(o, Z);
  return blur_box<T, CKT, NT>(o, Z);
}

// Zero the frame rows that an operator application wrote, after every
// gather has read the frame: the bounding box's rows (full pitch), and after
// the tiled direct blur (DIR: the direct forms ran; the tiled one stages z
// there) also the ck rows above and below them.  The tiled form needs
// ck == CKT, so those rows lie inside the frame's 2 CKT halo; the other forms
// write inside the box only.
template <typename T, int CKT, int NT, bool DIR>
__device__ __forceinline__ void clear_rows(const OpView<T>& o) {
  const int up = (DIR && tiled_ok<T, CKT>(o)) ? o.ck : 0;
  T* const R0 = o.F0 - (up * o.pitch + 2 * CKT);   // column 0 of frame row 2 CKT - up
  const int n = (o.h + 2 * up) * o.pitch;
  for (int e = threadIdx.x; e < n; e += NT) R0[e] = (T)0;
}

// Q = (L^T B^T B L + lambda H^T H) P for one item, all threads of the block:
// L as a gather into the frame (zero on entry), B^T B in place (banded passes
// for a rank-1 PSF, else the direct K x K form through Z), then L^T as a
// gather over the transposed operator (fixed order, no atomics) fused with
// lambda H^T H.  DIR selects the form (a kernel instantiation of each runs,
// the one that does not match the problem returning at entry, so that the
// banded kernels carry none of the direct form's registers).  On return the
// frame holds B^T B L P (the direct form also
// leaves z in the rows of the dilated box); the caller zeroes the rows of the
// dilated box (clear_rows) after a barrier.  Returns this thread's part of
// <P, Q>.
template <typename T, int CKT, int NT, bool DIR>
__device__ __forceinline__ double apply_normal(const OpView<T>& o, const T* __restrict__ P, T* __restrict__ Q) {
  gather_L<T, NT, DIR>(o, P);
  __syncthreads();
  if constexpr (!DIR) {   // the kernels of the banded form run only when the PSF is separable
    // w = B^T B y: banded pass along rows then along columns, in place
    const TapIdx ti(o.K);
    banded_pass<T, CKT, true>(o.F0, o.pitch, o.h, o.w, o.c0, o.nx, o.ck, o.taps + ti.ax, o.taps + ti.elx,
                              o.taps + ti.erx);
    __syncthreads();
    banded_pass<T, CKT, false>(o.F0, o.pitch, o.w, o.h, o.r0, o.ny, o.ck, o.taps + ti.ay, o.taps + ti.ely,
                               o.taps + ti.ery);
    __syncthreads();
  } else {
    forward_blur<T, CKT, NT>(o, o.Z);  // z = B y over the dilated region into global Z
    __syncthreads();
    adjoint_blur<T, CKT, NT>(o, o.Z);  // w = B^T z (at least) at the mapped pixels, in the frame
  }
  return gather_LT<T, NT, false>(o, P, Q);
}

template <typename T, int CKT, bool LDSF, bool PC, bool DIR>
__device__ __forceinline__ void run_item(const SolveArgs& a, const MemberInfo& mi, int m, int kl, unsigned char* smem) {
  constexpr int NT = kNTof<T>;   // threads of this block
  const int tid = threadIdx.x;
  const long out_idx = (long)m * a.n_lambda + kl;
  T* __restrict__ s_g = reinterpret_cast<T*>(a.s_all) + out_idx * a.I_max;
  // per-block scratch: the preconditioned launch runs beside the plain one and
  // takes the second half of the slots
  const long slot = (long)blockIdx.x + (PC ? (long)gridDim.x : 0L);
  T* __restrict__ r_g = reinterpret_cast<T*>(a.rbuf) + slot * a.I_max;
  const int ns = mi.ns, I = mi.I, M = mi.M, r0 = mi.r0, c0 = mi.c0;
  const int h = mi.r1 - mi.r0 + 1, w = mi.c1 - mi.c0 + 1;
  constexpr int HALO = 2 * CKT;
  const int pitch = (w + 2 * HALO) | 1;
  // kSegR extra rows absorb the tail of the last column window
  const int frame_elems = (h + 2 * HALO + kSegR) * pitch;
  const int J = a.nx * a.ny, n2 = a.n2, nx = a.nx, ny = a.ny, K = a.K, ck = a.ck;
  const T lamT = (T)a.lamv[kl];
  const bool ident = a.reg == SL_H_IDENTITY;
  T* P = reinterpret_cast<T*>(smem);
  T* Q = reinterpret_cast<T*>(smem + a.q_off);
  double* red = reinterpret_cast<double*>(smem + a.red_off);
  T* F;
  if (LDSF)
    F = reinterpret_cast<T*>(smem + a.frame_off);
  else
    F = reinterpret_cast<T*>(a.gframe) + (long)blockIdx.x * a.gframe_elems;
  T* const F0 = F + HALO * pitch + HALO;        // interior (0, 0) = image (r0, c0)
  T* const Frows = F + HALO * pitch;            // interior rows, contiguous
  T* Z = reinterpret_cast<T*>(a.gz) + slot * 2L * J;   // z, then W = B^T z (direct blur)
  const int32_t* pix = a.pix_list + (long)m * a.slot_cap;
  const int32_t* cellp = a.cell + (long)m * a.slot_cap * n2;
  const T* fxp = reinterpret_cast<const T*>(a.fx) + (long)m * a.slot_cap * n2;
  const T* fyp = reinterpret_cast<const T*>(a.fy) + (long)m * a.slot_cap * n2;
  const T* taps = reinterpret_cast<const T*>(a.taps_t);
  const TapIdx ti(K);
  const bool sep = a.consts->sep != 0;
  const T inv_n2 = (T)1 / (T)n2;
  const int fo = -r0 * pitch - c0;             // frame offset of image pixel (r, c): r*pitch + c + fo
  const int32_t* lt_rp = a.lt_ptr + (long)m * (a.I_max + 65);
  const int sell = __builtin_amdgcn_readfirstlane(mi.sell);
  const LtEntry<T>* lt_e = reinterpret_cast<const LtEntry<T>*>(a.lt_ent) + (long)m * a.lt_cap;
  // dilated region (direct-blur paths): rows/cols within ck of the bbox, inside the image
  const int Dr0 = max(mi.r0 - ck, 0), Dr1 = min(mi.r1 + ck, ny - 1);
  const int Dc0 = max(mi.c0 - ck, 0), Dc1 = min(mi.c1 + ck, nx - 1);
  const int Dh = Dr1 - Dr0 + 1, Dw = Dc1 - Dc0 + 1;

  // s = 0, r = p = b, Q = 0, frame (with its halo) = 0
  for (int e = tid; e < frame_elems; e += NT) F[e] = (T)0;
  double rr = 0.0;
  const double* bm = a.b + (long)m * a.I_max;
  for (int i = tid; i < I; i += NT) {
    const T bv = (T)bm[i];
    P[i] = bv;
    Q[i] = (T)0;
    s_g[i] = (T)0;
    r_g[i] = bv;
    rr += (double)bv * (double)bv;
  }
  rr = block_sum1<NT / kWave>(rr, red, 0);
  const double stop2 = a.tol * a.tol * rr;
  // PC: preconditioned CG with M = c I + lambda H^T H (FP32, curvature H; the
  // caller checks that the frame holds the n x n scratch): p0 = z0 = M^-1 b.
  double rz = rr;                                       // <r, z>
  if constexpr (PC && sizeof(T) == 4) {
    float* tab = reinterpret_cast<float*>(smem + a.pc_off);
    float* mu = tab + 2 * (ns + 1);
    const double nrm = sqrt(2.0 / (ns + 1)), pi = 3.14159265358979323846;
    for (int e = tid; e < 2 * (ns + 1); e += NT) tab[e] = (float)(nrm * sin(pi * e / (ns + 1)));
    for (int e = tid; e < ns; e += NT) {
      const double sn = sin(pi * (e + 1) / (2.0 * (ns + 1)));
      mu[e] = (float)(16.0 * sn * sn * sn * sn);
    }
    rz = pc_apply(reinterpret_cast<float*>(P), reinterpret_cast<float*>(Q), reinterpret_cast<float*>(F), tab, mu, ns,
                  reinterpret_cast<const float*>(r_g), mi.pc_c, (float)a.lamv[kl], 0.0, 1, red);
    __syncthreads();
  }
  int st = SL_ST_MAXIT, it = 0;
  for (it = 0; it < a.maxit; ++it) {
    if (__builtin_amdgcn_readfirstlane((int)(rr <= stop2))) {
      st = SL_ST_OK;
      break;
    }
    const OpView<T> ov{pix, cellp, fxp, fyp, F, F0, Z, Z + J, taps, lt_rp, lt_e, a.lt_perm + (long)m * a.I_max, ns,
                       I, M, r0, c0, h, w, pitch, fo, n2, nx, ny, K, ck, sell, Dr0, Dc0, Dh, Dw, sep, ident, inv_n2,
                       lamT, a.interp == SL_INTERP_BICUBIC};
    double pq = apply_normal<T, CKT, NT, DIR>(ov, P, Q);
    pq = block_sum1<NT / kWave>(pq, red, 0);
    // every gather has read the frame (barrier above): back to zero for the next iteration
    clear_rows<T, CKT, NT, DIR>(ov);
    if (__builtin_amdgcn_readfirstlane((int)!(pq > 0.0))) {
      st = SL_ST_BREAKDOWN;
      break;
    }
    const T alT = (T)((PC ? rz : rr) / pq);
    // Updates in chunks of kUpd nodes per thread: every global load of a chunk
    // is issued before the first use, and the updated residual stays in
    // registers for the direction update when the chunk covers all of I.
    double rn = 0.0;
    T rk[kUpd];
    for (int i0 = tid; i0 < I; i0 += kUpd * NT) {
      T sk[kUpd];
#pragma unroll
      for (int k = 0; k < kUpd; ++k) {
        const int i = i0 + k * NT;
        if (i < I) {
          sk[k] = s_g[i];
          rk[k] = r_g[i];
        }
      }
#pragma unroll
      for (int k = 0; k < kUpd; ++k) {
        const int i = i0 + k * NT;
        if (i < I) {
          s_g[i] = sk[k] + alT * P[i];
          rk[k] -= alT * Q[i];
          r_g[i] = rk[k];
          rn += (double)rk[k] * (double)rk[k];
        }
      }
    }
    rn = block_sum1<NT / kWave>(rn, red, 1);
    if constexpr (PC && sizeof(T) == 4) {
      float* tab = reinterpret_cast<float*>(smem + a.pc_off);
      rz = pc_apply(reinterpret_cast<float*>(P), reinterpret_cast<float*>(Q), reinterpret_cast<float*>(F), tab,
                    tab + 2 * (ns + 1), ns, reinterpret_cast<const float*>(r_g), mi.pc_c, (float)a.lamv[kl], rz, 0,
                    red);
    } else {
      const T beta = (T)(rn / rr);
      if (I <= kUpd * NT) {
#pragma unroll
        for (int k = 0; k < kUpd; ++k) {
          const int i = tid + k * NT;
          if (i < I) P[i] = rk[k] + beta * P[i];
        }
      } else {
        for (int i0 = tid; i0 < I; i0 += kUpd * NT) {
#pragma unroll
          for (int k = 0; k < kUpd; ++k) {
            const int i = i0 + k * NT;
            if (i < I) rk[k] = r_g[i];
          }
#pragma unroll
          for (int k = 0; k < kUpd; ++k) {
            const int i = i0 + k * NT;
            if (i < I) P[i] = rk[k] + beta * P[i];
          }
        }
      }
    }
    rr = rn;
    __syncthreads();
  }
  if (st == SL_ST_MAXIT && rr <= stop2) st = SL_ST_OK;
  // ---- chi^2 and ||H s||^2 from the explicit solution
  __syncthreads();
  for (int i = tid; i < I; i += NT) P[i] = s_g[i];
  for (int e = tid; e < h * pitch; e += NT) Frows[e] = (T)0;
  __syncthreads();
  for (int t = tid; t < M; t += NT) {
    const int rc = pix[t];
    if (rc >= 0)
      F0[(rc >> 16) * pitch + (rc & 0xFFFF) + fo] =
          pixel_gather(P, ns, n2, t, cellp, fxp, fyp, DIR && a.interp == SL_INTERP_BICUBIC) * inv_n2;
  }
  double regacc = 0.0;
  for (int i = tid; i < I; i += NT) regacc += reg_node(P, ns, i / ns, i % ns, a.reg);
  __syncthreads();
  double cacc = 0.0;
  for (int e = tid; e < Dh * Dw; e += NT) {
    const int rr_ = Dr0 + e / Dw, cc_ = Dc0 + e % Dw;
    T z = 0;
    for (int aa = 0; aa < K; ++aa) {
      const int yr = rr_ - aa + ck - r0;
      if (yr < 0 || yr >= h) continue;
      for (int bb = 0; bb < K; ++bb) {
        const int yc = cc_ - bb + ck - c0;
        if (yc < 0 || yc >= w) continue;
        z += taps[ti.psf + aa * K + bb] * F0[yr * pitch + yc];
      }
    }
    const double zd = (double)z;
    cacc += zd * zd - 2.0 * zd * a.d[rr_ * nx + cc_];
  }
  block_sum2(cacc, regacc, red);
  if (tid == 0) {
    a.chi2[out_idx] = (a.consts->sum_d2 + cacc) / (a.sigma * a.sigma);
    a.regv[out_idx] = regacc;
    a.iters[out_idx] = it;
    a.status[out_idx] = st;
  }
  __syncthreads();
}

// Next (member, lambda) item for this block, -1 when every queue is empty;
// thread 0 pops, the value is broadcast through LDS and made scalar.
template <bool PC>
__device__ __forceinline__ int fetch_item(const SolveArgs& a, int xcd, int* sh_item) {
  int* head = PC ? a.consts->pqhead : a.consts->qhead;
  const int* count = PC ? a.consts->pqcount : a.consts->qcount;
  const int* queues = PC ? a.pqueues : a.queues;
  if (threadIdx.x == 0) {
    int item = -1;
    for (int x = 0; x < 8 && item < 0; ++x) {
      const int q = (xcd + x) & 7;
      const int idx = atomicAdd(&head[q], 1);
      if (idx < count[q]) item = queues[q * a.qcap + idx];
    }
    *sh_item = item;
  }
  __syncthreads();
  const int item = __builtin_amdgcn_readfirstlane(*sh_item);
  __syncthreads();
  return item;
}

// Persistent CG kernel: each block pulls (member, lambda) items from its XCD's
// queue (then the others').  PC = true takes the preconditioned items that
// k_split selected (FP32 only); PC = false all the others.
template <typename T, int CKT, bool PC, bool DIR>
__global__ void __launch_bounds__(kNTof<T>) k_solve(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh_item;
  if (__builtin_amdgcn_readfirstlane(a.consts->sep) == (int)DIR) return;   // the other form's launch does the work
  const int xcd = blockIdx.x & 7;
  for (int item = fetch_item<PC>(a, xcd, &sh_item); item >= 0; item = fetch_item<PC>(a, xcd, &sh_item)) {
    const int m = item / a.n_lambda, kl = item % a.n_lambda;   // scalar
    const MemberInfo mi = a.minfo[m];                          // uniform address: scalar loads
    if constexpr (PC) {
      run_item<T, CKT, true, true, DIR>(a, mi, m, kl, smem);
    } else {
      const int status = __builtin_amdgcn_readfirstlane(mi.status);
      const int fits = __builtin_amdgcn_readfirstlane(mi.lds_frame);
      if (status != SL_ST_OK)
        trivial_item<T>(a, mi, m, kl);
      else if (fits)
        run_item<T, CKT, true, false, DIR>(a, mi, m, kl, smem);
      else
        run_item<T, CKT, false, false, DIR>(a, mi, m, kl, smem);
    }
  }
}

// ------------------------------------------------------------------ k_mcdof
// Next member of the Monte Carlo pass for this block (thread 0 takes it, the
// value is broadcast through LDS and made scalar), as fetch_item does.
__device__ __forceinline__ int fetch_counter(int* counter, int* sh_m) {
  if (threadIdx.x == 0) *sh_m = atomicAdd(counter, 1);
  __syncthreads();
  const int m = __builtin_amdgcn_readfirstlane(*sh_m);
  __syncthreads();
  return m;
}

// Monte Carlo degrees of freedom of one member at its corner lambda (Sec. 2.5).
// FP64: plain CG on the data system, and in lockstep the system with
// right-hand side A^T bhat advanced with the data system's alpha_k and beta_k
// (not its own); p of the data system stays in LDS (P), and the second
// system's direction is swapped into P for its operator application.  FP32:
// the second system by its own CG (see below).  Then gamma = <A^T bhat, xhat>
// = bhat^T A xhat and dof = bhat^T bhat - gamma.  Per-block scratch (global):
// r, xhat, rhat, phat and the saved p.
template <typename T, int CKT, bool LDSF, bool DIR>
__device__ __forceinline__ void run_mc_item(const SolveArgs& a, const MemberInfo& mi, int m, int kl,
                                            unsigned char* smem) {
  constexpr int NT = kNTof<T>;
  const int tid = threadIdx.x;
  const long slot = (long)blockIdx.x;
  T* __restrict__ r_g = reinterpret_cast<T*>(a.mcbuf) + slot * 5L * a.I_max;
  T* __restrict__ xh_g = r_g + a.I_max;
  T* __restrict__ rh_g = xh_g + a.I_max;
  T* __restrict__ ph_g = rh_g + a.I_max;
  T* __restrict__ pd_g = ph_g + a.I_max;
  const int ns = mi.ns, I = mi.I, M = mi.M, r0 = mi.r0, c0 = mi.c0;
  const int h = mi.r1 - mi.r0 + 1, w = mi.c1 - mi.c0 + 1;
  constexpr int HALO = 2 * CKT;
  const int pitch = (w + 2 * HALO) | 1;
  const int frame_elems = (h + 2 * HALO + kSegR) * pitch;
  const int J = a.nx * a.ny, n2 = a.n2, nx = a.nx, ny = a.ny, K = a.K, ck = a.ck;
  T* P = reinterpret_cast<T*>(smem);
  T* Q = reinterpret_cast<T*>(smem + a.q_off);
  double* red = reinterpret_cast<double*>(smem + a.red_off);
  T* F = LDSF ? reinterpret_cast<T*>(smem + a.frame_off) : reinterpret_cast<T*>(a.gframe) + slot * a.gframe_elems;
  T* const F0 = F + HALO * pitch + HALO;
  const int Dr0 = max(mi.r0 - ck, 0), Dr1 = min(mi.r1 + ck, ny - 1);
  const int Dc0 = max(mi.c0 - ck, 0), Dc1 = min(mi.c1 + ck, nx - 1);
  const OpView<T> ov{a.pix_list + (long)m * a.slot_cap, a.cell + (long)m * a.slot_cap * n2,
                     reinterpret_cast<const T*>(a.fx) + (long)m * a.slot_cap * n2,
                     reinterpret_cast<const T*>(a.fy) + (long)m * a.slot_cap * n2, F, F0,
                     reinterpret_cast<T*>(a.gz) + slot * 2L * J, reinterpret_cast<T*>(a.gz) + slot * 2L * J + J,
                     reinterpret_cast<const T*>(a.taps_t), a.lt_ptr + (long)m * (a.I_max + 65),
                     reinterpret_cast<const LtEntry<T>*>(a.lt_ent) + (long)m * a.lt_cap, a.lt_perm + (long)m * a.I_max,
                     ns, I, M, r0, c0, h, w, pitch, -r0 * pitch - c0, n2, nx, ny, K, ck,
                     __builtin_amdgcn_readfirstlane(mi.sell), Dr0, Dc0, Dr1 - Dr0 + 1, Dc1 - Dc0 + 1,
                     a.consts->sep != 0, a.reg == SL_H_IDENTITY, (T)1 / (T)n2, (T)a.lamv[kl],
                     a.interp == SL_INTERP_BICUBIC};
  for (int e = tid; e < frame_elems; e += NT) F[e] = (T)0;
  const double* bm = a.b + (long)m * a.I_max;
  const double* bhm = a.bh + (long)m * a.I_max;
  if constexpr (sizeof(T) == 4) {
    // FP32: the lockstep recurrence is linear in the second system with fixed
    // coefficients, so FP32 rounding injected at one step grows with the data
    // polynomial's later factors; here the second system is solved by its own
    // CG instead (same operator, same stopping rule relative to ||A^T bhat||),
    // which estimates the same Tikhonov gamma (Eq. 19) once converged.
    double rr = 0.0;
    for (int i = tid; i < I; i += NT) {
      const T nv = (T)bhm[i];
      P[i] = nv;
      rh_g[i] = nv;
      xh_g[i] = (T)0;
      rr += (double)nv * (double)nv;
    }
    rr = block_sum1<NT / kWave>(rr, red, 0);
    const double stop2 = a.tol * a.tol * rr;
    for (int it = 0; it < a.maxit; ++it) {
      if (__builtin_amdgcn_readfirstlane((int)(rr <= stop2))) break;
      double pq = apply_normal<T, CKT, NT, DIR>(ov, P, Q);
      pq = block_sum1<NT / kWave>(pq, red, 0);
      clear_rows<T, CKT, NT, DIR>(ov);
      if (__builtin_amdgcn_readfirstlane((int)!(pq > 0.0))) break;
      const T alT = (T)(rr / pq);
      double rn = 0.0;
      for (int i = tid; i < I; i += NT) {
        xh_g[i] += alT * P[i];
        const T rk = rh_g[i] - alT * Q[i];
        rh_g[i] = rk;
        rn += (double)rk * (double)rk;
      }
      rn = block_sum1<NT / kWave>(rn, red, 1);
      const T beta = (T)(rn / rr);
      for (int i = tid; i < I; i += NT) P[i] = rh_g[i] + beta * P[i];
      rr = rn;
      __syncthreads();
    }
  } else {
  double rr = 0.0;
  for (int i = tid; i < I; i += NT) {
    const T bv = (T)bm[i], nv = (T)bhm[i];
    P[i] = bv;
    r_g[i] = bv;
    rr += (double)bv * (double)bv;
    xh_g[i] = (T)0;
    rh_g[i] = nv;
    ph_g[i] = nv;
  }
  rr = block_sum1<NT / kWave>(rr, red, 0);
  const double stop2 = a.tol * a.tol * rr;
  for (int it = 0; it < a.maxit; ++it) {
    if (__builtin_amdgcn_readfirstlane((int)(rr <= stop2))) break;
    // data system: q = A p, alpha, r update, beta, new p (saved to global)
    double pq = apply_normal<T, CKT, NT, DIR>(ov, P, Q);
    pq = block_sum1<NT / kWave>(pq, red, 0);
    clear_rows<T, CKT, NT, DIR>(ov);
    if (__builtin_amdgcn_readfirstlane((int)!(pq > 0.0))) break;
    const T alT = (T)(rr / pq);
    double rn = 0.0;
    for (int i = tid; i < I; i += NT) {
      const T rk = r_g[i] - alT * Q[i];
      r_g[i] = rk;
      rn += (double)rk * (double)rk;
    }
    rn = block_sum1<NT / kWave>(rn, red, 1);
    const T beta = (T)(rn / rr);
    for (int i = tid; i < I; i += NT) {
      pd_g[i] = r_g[i] + beta * P[i];
      P[i] = ph_g[i];
    }
    __syncthreads();
    // second system with the same alpha and beta
    double pqh = apply_normal<T, CKT, NT, DIR>(ov, P, Q);
    pqh = block_sum1<NT / kWave>(pqh, red, 0);   // its barrier: every gather has read P and the frame
    (void)pqh;
    clear_rows<T, CKT, NT, DIR>(ov);
    for (int i = tid; i < I; i += NT) {
      const T ph = P[i];
      xh_g[i] += alT * ph;
      const T rk = rh_g[i] - alT * Q[i];
      rh_g[i] = rk;
      ph_g[i] = rk + beta * ph;
      P[i] = pd_g[i];
    }
    rr = rn;
    __syncthreads();
  }
  }
  double g = 0.0;
  for (int i = tid; i < I; i += NT) g += bhm[i] * (double)xh_g[i];
  g = block_sum1<NT / kWave>(g, red, 1);
  // every thread stores the same value: no lane-predicated store in the member loop
  a.dofv[m] = a.consts->sum_n2 - g;
  __syncthreads();
}

// One member per item, in member order, at the member's L-curve corner; a
// member without a solve (invalid, or no pixel maps) gets NaN.  The member
// loop holds no lane-predicated code besides the fetch (the form k_solve
// uses): a store under `threadIdx.x == 0` followed by `continue` was compiled
// into an inner loop that thread 0's lane left to do the store while the
// other lanes went on re-reading an item index that only thread 0 advances.
template <typename T, int CKT, bool DIR>
__global__ void __launch_bounds__(kNTof<T>) k_mcdof(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh_m;
  if (__builtin_amdgcn_readfirstlane(a.consts->sep) == (int)DIR) return;   // the other form's launch does the work
  for (int m = fetch_counter(&a.consts->mchead, &sh_m); m < a.n_members;
       m = fetch_counter(&a.consts->mchead, &sh_m)) {
    const MemberInfo mi = a.minfo[m];
    const int status = __builtin_amdgcn_readfirstlane(mi.status);
    if (status != SL_ST_OK) {
      a.dofv[m] = NAN;   // the same value from every thread
    } else {
      const int kl = __builtin_amdgcn_readfirstlane(a.k_star[m]);
      if (__builtin_amdgcn_readfirstlane(mi.lds_frame))
        run_mc_item<T, CKT, true, DIR>(a, mi, m, kl, smem);
      else
        run_mc_item<T, CKT, false, DIR>(a, mi, m, kl, smem);
    }
  }
}

// ------------------------------------------------------------------ k_implicit
// Implicit regularisation by the iteration count (Sec. 2.4, Sec. 2.6): CGLS
// on min ||A s - d|| (A = B L) from s = 0 with no lambda, for exactly
// n_lambda iterations.  Each iteration applies A once (L gather, then B over
// the dilated bounding box) and A^T once (B^T at the mapped pixels, then the
// L^T gather), as CGLS does: q = A p, alpha = ||g||^2 / ||q||^2,
// s += alpha p, e -= alpha q, g = A^T e, beta = ||g'||^2 / ||g||^2,
// p = g + beta p, with the image residual e = d - A s carried on the dilated
// box (pixels outside it keep e = d; A^T e reads only the box).  After
// iteration k the iterate goes to solution slot k of the member, with
// chi^2 = ||e||^2 / sigma^2 and the zeroth-order measure ||s_k||^2 (Sec. 2.6).
// g_0 = A^T d is the member's fixed-order right-hand side.  After a
// breakdown (A p = 0) the remaining slots repeat the last iterate.
//
// Monte Carlo degrees of freedom (Sec. 2.5; FP64 only, mcn not NULL): a
// second system with data bhat advanced with the data system's alpha_k and
// beta_k, not its own (xhat += alpha phat, ehat -= alpha A phat,
// phat = A^T ehat + beta phat, from xhat = 0, ehat = bhat, phat = A^T bhat),
// so that xhat_k is the data system's k-step filter applied to bhat; after
// every iteration bhat^T (bhat - A xhat_k) = ||bhat||^2 - <A^T bhat, xhat_k>
// goes to dofk, and k_corner takes the value at the corner.  Its vectors
// live in the block's global scratch: xhat, phat and A^T ehat in mcbuf, ehat
// on the dilated box in the second half of gz.
template <typename T, int CKT, bool LDSF>
__device__ __forceinline__ void run_implicit_item(const SolveArgs& a, const MemberInfo& mi, int m,
                                                  unsigned char* smem) {
  constexpr int NT = kNTof<T>;
  const int tid = threadIdx.x;
  const long slot = (long)blockIdx.x;
  const int K_it = a.n_lambda;
  const int ns = mi.ns, I = mi.I, M = mi.M, r0 = mi.r0, c0 = mi.c0;
  const int h = mi.r1 - mi.r0 + 1, w = mi.c1 - mi.c0 + 1;
  constexpr int HALO = 2 * CKT;
  const int pitch = (w + 2 * HALO) | 1;
  const int frame_elems = (h + 2 * HALO + kSegR) * pitch;
  const int J = a.nx * a.ny, n2 = a.n2, nx = a.nx, ny = a.ny, K = a.K, ck = a.ck;
  T* P = reinterpret_cast<T*>(smem);                      // search direction p
  T* G = reinterpret_cast<T*>(smem + a.q_off);            // gradient g = A^T e
  double* red = reinterpret_cast<double*>(smem + a.red_off);
  T* F = LDSF ? reinterpret_cast<T*>(smem + a.frame_off) : reinterpret_cast<T*>(a.gframe) + slot * a.gframe_elems;
  T* const F0 = F + HALO * pitch + HALO;
  const int Dr0 = max(mi.r0 - ck, 0), Dr1 = min(mi.r1 + ck, ny - 1);
  const int Dc0 = max(mi.c0 - ck, 0), Dc1 = min(mi.c1 + ck, nx - 1);
  const int Dh = Dr1 - Dr0 + 1, Dw = Dc1 - Dc0 + 1;
  T* __restrict__ Zq = reinterpret_cast<T*>(a.gz) + slot * 2L * J;   // q = A p on the dilated box, then W
  T* __restrict__ E = reinterpret_cast<T*>(a.ibuf) + slot * J;        // e on the dilated box
  const bool mc = sizeof(T) == 8 && a.mcn != nullptr;               // uniform: a kernel argument
  T* __restrict__ xh = reinterpret_cast<T*>(a.mcbuf) + slot * 5L * a.I_max;
  T* __restrict__ ph = xh + a.I_max;
  T* __restrict__ gh = ph + a.I_max;
  T* __restrict__ Eh = reinterpret_cast<T*>(a.gz) + ((long)gridDim.x + slot) * 2L * J;   // ehat on the dilated box
  const double* bhm = a.bh + (long)m * a.I_max;
  const OpView<T> ov{a.pix_list + (long)m * a.slot_cap, a.cell + (long)m * a.slot_cap * n2,
                     reinterpret_cast<const T*>(a.fx) + (long)m * a.slot_cap * n2,
                     reinterpret_cast<const T*>(a.fy) + (long)m * a.slot_cap * n2, F, F0, Zq, Zq + J,
                     reinterpret_cast<const T*>(a.taps_t), a.lt_ptr + (long)m * (a.I_max + 65),
                     reinterpret_cast<const LtEntry<T>*>(a.lt_ent) + (long)m * a.lt_cap, a.lt_perm + (long)m * a.I_max,
                     ns, I, M, r0, c0, h, w, pitch, -r0 * pitch - c0, n2, nx, ny, K, ck,
                     __builtin_amdgcn_readfirstlane(mi.sell), Dr0, Dc0, Dh, Dw,
                     a.consts->sep != 0, true, (T)1 / (T)n2, (T)0, a.interp == SL_INTERP_BICUBIC};
  // Frame: zero outside the mapped pixels whenever L p is gathered into it
  // (the adjoint blur's other writes are cleared after each L^T gather).
  for (int e = tid; e < frame_elems; e += NT) F[e] = (T)0;
  const double* bm = a.b + (long)m * a.I_max;
  double gg = 0.0, din = 0.0;
  for (int i = tid; i < I; i += NT) {
    const T bv = (T)bm[i];
    P[i] = bv;
    gg += (double)bv * (double)bv;
  }
  for (int e = tid; e < Dh * Dw; e += NT) {
    const double dv = a.d[(Dr0 + e / Dw) * nx + Dc0 + e % Dw];
    E[e] = (T)dv;
    din += dv * dv;
  }
  if (mc) {
    for (int i = tid; i < I; i += NT) {
      xh[i] = (T)0;
      ph[i] = (T)bhm[i];
    }
    for (int e = tid; e < Dh * Dw; e += NT) Eh[e] = (T)a.mcn[(Dr0 + e / Dw) * nx + Dc0 + e % Dw];
  }
  block_sum2(gg, din, red + 32);
  const double d_out = a.consts->sum_d2 - din;   // sum of d^2 outside the dilated box
  const double inv_s2 = 1.0 / (a.sigma * a.sigma);
  int k = 0, st = SL_ST_OK;
  double chi2_last = a.consts->sum_d2 * inv_s2, reg_last = 0.0, dof_last = a.consts->sum_n2;
  for (; k < K_it; ++k) {
    if (__builtin_amdgcn_readfirstlane((int)(gg <= 0.0))) break;
    gather_L<T, NT>(ov, P);                               // frame = L p
    __syncthreads();
    double qq = forward_blur<T, CKT, NT>(ov, Zq);         // q = B L p
    qq = block_sum1<NT / kWave>(qq, red, 0);
    if (__builtin_amdgcn_readfirstlane((int)!(qq > 0.0))) {
      st = SL_ST_BREAKDOWN;
      break;
    }
    const T alT = (T)(gg / qq);
    const T* s_prev = reinterpret_cast<const T*>(a.s_all) + ((long)m * K_it + (k > 0 ? k - 1 : 0)) * a.I_max;
    T* s_k = reinterpret_cast<T*>(a.s_all) + ((long)m * K_it + k) * a.I_max;
    double reg = 0.0, ee = 0.0;
    for (int i = tid; i < I; i += NT) {
      const T sv = (k ? s_prev[i] : (T)0) + alT * P[i];
      s_k[i] = sv;
      reg += (double)sv * (double)sv;
    }
    for (int e = tid; e < Dh * Dw; e += NT) {
      const T ev = E[e] - alT * Zq[e];
      E[e] = ev;
      ee += (double)ev * (double)ev;
    }
    block_sum2(reg, ee, red + 32);                        // also orders the E writes before B^T reads them
    chi2_last = (d_out + ee) * inv_s2;
    reg_last = reg;
    {   // every thread stores the same block-reduced values: no lane-predicated code in the loop
      const long o = (long)m * K_it + k;
      a.chi2[o] = chi2_last;
      a.regv[o] = reg_last;
      a.iters[o] = k + 1;
      a.status[o] = SL_ST_OK;
    }
    adjoint_blur<T, CKT, NT>(ov, E);                      // frame = B^T e at the mapped pixels
    double gn = gather_LT<T, NT, true>(ov, P, G);         // g = L^T B^T e
    gn = block_sum1<NT / kWave>(gn, red, 1);
    clear_rows<T, CKT, NT, true>(ov);                           // every gather has read the frame
    const T beta = (T)(gn / gg);
    for (int i = tid; i < I; i += NT) P[i] = G[i] + beta * P[i];
    gg = gn;
    if (mc) {   // the second system with this iteration's alpha and beta
      __syncthreads();                                    // the frame is clear again
      gather_L<T, NT>(ov, ph);
      __syncthreads();
      forward_blur<T, CKT, NT>(ov, Zq);                   // A phat
      __syncthreads();
      double gam = 0.0;
      for (int i = tid; i < I; i += NT) {
        const T xv = xh[i] + alT * ph[i];
        xh[i] = xv;
        gam += bhm[i] * (double)xv;
      }
      for (int e = tid; e < Dh * Dw; e += NT) Eh[e] -= alT * Zq[e];
      gam = block_sum1<NT / kWave>(gam, red, 0);          // its barrier: ehat complete
      adjoint_blur<T, CKT, NT>(ov, Eh);
      gather_LT<T, NT, true>(ov, ph, gh);                 // A^T ehat
      __syncthreads();
      clear_rows<T, CKT, NT, true>(ov);
      for (int i = tid; i < I; i += NT) ph[i] = gh[i] + beta * ph[i];
      dof_last = a.consts->sum_n2 - gam;
      a.dofk[(long)m * K_it + k] = dof_last;              // the same value from every thread
    }
    __syncthreads();
  }
  // slots past an early stop repeat the last iterate (s = 0 when there is none)
  for (int kk = k; kk < K_it; ++kk) {
    const T* s_prev = reinterpret_cast<const T*>(a.s_all) + ((long)m * K_it + (kk > 0 ? kk - 1 : 0)) * a.I_max;
    T* s_k = reinterpret_cast<T*>(a.s_all) + ((long)m * K_it + kk) * a.I_max;
    for (int i = tid; i < I; i += NT) s_k[i] = kk ? s_prev[i] : (T)0;
    const long o = (long)m * K_it + kk;
    a.chi2[o] = chi2_last;
    a.regv[o] = reg_last;
    a.iters[o] = k;
    a.status[o] = st;
    if (mc) a.dofk[o] = dof_last;
    __syncthreads();
  }
}

// One member per item; members without a solve get the trivial result.
template <typename T, int CKT>
__global__ void __launch_bounds__(kNTof<T>) k_implicit(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh_m;
  for (int m = fetch_counter(&a.consts->imhead, &sh_m); m < a.n_members; m = fetch_counter(&a.consts->imhead, &sh_m)) {
    const MemberInfo mi = a.minfo[m];
    const int status = __builtin_amdgcn_readfirstlane(mi.status);
    if (status != SL_ST_OK) {   // same values from every thread, as trivial_item writes them
      const double c2 = status == SL_ST_INVALID ? NAN : a.consts->sum_d2 / (a.sigma * a.sigma);
      for (int k = 0; k < a.n_lambda; ++k) {
        T* s_dst = reinterpret_cast<T*>(a.s_all) + ((long)m * a.n_lambda + k) * a.I_max;
        for (int i = threadIdx.x; i < mi.I; i += kNTof<T>) s_dst[i] = (T)0;
        const long o = (long)m * a.n_lambda + k;
        a.chi2[o] = c2;
        a.regv[o] = status == SL_ST_INVALID ? NAN : 0.0;
        a.iters[o] = 0;
        a.status[o] = status;
      }
    } else if (__builtin_amdgcn_readfirstlane(mi.lds_frame)) {
      run_implicit_item<T, CKT, true>(a, mi, m, smem);
    } else {
      run_implicit_item<T, CKT, false>(a, mi, m, smem);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ k_chi2_src
// Image chi^2 of candidate sources for one lens: the fitness of the
// source-refinement search (Sec. 3.2), where every source node is a free
// parameter and the lens is held fixed.  chi2[p] = ||B L s_p - d||^2 / sigma^2
// over all J pixels (Eq. 4; pixels outside the dilated bounding box of the
// mapped pixels keep their data).  k_setup and k_prep have built member 0's
// trace table.  Persistent over the candidates: block b takes p = b, b +
// gridDim.x, ...; the source is staged in LDS (in the bulk type), L gathers
// it into the frame, B runs over the dilated box into Z, and the residual
// sum is FP64.  The frame holds values at the mapped pixels only, each of
// which every gather overwrites, so it is zeroed once.
template <typename T, int CKT>
__global__ void __launch_bounds__(kNTof<T>) k_chi2_src(SolveArgs a, const double* src, int n_src, double* chi2) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NT = kNTof<T>;
  const int tid = threadIdx.x;
  const MemberInfo mi = a.minfo[0];
  const int status = __builtin_amdgcn_readfirstlane(mi.status);
  const double inv_s2 = 1.0 / (a.sigma * a.sigma);
  if (status != SL_ST_OK) {   // no mapped pixel (chi^2 of s = 0) or invalid lens (NaN)
    const double c2 = status == SL_ST_INVALID ? NAN : a.consts->sum_d2 * inv_s2;
    for (int p = blockIdx.x; p < n_src; p += gridDim.x) chi2[p] = c2;   // the same value from every thread
    return;
  }
  const int ns = mi.ns, I = mi.I, M = mi.M, r0 = mi.r0, c0 = mi.c0;
  const int h = mi.r1 - mi.r0 + 1, w = mi.c1 - mi.c0 + 1;
  constexpr int HALO = 2 * CKT;
  const int pitch = (w + 2 * HALO) | 1;
  const int frame_elems = (h + 2 * HALO + kSegR) * pitch;
  const int J = a.nx * a.ny, n2 = a.n2, nx = a.nx, ny = a.ny, K = a.K, ck = a.ck;
  const long slot = (long)blockIdx.x;
  T* S = reinterpret_cast<T*>(smem);
  double* red = reinterpret_cast<double*>(smem + a.red_off);
  T* F = __builtin_amdgcn_readfirstlane(mi.lds_frame) ? reinterpret_cast<T*>(smem + a.frame_off)
                                                       : reinterpret_cast<T*>(a.gframe) + slot * a.gframe_elems;
  T* const F0 = F + HALO * pitch + HALO;
  const int Dr0 = max(mi.r0 - ck, 0), Dr1 = min(mi.r1 + ck, ny - 1);
  const int Dc0 = max(mi.c0 - ck, 0), Dc1 = min(mi.c1 + ck, nx - 1);
  const int Dh = Dr1 - Dr0 + 1, Dw = Dc1 - Dc0 + 1;
  T* __restrict__ Z = reinterpret_cast<T*>(a.gz) + slot * 2L * J;
  const OpView<T> ov{a.pix_list, a.cell, reinterpret_cast<const T*>(a.fx), reinterpret_cast<const T*>(a.fy), F, F0,
                     Z, Z + J, reinterpret_cast<const T*>(a.taps_t), a.lt_ptr,
                     reinterpret_cast<const LtEntry<T>*>(a.lt_ent), a.lt_perm, ns, I, M, r0, c0, h, w, pitch,
                     -r0 * pitch - c0, n2, nx, ny, K, ck, __builtin_amdgcn_readfirstlane(mi.sell), Dr0, Dc0, Dh, Dw,
                     a.consts->sep != 0, true, (T)1 / (T)n2, (T)0, a.interp == SL_INTERP_BICUBIC};
  for (int e = tid; e < frame_elems; e += NT) F[e] = (T)0;
  double din = 0.0;
  for (int e = tid; e < Dh * Dw; e += NT) {
    const double dv = a.d[(Dr0 + e / Dw) * nx + Dc0 + e % Dw];
    din += dv * dv;
  }
  din = block_sum1<NT / kWave>(din, red, 0);
  const double d_out = a.consts->sum_d2 - din;   // data outside the dilated box
  for (int p = blockIdx.x; p < n_src; p += gridDim.x) {
    const double* sp = src + (long)p * I;
    for (int i = tid; i < I; i += NT) S[i] = (T)sp[i];
    __syncthreads();
    gather_L<T, NT>(ov, S);                      // frame = L s_p at the mapped pixels
    __syncthreads();
    forward_blur<T, CKT, NT>(ov, Z);             // Z = B L s_p over the dilated box
    __syncthreads();
    double acc = 0.0;
    for (int e = tid; e < Dh * Dw; e += NT) {
      const double r = (double)Z[e] - a.d[(Dr0 + e / Dw) * nx + Dc0 + e % Dw];
      acc += r * r;
    }
    acc = block_sum1<NT / kWave>(acc, red, 1);   // its barrier: every read of S, the frame and Z is done
    chi2[p] = (acc + d_out) * inv_s2;            // the same value from every thread
    __syncthreads();
  }
}

// The candidate-source chi^2 kernel of the bulk type and window (the windows
// the solve kernels are compiled for).
using Chi2Kernel = void (*)(SolveArgs, const double*, int, double*);
template <typename T>
static Chi2Kernel pick_chi2_kernel(int ckt) {
  if (sizeof(T) == 4) {
    switch (ckt) {
      case 2: return k_chi2_src<float, 2>;
      case 4: return k_chi2_src<float, 4>;
      case 7: return k_chi2_src<float, 7>;
      case 10: return k_chi2_src<float, 10>;
      case 16: return k_chi2_src<float, 16>;
    }
  } else {
    switch (ckt) {
      case 2: return k_chi2_src<double, 2>;
      case 7: return k_chi2_src<double, 7>;
      case 10: return k_chi2_src<double, 10>;
    }
  }
  return nullptr;
}

// Moves the items that take the spectral preconditioner into their own queues
// (stable, per XCD queue): valid member, FP32, curvature H, frame in LDS with
// room for the n x n scratch, and lambda >= pc_theta c.  One block.
template <typename T>
__global__ void __launch_bounds__(64) k_split(SolveArgs a) {
  const int q = threadIdx.x;
  if (q < 8) {
    const int n = a.consts->qcount[q];
    int keep = 0, moved = 0;
    for (int k = 0; k < n; ++k) {   // in place: keep <= k, so no unread item is overwritten
      const int item = a.queues[q * a.qcap + k];
      const MemberInfo mi = a.minfo[item / a.n_lambda];
      const double lam = a.lamv[item % a.n_lambda];
      const bool fits = mi.lds_frame != 0;
      const bool pc = sizeof(T) == 4 && a.reg == SL_H_CURVATURE && !a.plain_cg && mi.status == SL_ST_OK && fits &&
                      mi.ns * mi.ns <= a.lds_frame_cap && lam >= (double)a.pc_theta * mi.pc_c;
      // Both stores unconditionally, then bump one count: the store not
      // taken lands at or past its queue's final count, where nothing reads.
      // (The if/else form selected the base pointer per lane, and hipcc put
      // the preconditioned base on lanes that only failed the lambda test.)
      a.pqueues[q * a.qcap + moved] = item;
      a.queues[q * a.qcap + keep] = item;
      moved += pc ? 1 : 0;
      keep += pc ? 0 : 1;
    }
    a.consts->qcount[q] = keep;
    a.consts->pqcount[q] = moved;
    a.consts->pqhead[q] = 0;
  }
}

// ------------------------------------------------------------------ k_corner
template <typename T>
__global__ void __launch_bounds__(256) k_corner(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* scratch = reinterpret_cast<double*>(smem);
  __shared__ int sh_k;
  const int m = blockIdx.x;
  const int nl = a.n_lambda;
  const MemberInfo mi = a.minfo[m];
  // the corner by the whole block (the condition is the same for every thread)
  const int kk = (mi.status == SL_ST_OK && nl >= 4)
                     ? lcurve_corner_block(a.regv + (long)m * nl, a.chi2 + (long)m * nl, nl, scratch)
                     : -1;
  if (threadIdx.x == 0) {
    int k = 0, cst = mi.status;
    if (mi.status == SL_ST_OK) {
      if (nl >= 4) {
        if (kk >= 0)
          k = kk;
        else
          cst = SL_ST_LCURVE;
      } else if (nl > 1) {
        cst = SL_ST_LCURVE;
      }
    }
    // a curve through an unconverged point is flagged (its corner is still computed)
    if (cst == SL_ST_OK)
      for (int j = 0; j < nl; ++j) {
        const int sj = a.status[(long)m * nl + j];
        if (sj == SL_ST_MAXIT || sj == SL_ST_BREAKDOWN) {
          cst = sj;
          break;
        }
      }
    a.k_star[m] = k;
    a.corner_status[m] = cst;
    if (a.implicit && a.dofv) a.dofv[m] = mi.status == SL_ST_OK ? a.dofk[(long)m * nl + k] : NAN;
    sh_k = k;
  }
  __syncthreads();
  const T* src = reinterpret_cast<const T*>(a.s_all) + ((long)m * nl + sh_k) * a.I_max;
  for (int i = threadIdx.x; i < mi.I; i += blockDim.x) a.s_corner[mi.off + i] = (double)src[i];
}

// ------------------------------------------------------------------ host side
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// k_setup's dynamic LDS: the tap table and the PSF of the largest PSF size
// (65.5 + 31.8 KB at 63 x 63)
static const size_t kSetupLds = sizeof(double) * ((size_t)TapIdx(SL_MAX_PSF).total + SL_MAX_PSF * SL_MAX_PSF);

template <typename T>
static int setup_lds_attr() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    err = hipFuncSetAttribute((const void*)k_setup<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSetupLds);
  });
  SL_HIP(err);
  return SL_OK;
}

// Bytes after the solve's workspace that sl_chi2_sources uses: the device
// copy of ns, then the member offsets k_setup writes.
constexpr size_t kSrcTail = 512;

// *p = v, from a launch argument (so that the write can be captured).
__global__ void k_put_int(int32_t* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

static Layout make_layout(const sl_problem* pb, int max_ns, int M, int NL, int n_wg) {
  Layout L{};
  const size_t sz = pb->dtype == SL_F64 ? 8 : 4;
  L.J = pb->img.nx * pb->img.ny;
  L.n2 = pb->img.nsub * pb->img.nsub;
  L.I_max = max_ns * max_ns;
  L.n_wg = n_wg;
  L.qcap = ((M + 7) / 8) * NL;
  const TapIdx ti(pb->k);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.consts = take(sizeof(Consts));
  L.lam = take(sizeof(double) * SL_MAX_LAMBDA);
  L.taps_d = take(sizeof(double) * ti.total);
  L.taps_f = take(sz * ti.total);
  L.minfo = take(sizeof(MemberInfo) * M);
  L.queues = take(sizeof(int) * 8 * (size_t)L.qcap);
  L.pqueues = take(sizeof(int) * 8 * (size_t)L.qcap);
  L.slot_cap = L.J + 64;
  L.pix = take(sizeof(int32_t) * (size_t)M * L.slot_cap);
  L.cell = take(sizeof(int32_t) * (size_t)M * L.slot_cap * L.n2);
  L.fx = take(sz * (size_t)M * L.slot_cap * L.n2);
  L.fy = take(sz * (size_t)M * L.slot_cap * L.n2);
  L.b = take(sizeof(double) * (size_t)M * L.I_max);
  L.bh = take(sizeof(double) * (size_t)M * L.I_max);   // A^T bhat (Monte Carlo degrees of freedom)
  L.dofk = take(sizeof(double) * (size_t)M * NL);      // per-iterate estimate of the implicit solve
  L.ltc = take(sizeof(int) * (size_t)M * L.I_max * kFillW);   // per-wave fill cursors (k_prep)
  L.s_all = take(sz * (size_t)M * NL * L.I_max);
  L.gframe_elems = (pb->img.ny + 4 * 16 + kSegR) * ((pb->img.nx + 4 * 16) | 1);   // widest window's halo
  L.gframe = take(sz * (size_t)n_wg * L.gframe_elems);
  L.gz = take(sz * 4 * (size_t)n_wg * L.J);          // [plain | preconditioned launch][slot]: z, B^T z
  L.rbuf = take(sz * 2 * (size_t)n_wg * L.I_max);
  L.mcbuf = take(sz * 5 * (size_t)n_wg * L.I_max);
  L.ibuf = take(sz * (size_t)n_wg * L.J);   // image residual of the implicit-regularisation solve
  L.lt_ptr = take(sizeof(int32_t) * (size_t)M * (L.I_max + 65));
  L.lt_perm = take(sizeof(int32_t) * (size_t)M * L.I_max);
  // twice the unpadded bound (4 or, bicubic, 16 nodes per subpixel): room for slice padding
  L.lt_cap = (pb->interp == SL_INTERP_BICUBIC ? 32LL : 8LL) * L.n2 * L.slot_cap;
  L.lt_ent = take((sz == 8 ? 16 : 8) * (size_t)M * (size_t)L.lt_cap);
  L.total = off;
  return L;
}

static int check_problem(const sl_problem* pb, int max_ns, int M, int NL) {
  SL_REQUIRE(pb != nullptr, "problem is NULL");
  const sl_image_grid& g = pb->img;
  SL_REQUIRE(g.nx >= 1 && g.ny >= 1 && g.nx <= 256 && g.ny <= 256,
             "batched solve supports images up to 256 x 256 (got %d x %d)", g.nx, g.ny);
  SL_REQUIRE(std::isfinite(g.pix) && g.pix > 0.0, "pixel size must be positive");
  SL_REQUIRE(g.nsub >= 1 && g.nsub <= SL_MAX_NSUB, "nsub %d outside [1, %d]", g.nsub, SL_MAX_NSUB);
  SL_REQUIRE(pb->k >= 1 && pb->k <= SL_MAX_PSF && (pb->k & 1), "PSF side %d must be odd, <= %d", pb->k,
             SL_MAX_PSF);
  SL_REQUIRE(std::isfinite(pb->sigma) && pb->sigma > 0.0, "sigma must be positive");
  SL_REQUIRE(std::isfinite(pb->half_width) && pb->half_width > 0.0, "half_width must be positive");
  SL_REQUIRE(pb->reg == SL_H_IDENTITY || pb->reg == SL_H_CURVATURE, "unknown reg %d", pb->reg);
  SL_REQUIRE(pb->dtype == SL_F32 || pb->dtype == SL_F64, "unknown dtype %d", pb->dtype);
  SL_REQUIRE(pb->psf_general == 0 || pb->psf_general == 1, "psf_general must be 0 or 1");
  SL_REQUIRE(pb->interp == SL_INTERP_BILINEAR || pb->interp == SL_INTERP_NEAREST || pb->interp == SL_INTERP_BICUBIC,
             "unknown interp %d", pb->interp);
  SL_REQUIRE(max_ns >= 2 && max_ns <= 128, "max_ns %d outside [2, 128]", max_ns);
  SL_REQUIRE(M >= 1 && M <= (1 << 20), "n_members %d out of range", M);
  SL_REQUIRE(NL >= 1 && NL <= SL_MAX_LAMBDA, "n_lambda %d outside [1, %d]", NL, SL_MAX_LAMBDA);
  SL_REQUIRE((long)M * NL < (1L << 30), "too many (member, lambda) items");
  return SL_OK;
}

using SolveKernel = void (*)(SolveArgs);

// Kernel variants: bulk type T and banded half-width CKT (>= ck of the PSF).
// Compiled banded-window sizes (CKT >= ck).  `wide` takes the next size up;
// nullptr when that variant does not exist.
// pc selects the preconditioned kernel of the same window size.
template <bool DIR>
static SolveKernel pick_kernel_f(int ck, bool wide, int* ckt, bool pc = false) {
  static const int sizes[] = {2, 4, 7, 10, 16};
  static const SolveKernel ks[] = {k_solve<float, 2, false, DIR>, k_solve<float, 4, false, DIR>,
                                   k_solve<float, 7, false, DIR>, k_solve<float, 10, false, DIR>,
                                   k_solve<float, 16, false, DIR>};
  static const SolveKernel kp[] = {k_solve<float, 2, true, DIR>, k_solve<float, 4, true, DIR>,
                                   k_solve<float, 7, true, DIR>, k_solve<float, 10, true, DIR>,
                                   k_solve<float, 16, true, DIR>};
  const SolveKernel* k = pc ? kp : ks;
  int i = 0;
  while (i < 5 && sizes[i] < ck) ++i;
  if (i == 5) {   // wider PSFs: direct path only
    *ckt = 2;
    return wide ? nullptr : k[0];
  }
  if (wide && ++i == 5) return nullptr;
  *ckt = sizes[i];
  return k[i];
}

// The Monte Carlo degrees-of-freedom kernel of the same bulk type and window as the solve.
template <typename T, bool DIR>
static SolveKernel pick_mc_kernel(int ckt) {
  if (sizeof(T) == 4) {
    switch (ckt) {
      case 2: return k_mcdof<float, 2, DIR>;
      case 4: return k_mcdof<float, 4, DIR>;
      case 7: return k_mcdof<float, 7, DIR>;
      case 10: return k_mcdof<float, 10, DIR>;
      case 16: return k_mcdof<float, 16, DIR>;
    }
  } else {
    switch (ckt) {
      case 2: return k_mcdof<double, 2, DIR>;
      case 7: return k_mcdof<double, 7, DIR>;
      case 10: return k_mcdof<double, 10, DIR>;
    }
  }
  return nullptr;
}

// The implicit-regularisation kernel of the same bulk type and window as the solve.
template <typename T>
static SolveKernel pick_implicit_kernel(int ckt) {
  if (sizeof(T) == 4) {
    switch (ckt) {
      case 2: return k_implicit<float, 2>;
      case 4: return k_implicit<float, 4>;
      case 7: return k_implicit<float, 7>;
      case 10: return k_implicit<float, 10>;
      case 16: return k_implicit<float, 16>;
    }
  } else {
    switch (ckt) {
      case 2: return k_implicit<double, 2>;
      case 7: return k_implicit<double, 7>;
      case 10: return k_implicit<double, 10>;
    }
  }
  return nullptr;
}

template <bool DIR>
static SolveKernel pick_kernel_d(int ck, bool wide, int* ckt) {
  static const int sizes[] = {2, 7, 10};
  static const SolveKernel ks[] = {k_solve<double, 2, false, DIR>, k_solve<double, 7, false, DIR>,
                                   k_solve<double, 10, false, DIR>};
  int i = 0;
  while (i < 3 && sizes[i] < ck) ++i;
  if (i == 3) {
    *ckt = 2;
    return wide ? nullptr : ks[0];
  }
  if (wide && ++i == 3) return nullptr;
  *ckt = sizes[i];
  return ks[i];
}

// ------------------------------------------------------------------ profiling
struct ProfileState {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
static ProfileState g_prof;

// Per-device side stream for the preconditioned launch and the events that
// fork it from, and join it to, the caller's stream; created on first use
// (default priority, non-blocking).
// Two side streams: the banded and the direct form of the preconditioned
// launch go on separate streams, so that the form that returns at entry
// never holds the other back while its blocks wait for CUs.
struct SideStream {
  hipStream_t s = nullptr, s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, join2 = nullptr;
};
static std::mutex g_side_mu;
static SideStream g_side[64];

static int side_stream(SideStream** out) {
  int dev = 0;
  SL_HIP(hipGetDevice(&dev));
  SL_REQUIRE(dev >= 0 && dev < 64, "device index %d out of range", dev);
  SideStream& x = g_side[dev];
  if (!x.s) {
    SL_HIP(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
    SL_HIP(hipStreamCreateWithFlags(&x.s2, hipStreamNonBlocking));
    SL_HIP(hipEventCreateWithFlags(&x.fork, hipEventDisableTiming));
    SL_HIP(hipEventCreateWithFlags(&x.join, hipEventDisableTiming));
    SL_HIP(hipEventCreateWithFlags(&x.join2, hipEventDisableTiming));
  }
  *out = &x;
  return SL_OK;
}

// Each solve kernel comes as a pair: the banded-blur form and the direct
// form (suffix d); both are launched and the one that does not match the
// problem returns at entry.
struct LaunchCfg {
  SolveKernel kim = nullptr;   // implicit-regularisation solve (replaces k_split / k_solve)
  SolveKernel ks = nullptr, ksd = nullptr;
  SolveKernel kpc = nullptr, kpcd = nullptr;   // preconditioned kernels, when some items may take them
  SolveKernel kmc = nullptr, kmcd = nullptr;   // Monte Carlo degrees-of-freedom pass, when requested
  size_t lds = 0, prep_lds = 0, corner_lds = 0;
};

// Chooses the CG kernel of variant v and its LDS budget and sets the
// kernels' LDS attributes (host-side, outside any stream capture).
template <typename T>
static int configure(SolveArgs& A, const Layout& L, const sl_tuning& v, LaunchCfg* c) {
  const size_t sz = sizeof(T);
  int ckt = 2;
  SolveKernel ks = sizeof(T) == 4 ? pick_kernel_f<false>(A.ck, v.wide_window != 0, &ckt)
                                  : pick_kernel_d<false>(A.ck, v.wide_window != 0, &ckt);
  int ckt_d = 2;
  SolveKernel ksd = sizeof(T) == 4 ? pick_kernel_f<true>(A.ck, v.wide_window != 0, &ckt_d)
                                   : pick_kernel_d<true>(A.ck, v.wide_window != 0, &ckt_d);
  if (!ks) {
    set_error("kernel variant does not exist for this PSF size and dtype");
    return SL_ENOIMPL;
  }
  A.ckt = ckt;
  A.force_csr = v.lt_csr != 0;
  A.force_direct = v.blur_direct != 0 || A.psf_general != 0 || A.interp == SL_INTERP_BICUBIC;
  A.plain_cg = v.plain_cg != 0;
  A.pc_theta = (v.pc_theta_pct > 0 ? v.pc_theta_pct : kPcThetaPct) * 0.01f;
  A.heavy = v.heavy > 0 ? v.heavy : kHeavy;
  // dynamic LDS: source vector | reduction scratch | frame (up to the full image)
  A.q_off = (int)align256(sz * L.I_max);
  A.red_off = A.q_off + (int)align256(sz * L.I_max);
  A.pc_off = A.red_off + 64 * (int)sizeof(double);
  // sine table 2 (max_ns + 1) and eigenvalues max_ns of the spectral preconditioner
  A.frame_off = A.pc_off + (int)align256(sizeof(float) * (3 * A.max_ns + 8));
  const size_t fixed = (size_t)A.frame_off;
  size_t lds = fixed + sz * (size_t)(A.ny + 4 * ckt + kSegR) * (size_t)((A.nx + 4 * ckt) | 1);
  const size_t lds_max = 160 * 1024 - 1024;
  if (lds > lds_max) lds = lds_max;
  SL_REQUIRE(lds > fixed + 64 * sz, "source grid too large for LDS");
  A.lds_frame_cap = (int)((lds - fixed) / sz);
  c->ks = ks;
  c->ksd = ksd;
  if (sizeof(T) == 4 && A.reg == SL_H_CURVATURE && !A.plain_cg && !A.implicit) {
    int ckt2 = 0;
    c->kpc = pick_kernel_f<false>(A.ck, v.wide_window != 0, &ckt2, true);
    c->kpcd = pick_kernel_f<true>(A.ck, v.wide_window != 0, &ckt2, true);
  }
  c->lds = lds;
  if (A.implicit) {
    c->kim = pick_implicit_kernel<T>(ckt);
    c->kpc = c->kpcd = nullptr;
    if (!c->kim) {
      set_error("no implicit-regularisation kernel for window %d", ckt);
      return SL_ENOIMPL;
    }
  }
  if (A.mcn && !A.implicit) {   // the implicit solve runs its own lockstep system
    c->kmc = pick_mc_kernel<T, false>(ckt);
    c->kmcd = pick_mc_kernel<T, true>(ckt);
    if (!c->kmc || !c->kmcd) {
      set_error("no Monte Carlo degrees-of-freedom kernel for window %d", ckt);
      return SL_ENOIMPL;
    }
  }
  // FP64 right-hand-side accumulator, reused by the transposed-operator build (2 I + 192 ints),
  // then one conflict tag per node when that fits in LDS
  c->prep_lds = std::max(sizeof(double) * L.I_max, sizeof(int) * (2 * L.I_max + 192));
  const size_t tagged = 8 * (size_t)L.I_max + 768 + sizeof(int) * (size_t)L.I_max;
  A.prep_tags = tagged <= 159 * 1024;
  if (A.prep_tags) c->prep_lds = tagged;
  // lcurve_corner_block: 12 n + 2 n^2 doubles (both spline systems at once)
  c->corner_lds = sizeof(double) * (2 * A.n_lambda * A.n_lambda + 12 * A.n_lambda + 16);
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  for (SolveKernel k : {c->ks, c->ksd, c->kpc, c->kpcd, c->kmc, c->kmcd})
    if (k) SL_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (c->kim)
    SL_HIP(hipFuncSetAttribute((const void*)c->kim, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  SL_HIP(hipFuncSetAttribute((const void*)k_prep<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)c->prep_lds));
  // up to 72 KB at SL_MAX_LAMBDA points
  SL_HIP(hipFuncSetAttribute((const void*)k_corner<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)c->corner_lds));
  return SL_OK;
}

// Launches the banded and the direct form of a persistent kernel on st, the
// banded one first; the one that does not match the problem (the separability
// flag k_setup leaves in the workspace) returns at entry.
// With force_direct the device's separability flag is 0 and the banded form
// would return at entry, so only the direct form is launched.
template <typename T>
static int launch_pair(SolveKernel kb, SolveKernel kd, const Layout& L, const LaunchCfg& c, hipStream_t st,
                       const SolveArgs& A, const char* what) {
  if (!A.force_direct) {
    hipLaunchKernelGGL(kb, dim3(L.n_wg), dim3(kNTof<T>), c.lds, st, A);
    if (int e = check_launch(what)) return e;
  }
  hipLaunchKernelGGL(kd, dim3(L.n_wg), dim3(kNTof<T>), c.lds, st, A);
  return check_launch(what);
}

// Enqueues the launches of one solve on st: k_setup, k_prep, [k_split], the
// plain k_solve [beside the preconditioned k_solve on the side stream, joined
// back to st], k_corner.  `profile` records HIP events on st around the CG
// phase when profiling is on (never inside a capture).
// `priv` (nullable): a side stream and events owned by the caller (a graph
// capture uses its own, so that no other thread's eager solve can fork onto
// a stream that is part of the capture); NULL takes the per-device one under
// its lock.
template <typename T>
static int enqueue(const SolveArgs& A, const LamList& lams, const Layout& L, const LaunchCfg& c, hipStream_t st,
                   bool profile, SideStream* priv = nullptr) {
  if (int e = setup_lds_attr<T>()) return e;
  hipLaunchKernelGGL(k_setup<T>, dim3(1), dim3(1024), kSetupLds, st, A, lams);
  if (int e = check_launch("k_setup")) return e;
  hipLaunchKernelGGL(k_prep<T>, dim3(A.n_members), dim3(1024), c.prep_lds, st, A);
  if (int e = check_launch("k_prep")) return e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (profile) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    if (g_prof.on) {
      SL_HIP(hipEventCreate(&e0));
      SL_HIP(hipEventCreate(&e1));
      SL_HIP(hipEventRecord(e0, st));
    }
  }
  if (c.kim) {
    hipLaunchKernelGGL(c.kim, dim3(L.n_wg), dim3(kNTof<T>), c.lds, st, A);
    if (int e = check_launch("k_implicit")) return e;
  } else if (c.kpc) {
    hipLaunchKernelGGL(k_split<T>, dim3(1), dim3(64), 0, st, A);
    if (int e = check_launch("k_split")) return e;
    // The plain launch first on st, the preconditioned one on the side
    // stream: both are persistent, so its blocks take the CUs that the plain
    // launch's last long items leave idle.  They share no queue and no
    // per-block scratch.
    std::unique_lock<std::mutex> g(g_side_mu, std::defer_lock);
    SideStream* ss = priv;
    if (!ss) {
      g.lock();
      if (int e = side_stream(&ss)) return e;
    }
    SL_HIP(hipEventRecord(ss->fork, st));
    if (int e = launch_pair<T>(c.ks, c.ksd, L, c, st, A, "k_solve")) return e;
    SL_HIP(hipStreamWaitEvent(ss->s, ss->fork, 0));
    SL_HIP(hipStreamWaitEvent(ss->s2, ss->fork, 0));
    if (!A.force_direct) {
      hipLaunchKernelGGL(c.kpc, dim3(L.n_wg), dim3(kNTof<T>), c.lds, ss->s, A);
      if (int e = check_launch("k_solve (preconditioned)")) return e;
    }
    hipLaunchKernelGGL(c.kpcd, dim3(L.n_wg), dim3(kNTof<T>), c.lds, ss->s2, A);
    if (int e = check_launch("k_solve (preconditioned, direct blur)")) return e;
    SL_HIP(hipEventRecord(ss->join, ss->s));
    SL_HIP(hipEventRecord(ss->join2, ss->s2));
    SL_HIP(hipStreamWaitEvent(st, ss->join, 0));
    SL_HIP(hipStreamWaitEvent(st, ss->join2, 0));
  } else {
    if (int e = launch_pair<T>(c.ks, c.ksd, L, c, st, A, "k_solve")) return e;
  }
  if (e1) {
    SL_HIP(hipEventRecord(e1, st));
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.ev.emplace_back(e0, e1);
  }
  hipLaunchKernelGGL(k_corner<T>, dim3(A.n_members), dim3(256), c.corner_lds, st, A);
  if (int e = check_launch("k_corner")) return e;
  if (c.kmc) return launch_pair<T>(c.kmc, c.kmcd, L, c, st, A, "k_mcdof");
  return SL_OK;
}

static int configure_any(int dtype, SolveArgs& A, const Layout& L, const sl_tuning& v, LaunchCfg* c) {
  return dtype == SL_F32 ? configure<float>(A, L, v, c) : configure<double>(A, L, v, c);
}

static int enqueue_any(int dtype, const SolveArgs& A, const LamList& lams, const Layout& L, const LaunchCfg& c,
                       hipStream_t st, bool profile, SideStream* priv = nullptr) {
  return dtype == SL_F32 ? enqueue<float>(A, lams, L, c, st, profile, priv)
                         : enqueue<double>(A, lams, L, c, st, profile, priv);
}

// ------------------------------------------------------------------ autotuner table
using TuneKey = std::array<int, 9>;

static TuneKey tune_key(const sl_problem* pb, int max_ns, int n_members, int n_lambda) {
  return {pb->dtype, pb->img.nx, pb->img.ny, pb->img.nsub, pb->k, pb->reg, max_ns, n_members, n_lambda};
}

struct TuneTable {
  std::mutex mu;
  std::map<TuneKey, sl_tuning> best;
};
static TuneTable g_tune;

static sl_tuning resolve_tuning(const sl_problem* pb, int max_ns, int n_members, int n_lambda,
                                const sl_solve_opts* opt) {
  if (opt->tuning) return *opt->tuning;
  std::lock_guard<std::mutex> g(g_tune.mu);
  auto it = g_tune.best.find(tune_key(pb, max_ns, n_members, n_lambda));
  return it == g_tune.best.end() ? sl_tuning{0, 0, 0, 0, 0, 0} : it->second;
}

// The autotuner's search, in three stages.  Variants 0..7: the structural
// switches (window, L^T layout, blur form) at the default threshold and
// queue order.  8..11: the preconditioner threshold theta (percent of c) on
// the best of 0..7.  12..15: the count of smallest lambdas queued first on
// the best of 0..11.
static const int kThetaPct[4] = {5, 10, 25, 40};
static const int kHeavyN[4] = {2, 3, 6, 8};
static sl_tuning variant_of(int i, const sl_tuning& base) {
  if (i < 8) return sl_tuning{i & 1, (i >> 1) & 1, (i >> 2) & 1, 0, 0, 0};
  sl_tuning v = base;
  if (i < 12)
    v.pc_theta_pct = kThetaPct[i - 8];
  else
    v.heavy = kHeavyN[i - 12];
  return v;
}

// Validates the arguments of a solve and fills the kernel arguments.
static int prepare(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns, int n_members,
                   const double* lambdas, int n_lambda, const sl_solve_opts* opt, void* workspace,
                   size_t workspace_bytes, const sl_result* out, SolveArgs* Ap, Layout* Lp, LamList* lams) {
  if (int e = check_problem(pb, max_ns, n_members, n_lambda)) return e;
  SL_REQUIRE(lens && ns && pb->d && pb->psf, "NULL device input");
  SL_REQUIRE(lambdas != nullptr, "lambdas is NULL");
  for (int k = 0; k < n_lambda; ++k) {
    SL_REQUIRE(std::isfinite(lambdas[k]) && lambdas[k] > 0.0, "lambda[%d] must be positive", k);
    SL_REQUIRE(k == 0 || lambdas[k] > lambdas[k - 1], "lambdas must be strictly ascending");
  }
  SL_REQUIRE(opt != nullptr, "opts is NULL");
  SL_REQUIRE(std::isfinite(opt->tol) && opt->tol >= 0.0, "tol must be >= 0");
  SL_REQUIRE(opt->maxit >= 1, "maxit must be >= 1");
  SL_REQUIRE(out && out->s_corner && out->s_off && out->chi2 && out->reg && out->iters && out->status &&
                 out->k_star && out->corner_status,
             "NULL result pointer");
  SL_REQUIRE(!opt->mc_noise || out->dof, "mc_noise given but the result has no dof array");
  SL_REQUIRE(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
             "workspace must be non-NULL and 256-byte aligned");
  const Layout L = make_layout(pb, max_ns, n_members, n_lambda, device_cus());
  SL_REQUIRE(workspace_bytes >= L.total, "workspace too small: %zu < %zu bytes", workspace_bytes, L.total);
  SolveArgs A{};
  A.nx = pb->img.nx;
  A.ny = pb->img.ny;
  A.nsub = pb->img.nsub;
  A.n2 = L.n2;
  A.K = pb->k;
  A.ck = (pb->k - 1) / 2;
  A.reg = pb->reg;
  A.psf_general = pb->psf_general != 0;
  A.interp = pb->interp;
  A.n_members = n_members;
  A.n_lambda = n_lambda;
  A.max_ns = max_ns;
  A.maxit = opt->maxit;
  A.pix = pb->img.pix;
  A.R = pb->half_width;
  A.sigma = pb->sigma;
  A.tol = opt->tol;
  A.lens = lens;
  A.ns = ns;
  A.d = pb->d;
  A.psf = pb->psf;
  A.s_corner = out->s_corner;
  A.s_off = out->s_off;
  A.chi2 = out->chi2;
  A.regv = out->reg;
  A.iters = out->iters;
  A.status = out->status;
  A.k_star = out->k_star;
  A.corner_status = out->corner_status;
  unsigned char* ws = (unsigned char*)workspace;
  A.consts = (Consts*)(ws + L.consts);
  A.lamv = (double*)(ws + L.lam);
  A.taps_d = (double*)(ws + L.taps_d);
  A.taps_t = ws + L.taps_f;
  A.minfo = (MemberInfo*)(ws + L.minfo);
  A.queues = (int*)(ws + L.queues);
  A.pqueues = (int*)(ws + L.pqueues);
  A.qcap = L.qcap;
  A.pix_list = (int32_t*)(ws + L.pix);
  A.cell = (int32_t*)(ws + L.cell);
  A.fx = ws + L.fx;
  A.fy = ws + L.fy;
  A.b = (double*)(ws + L.b);
  A.bh = (double*)(ws + L.bh);
  A.dofk = (double*)(ws + L.dofk);
  A.ltc = (int*)(ws + L.ltc);
  A.mcbuf = ws + L.mcbuf;
  A.ibuf = ws + L.ibuf;
  A.mcn = opt->mc_noise;
  A.dofv = opt->mc_noise ? out->dof : nullptr;
  A.s_all = ws + L.s_all;
  A.gframe = ws + L.gframe;
  A.gframe_elems = L.gframe_elems;
  A.slot_cap = L.slot_cap;
  A.gz = ws + L.gz;
  A.rbuf = ws + L.rbuf;
  A.lt_ptr = (int32_t*)(ws + L.lt_ptr);
  A.lt_perm = (int32_t*)(ws + L.lt_perm);
  A.lt_ent = ws + L.lt_ent;
  A.lt_cap = L.lt_cap;
  A.I_max = L.I_max;
  *lams = LamList{};
  for (int k = 0; k < n_lambda; ++k) lams->v[k] = lambdas[k];
  *Ap = A;
  *Lp = L;
  return SL_OK;
}

}  // namespace sl

using namespace sl;

extern "C" {

int sl_solve_semilinear(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns,
                        int n_members, const double* lambdas, int n_lambda, const sl_solve_opts* opt,
                        void* workspace, size_t workspace_bytes, sl_result* out, void* stream) {
  SolveArgs A;
  Layout L;
  LamList lams;
  if (int e = prepare(pb, lens, ns, max_ns, n_members, lambdas, n_lambda, opt, workspace, workspace_bytes, out, &A,
                      &L, &lams))
    return e;
  LaunchCfg c;
  if (int e = configure_any(pb->dtype, A, L, resolve_tuning(pb, max_ns, n_members, n_lambda, opt), &c)) return e;
  return enqueue_any(pb->dtype, A, lams, L, c, (hipStream_t)stream, true);
}

int sl_solve_implicit(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns, int n_members,
                      int n_iter, const sl_solve_opts* opt, void* workspace, size_t workspace_bytes, sl_result* out,
                      void* stream) {
  SL_REQUIRE(n_iter >= 4 && n_iter <= SL_MAX_LAMBDA, "n_iter %d outside [4, %d]", n_iter, SL_MAX_LAMBDA);
  SL_REQUIRE(opt != nullptr, "opts is NULL");
  SL_REQUIRE(opt->mc_noise == nullptr || pb->dtype == SL_F64,
             "mc_noise with the implicit-regularisation solve needs FP64: its lockstep system amplifies FP32 "
             "rounding of the step lengths past the first few iterations");
  double idx[SL_MAX_LAMBDA];   // placeholders for the argument checks: one slot per iterate
  for (int k = 0; k < n_iter; ++k) idx[k] = k + 1.0;
  SolveArgs A;
  Layout L;
  LamList lams;
  if (int e = prepare(pb, lens, ns, max_ns, n_members, idx, n_iter, opt, workspace, workspace_bytes, out, &A, &L,
                      &lams))
    return e;
  A.implicit = 1;
  LaunchCfg c;
  const sl_tuning dflt{0, 0, opt->tuning ? opt->tuning->blur_direct : 0, 1, 0, 0};
  if (int e = configure_any(pb->dtype, A, L, dflt, &c)) return e;
  return enqueue_any(pb->dtype, A, lams, L, c, (hipStream_t)stream, true);
}

size_t sl_chi2_sources_workspace_size(const sl_problem* pb, int ns) {
  const size_t n = sl_solve_workspace_size(pb, ns, 1, 1);
  return n ? align256(n) + kSrcTail : 0;
}

int sl_chi2_sources(const sl_problem* pb, const double* lens, int ns, const double* sources, int n_sources,
                    void* workspace, size_t workspace_bytes, double* chi2, void* stream) {
  SL_REQUIRE(pb != nullptr, "problem is NULL");
  SL_REQUIRE(ns >= 2 && ns <= 128, "ns %d outside [2, 128]", ns);
  SL_REQUIRE(n_sources >= 1 && n_sources <= (1 << 24), "n_sources %d out of range", n_sources);
  SL_REQUIRE(lens && sources && chi2, "NULL device pointer");
  const size_t base = sl_solve_workspace_size(pb, ns, 1, 1);
  SL_REQUIRE(base != 0, "%s", sl_last_error());
  SL_REQUIRE(workspace_bytes >= align256(base) + kSrcTail, "workspace too small: %zu < %zu bytes", workspace_bytes,
             align256(base) + kSrcTail);
  // the tail holds the device copy of ns and the member offsets k_setup writes
  unsigned char* tail = static_cast<unsigned char*>(workspace) + align256(base);
  int32_t* ns_dev = reinterpret_cast<int32_t*>(tail);
  sl_result dummy{};
  dummy.s_off = reinterpret_cast<int64_t*>(tail + 256);
  dummy.s_corner = reinterpret_cast<double*>(tail + 256);
  dummy.chi2 = dummy.reg = dummy.s_corner;
  dummy.iters = dummy.status = dummy.k_star = dummy.corner_status = ns_dev;
  const double lam1 = 1.0;
  const sl_solve_opts opt{0.0, 1, nullptr, nullptr};
  SolveArgs A;
  Layout L;
  LamList lams;
  if (int e = prepare(pb, lens, ns_dev, ns, 1, &lam1, 1, &opt, workspace, base, &dummy, &A, &L, &lams)) return e;
  LaunchCfg c;
  const sl_tuning dflt{0, 0, 0, 1, 0, 0};
  if (int e = configure_any(pb->dtype, A, L, dflt, &c)) return e;
  hipStream_t st = (hipStream_t)stream;
  const int nb = std::min(L.n_wg, n_sources);
  const int nt = pb->dtype == SL_F32 ? kNTof<float> : kNTof<double>;
  const Chi2Kernel kc = pb->dtype == SL_F32 ? pick_chi2_kernel<float>(A.ckt) : pick_chi2_kernel<double>(A.ckt);
  if (!kc) {
    set_error("no candidate-source chi^2 kernel for window %d", A.ckt);
    return SL_ENOIMPL;
  }
  {
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    SL_HIP(hipFuncSetAttribute((const void*)kc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds));
  }
  hipLaunchKernelGGL(k_put_int, dim3(1), dim3(64), 0, st, ns_dev, ns);
  if (int e = check_launch("k_put_int")) return e;
  if (pb->dtype == SL_F32) {
    if (int e = setup_lds_attr<float>()) return e;
    hipLaunchKernelGGL(k_setup<float>, dim3(1), dim3(1024), kSetupLds, st, A, lams);
    if (int e = check_launch("k_setup")) return e;
    hipLaunchKernelGGL(k_prep<float>, dim3(1), dim3(1024), c.prep_lds, st, A);
  } else {
    if (int e = setup_lds_attr<double>()) return e;
    hipLaunchKernelGGL(k_setup<double>, dim3(1), dim3(1024), kSetupLds, st, A, lams);
    if (int e = check_launch("k_setup")) return e;
    hipLaunchKernelGGL(k_prep<double>, dim3(1), dim3(1024), c.prep_lds, st, A);
  }
  if (int e = check_launch("k_prep")) return e;
  hipLaunchKernelGGL(kc, dim3(nb), dim3(nt), c.lds, st, A, sources, n_sources, chi2);
  return check_launch("k_chi2_src");
}

int sl_solve_autotune(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns, int n_members,
                      const double* lambdas, int n_lambda, const sl_solve_opts* opt, void* workspace,
                      size_t workspace_bytes, sl_result* out, void* stream, sl_tuning* best, double* ms) {
  SolveArgs A0;
  Layout L;
  LamList lams;
  if (int e = prepare(pb, lens, ns, max_ns, n_members, lambdas, n_lambda, opt, workspace, workspace_bytes, out,
                      &A0, &L, &lams))
    return e;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  SL_HIP(hipEventCreate(&e0));
  SL_HIP(hipEventCreate(&e1));
  double t_best = 1e300;
  int i_best = -1, i_last = -1;
  sl_tuning v_best{0, 0, 0, 0, 0, 0}, base{0, 0, 0, 0, 0, 0};
  // the threshold matters only where the preconditioner can run
  const bool pc_possible = pb->dtype == SL_F32 && pb->reg == SL_H_CURVATURE;
  // SL_AUTOTUNE_VERBOSE=1: one line per variant on stderr as it is timed
  const char* ve = std::getenv("SL_AUTOTUNE_VERBOSE");
  const bool verbose = ve && ve[0] == '1';
  int rc = SL_OK;
  for (int i = 0; i < SL_N_VARIANTS && rc == SL_OK; ++i) {
    if (ms) ms[i] = -1.0;
    if (i == 8 || i == 12) base = v_best;   // the next stage starts from the best so far
    if (i >= 8 && i < 12 && !pc_possible) continue;
    const sl_tuning vi = variant_of(i, base);
    SolveArgs A = A0;
    LaunchCfg c;
    const int ce = configure_any(pb->dtype, A, L, vi, &c);
    if (ce == SL_ENOIMPL) continue;
    if ((rc = ce) != SL_OK) break;
    if ((rc = enqueue_any(pb->dtype, A, lams, L, c, st, false)) != SL_OK) break;   // untimed
    float t = 1e30f;
    for (int rep = 0; rep < 2 && rc == SL_OK; ++rep) {   // the faster of two timed runs
      float tr = 0.0f;
      if (hipEventRecord(e0, st) != hipSuccess) { rc = SL_EHIP; break; }
      if ((rc = enqueue_any(pb->dtype, A, lams, L, c, st, false)) != SL_OK) break;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&tr, e0, e1) != hipSuccess) {
        set_error("autotune timing failed: %s", hipGetErrorString(hipGetLastError()));
        rc = SL_EHIP;
        break;
      }
      t = std::min(t, tr);
    }
    if (rc != SL_OK) break;
    if (ms) ms[i] = t;
    if (verbose) {
      std::fprintf(stderr, "sl_solve_autotune: variant %d {%d %d %d theta %d%% heavy %d}: %.2f ms\n", i,
                   vi.wide_window, vi.lt_csr, vi.blur_direct, vi.pc_theta_pct ? vi.pc_theta_pct : kPcThetaPct,
                   vi.heavy ? vi.heavy : kHeavy, t);
      std::fflush(stderr);
    }
    i_last = i;
    if (t < t_best) {
      t_best = t;
      i_best = i;
      v_best = vi;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SL_OK) return rc;
  SL_REQUIRE(i_best >= 0, "no kernel variant exists for this problem");
  const sl_tuning v = v_best;
  {
    std::lock_guard<std::mutex> g(g_tune.mu);
    g_tune.best[tune_key(pb, max_ns, n_members, n_lambda)] = v;
  }
  if (best) *best = v;
  if (i_best != i_last) {   // leave the best variant's results in `out`
    SolveArgs A = A0;
    LaunchCfg c;
    if (int e = configure_any(pb->dtype, A, L, v, &c)) return e;
    if (int e = enqueue_any(pb->dtype, A, lams, L, c, st, false)) return e;
  }
  return SL_OK;
}

}  // extern "C"

struct sl_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

int sl_plan_create(const sl_problem* pb, const double* lens, const int32_t* ns, int max_ns, int n_members,
                   const double* lambdas, int n_lambda, const sl_solve_opts* opt, void* workspace,
                   size_t workspace_bytes, const sl_result* out, sl_plan** plan) {
  SL_REQUIRE(plan != nullptr, "plan is NULL");
  *plan = nullptr;
  SolveArgs A;
  Layout L;
  LamList lams;
  if (int e = prepare(pb, lens, ns, max_ns, n_members, lambdas, n_lambda, opt, workspace, workspace_bytes, out, &A,
                      &L, &lams))
    return e;
  LaunchCfg c;
  if (int e = configure_any(pb->dtype, A, L, resolve_tuning(pb, max_ns, n_members, n_lambda, opt), &c)) return e;
  // The capture forks onto a side stream of its own, created before the
  // capture starts (default priority) and destroyed once it has ended.
  SideStream own;
  if (c.kpc) {
    SL_HIP(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking));
    SL_HIP(hipStreamCreateWithFlags(&own.s2, hipStreamNonBlocking));
    SL_HIP(hipEventCreateWithFlags(&own.fork, hipEventDisableTiming));
    SL_HIP(hipEventCreateWithFlags(&own.join, hipEventDisableTiming));
    SL_HIP(hipEventCreateWithFlags(&own.join2, hipEventDisableTiming));
  }
  auto drop_own = [&]() {
    if (own.s) (void)hipStreamDestroy(own.s);
    if (own.s2) (void)hipStreamDestroy(own.s2);
    if (own.fork) (void)hipEventDestroy(own.fork);
    if (own.join) (void)hipEventDestroy(own.join);
    if (own.join2) (void)hipEventDestroy(own.join2);
  };
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    drop_own();
    set_error("hipStreamCreateWithFlags failed");
    return SL_EHIP;
  }
  hipGraph_t g = nullptr;
  int rc = SL_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("hipStreamBeginCapture failed: %s", hipGetErrorString(hipGetLastError()));
    rc = SL_EHIP;
  } else {
    rc = enqueue_any(pb->dtype, A, lams, L, c, cs, false, c.kpc ? &own : nullptr);
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    if (rc == SL_OK && ee != hipSuccess) {
      set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ee));
      rc = SL_EHIP;
    }
  }
  (void)hipStreamDestroy(cs);
  drop_own();
  hipGraphExec_t ge = nullptr;
  if (rc == SL_OK) {
    const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
      rc = SL_EHIP;
    }
  }
  if (rc != SL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  sl_plan* p = new sl_plan;
  p->graph = g;
  p->exec = ge;
  *plan = p;
  return SL_OK;
}

int sl_plan_launch(sl_plan* plan, void* stream) {
  SL_REQUIRE(plan && plan->exec, "invalid plan");
  SL_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
  return SL_OK;
}

int sl_plan_destroy(sl_plan* plan) {
  if (!plan) return SL_OK;
  hipError_t e1 = plan->exec ? hipGraphExecDestroy(plan->exec) : hipSuccess;
  hipError_t e2 = plan->graph ? hipGraphDestroy(plan->graph) : hipSuccess;
  delete plan;
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_error("graph destroy failed");
    return SL_EHIP;
  }
  return SL_OK;
}

size_t sl_solve_workspace_size(const sl_problem* pb, int max_ns, int n_members, int n_lambda) {
  if (check_problem(pb, max_ns, n_members, n_lambda) != SL_OK) return 0;
  return make_layout(pb, max_ns, n_members, n_lambda, device_cus()).total;
}


int sl_solve_member_info(const sl_problem* pb, int max_ns, int n_members, int n_lambda, const void* workspace,
                         int32_t* info_host) {
  if (int e = check_problem(pb, max_ns, n_members, n_lambda)) return e;
  SL_REQUIRE(workspace && info_host, "NULL pointer");
  const Layout L = make_layout(pb, max_ns, n_members, n_lambda, device_cus());
  std::vector<MemberInfo> mi(n_members);
  SL_HIP(hipDeviceSynchronize());
  SL_HIP(hipMemcpy(mi.data(), (const unsigned char*)workspace + L.minfo, sizeof(MemberInfo) * n_members,
                   hipMemcpyDeviceToHost));
  for (int m = 0; m < n_members; ++m) {
    int32_t* o = info_host + 10 * m;
    o[0] = mi[m].ns;
    o[1] = mi[m].I;
    o[2] = mi[m].Mtrue;
    o[3] = mi[m].r0;
    o[4] = mi[m].r1;
    o[5] = mi[m].c0;
    o[6] = mi[m].c1;
    o[7] = mi[m].status;
    o[8] = mi[m].status == SL_ST_OK ? mi[m].sell : -1;
    o[9] = mi[m].status == SL_ST_OK ? mi[m].lds_frame : -1;
  }
  return SL_OK;
}

int sl_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  for (auto& p : g_prof.ev) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  g_prof.ev.clear();
  g_prof.on = on != 0;
  return SL_OK;
}

int sl_profile_solve_ms(double* ms_total, int32_t* launches) {
  SL_REQUIRE(ms_total && launches, "NULL pointer");
  std::lock_guard<std::mutex> g(g_prof.mu);
  double tot = 0.0;
  for (auto& p : g_prof.ev) {
    SL_HIP(hipEventSynchronize(p.second));
    float ms = 0.f;
    SL_HIP(hipEventElapsedTime(&ms, p.first, p.second));
    tot += ms;
  }
  *ms_total = tot;
  *launches = (int32_t)g_prof.ev.size();
  return SL_OK;
}

}  // extern "C"
