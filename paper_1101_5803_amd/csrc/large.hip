// Large single-lens solve and the blur in Fourier space (gfx950).
//
// The paper's large-scale test (Sec. 4) fits one lens to a 640 x 640 image
// with a 512 x 512 source grid and a 65 x 65 PSF by 40 CGLS iterations, and
// the paper convolves with the PSF in Fourier space (Sec. 2.2).  One such
// problem fills the GPU by itself, so it runs as a short sequence of
// grid-wide kernels per CGLS iteration rather than as one persistent block
// per lens.  FP32 with a PSF of at most 65 x 65 (the large shape) blurs by
// overlap-save tiles, each transformed whole in one block's LDS:
//
//   k_gather   y = L p                            one thread per pixel
//   k_tile<B>  q = B y on each tile's owned 32 x 64 pixels, |q|^2
//                                                 one block per 96 x 128 tile
//   k_tile<BT> e -= alpha q (owned pixels, recomputed on the halo), |e|^2,
//              w = B^T e                          one block per tile
//   k_lt       L^T as a gather over a node-major table, with |g|^2
//                                                 8 lanes per node; nodes with
//                                                 many entries one wave each
//   k_update   s += alpha p, p = g + beta p, |s|^2, the iterate kept
//                                                 one thread per node
//
// FP64, or a wider PSF, blurs on a padded frame in three passes per blur:
//
//   k_rowfwd   row FFTs of L p (the gather fused)  one block per pair of rows
//   k_col      column FFT, product with the PSF spectrum, inverse column FFT
//                                                 one block per frequency column
//   k_rowinv   inverse row FFTs of q = B L p, cut to the image, |q|^2, and
//              forward again: q's row spectra     one block per pair of rows
//   k_col      the residual update e -= alpha q on the row spectra, |e|^2 by
//              Parseval, and the columns of B^T e
//   k_rowinv   inverse row FFTs: w = B^T e
//   k_lt, k_update as above (16 lanes per node)
//
// On the frame the residual e = d - A s lives only as row spectra: it starts as those of
// d, and q enters them cut to the image (the frame's columns from nx on are
// zero), so e stays the spectrum of an image row padded with zeros.
//
// Images are real, so two rows go through one complex FFT (row r as the real
// part, row r + 1 as the imaginary part) and only the columns kx = 0..Nx/2
// of the spectrum are kept.  The frame is Ny x Nx, powers of two with
// Ny >= ny + ck and Nx >= nx + ck: the circular convolution on that frame
// then equals the zero-padded one on the image.  The 1/(Nx Ny) of the inverse
// transform is folded into the PSF spectrum, which is computed once per call
// by a separable discrete Fourier transform of the K x K PSF in FP64.
//
// Reductions are FP64: each block writes its partial sum, and every
// consumer adds the partials in block order, so each run gives the same
// bits.  L^T sums each node's terms in ascending pixel order (the table is
// sorted once per call); with bilinear or nearest-neighbour L and at most
// 2 x 2 subpixels a pixel's terms for one node are merged into one entry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.h"
#include "semilin.h"

namespace sl {
namespace large {

constexpr int kNT = 256;              // threads of most blocks
constexpr int kRowNT = 512;           // threads of the row-FFT blocks
constexpr int kLtNT = 1024;           // threads of the L^T blocks
constexpr int kNodeNT = 1024;         // threads of the start and update blocks (each sums every |g|^2 partial)
// L^T lanes per node and node groups per thread in flight.  FP32: 8 lanes
// (most nodes have fewer entries than that), 4 groups.  FP64: 16 lanes, one
// group (its 16-byte entries: more groups cost the second block per compute
// unit and measured slower).
template <typename T>
constexpr int lt_lanes() { return sizeof(T) == 4 ? 8 : 16; }
template <typename T>
constexpr int lt_groups() { return sizeof(T) == 4 ? 4 : 1; }
// FP32: a node with more entries than this (the few nodes near the critical
// curves, up to ~300 entries) is summed by a wave of its own in extra blocks
// of the L^T launch instead of by lt_lanes lanes, which would make it the
// launch's longest chain of loads
template <typename T>
constexpr int lt_heavy() { return sizeof(T) == 4 ? 64 : 0x7fffffff; }
constexpr int kLtHeavyBlocks = 64;
constexpr int kSortChunk = 1024;      // keys of one node staged in LDS by the sort
constexpr int kMaxParts = 1024;       // blocks of the node kernels (grid-stride loops)
constexpr int kMaxImage = 2048;       // image side
constexpr int kMaxFrame = 4096;       // FFT frame side
constexpr int kMaxNs = 1024;          // source grid side
constexpr int kMaxPsf = 129;          // PSF side

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

// One subpixel of the trace table: its cell (-1 off the grid) and fractions,
// read together by one load.
template <typename T>
struct alignas(sizeof(T) == 8 ? 8 : 4) Sub {
  int32_t cell;
  T fx, fy;
};
static_assert(sizeof(Sub<float>) == 12, "three words per record: the vector loads of gather_L");

// One entry of the node-major L^T table: pixel and weight.
template <typename T>
struct alignas(8) LtE {
  int32_t pix;
  T w;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {   // a conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

static inline int frame_side(int n, int ck) {
  int f = 4;
  while (f < n + ck) f *= 2;
  return f;
}

// Everything one call works on.  T is the arithmetic of the bulk work.
template <typename T>
struct Args {
  int nx, ny, nsub, n2, ns, I, J, K, ck, interp, taps;
  int Nx, Ny, Nh;
  double pix, R, sigma;
  const double* lens;   // device [7]
  const double* d;      // device [ny * nx]
  const double* psf;    // device [K * K]
  cpx<T>* twx;          // [Nx] exp(-2 pi i m / Nx)
  cpx<T>* twy;          // [Ny]
  cpx<double>* twdx;    // the same in FP64 (PSF transform)
  cpx<double>* twdy;
  cpx<T>* H;            // [Nh][Ny] PSF spectrum / (Nx Ny)
  cpx<T>* S;            // [Nh][Ny] spectrum of the image in flight (rows < ny used in the row passes)
  cpx<T>* E;            // [Nh][Ny] row spectra of the image residual e = d - A s (rows < ny)
  cpx<T>* SQ;           // [Nh][Ny] row spectra of q = A p (rows < ny)
  cpx<double>* T1;      // [K][Nh] first stage of the PSF transform
  Sub<T>* sub;          // [J n^2] cell and fractions of each subpixel
  int32_t* cnt;         // [I] entries per node
  int32_t* tsum;        // [tiles] entries per tile of 1024 nodes, then the tile's start
  int32_t* hsum;        // [tiles + 1] heavy nodes (more than lt_heavy entries) per tile, then the
                        // tile's start in heavy[]; hsum[tiles] = their count
  int32_t* heavy;       // [I] the heavy nodes in ascending order
  int32_t* rowptr;      // [I + 1]
  int32_t* cursor;      // [I]
  int32_t* key;         // [cap] (subpixel, tap) of each entry, in fill order
  T* wtmp;              // [cap]
  LtE<T>* lt;           // [cap] pixel and weight (with the 1/n^2 average), sorted within each node
  T* w;                 // [J] B^T e
  // tiled blur (FP32, PSF side <= 65): overlap-save on 128 x 128 tiles
  T* y;                 // [J] L p
  T* q;                 // [J] B L p
  T* e0;                // [J] image residual, two buffers used in turn
  T* e1;
  cpx<T>* Ht;           // [96][65] PSF spectrum on the tile / (128 96), [ky][kx]
  cpx<T>* twt;          // [128] exp(-2 pi i m / 128)
  cpx<T>* twc;          // [96] exp(-2 pi i m / 96)
  cpx<double>* T1t;     // [K][65] first stage of the tile's PSF transform
  int tiled, tiles_x, tiles_y, nb_qq, nb_ee;
  T* s;                 // [I]
  T* p;
  T* g;
  T* s_iter;            // [n_iter][I] every iterate
  double* part;         // [4][n_iter + 1][max_blocks]: qq, ee, gg, ss partials
  double* gg;           // [n_iter + 1]: |g|^2 before iteration k
  double* alpha;        // [n_iter]: step length of iteration k (0 when it did not move)
  int32_t* done;        // [n_iter + 1]: the iteration stopped before iteration k
  int32_t* upd;         // [n_iter]: iteration k updated s
  int32_t* flags;       // [2]: invalid genome; count of rows the sort leaves to whole waves
  int n_iter, max_blocks, nb_row, nb_node, nb_lt, nb_heavy;
};

enum { P_QQ = 0, P_EE = 1, P_GG = 2, P_SS = 3 };

template <typename T>
__device__ __forceinline__ double* part_of(const Args<T>& a, int which, int it) {
  return a.part + ((long)which * (a.n_iter + 1) + it) * a.max_blocks;
}

// Sum of n block partials, the same in every block of the same size: thread
// t adds p[t], p[t + blockDim], ... in order, then the block sum adds the
// threads' sums in a fixed order.  Every thread receives the total; all
// threads must call it (barriers).  The producers keep n at most kMaxParts.
__device__ __forceinline__ double block_total(const double* p, int n) {
  __shared__ double red[kLtNT / kWave];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
  return block_sum(v, red);
}

// Block FP64 sum written as partial `idx` (by default this block's) of
// reduction `which`, slot `it` (all threads call it: barriers).
template <typename T>
__device__ __forceinline__ void put_partial(const Args<T>& a, double v, int which, int it, int idx = -1) {
  __shared__ double red[kLtNT / kWave];
  v = block_sum(v, red);
  if (threadIdx.x == 0) part_of(a, which, it)[idx < 0 ? (int)blockIdx.x : idx] = v;
}

// Work item of block b among n: blocks b = x, x + 8, ... run on XCD x (the
// launch deals workgroups to the eight XCDs in turn), and each XCD takes a
// contiguous range of items, so that neighbouring tiles or node ranges share
// that XCD's L2 (a tile's halo is its neighbours' interior).  A bijection of
// [0, n); partial sums stay indexed by item, so the reductions add in the
// same order whatever block computes an item.
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int kXcd = 8;
  const int per = n / kXcd, rem = n % kXcd;
  const int x = b % kXcd, k = b / kXcd;
  return x * per + (x < rem ? x : rem) + k;
}

// ---------------------------------------------------------------- FFT in LDS
// Complex FFT of length N (a power of two >= 2) of the data in LDS buffer `a`
// (b: a second buffer of N elements); returns the buffer with the result.
// Stockham autosort form (Govindaraju et al. 2008): stages of span Ns = 1,
// R, R R', ...; butterfly j of a stage reads a[j + r N/R] (r < R), turns
// input r by w^(r (j mod Ns) N/(Ns R)) and writes its radix-R DFT to
// b[(j - j mod Ns) R + j mod Ns + r Ns].  Radix 4 while 4 divides N/Ns, then
// one radix-2 stage.  INV: conjugate twiddles and DFT (no 1/N).  All threads
// of the block take part; one barrier per stage.
template <typename T, bool INV>
__device__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, int N, const cpx<T>* __restrict__ tw) {
  for (int Ns = 1; Ns < N;) {
    const int R = ((N / Ns) & 3) == 0 ? 4 : 2;
    const int nb = N / R;
    const int step = N / (Ns * R);
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
      const int k = j & (Ns - 1);
      const int o = (j - k) * R + k;
      if (R == 4) {
        cpx<T> v0 = a[j], v1 = a[j + nb], v2 = a[j + 2 * nb], v3 = a[j + 3 * nb];
        if (k) {
          const cpx<T> w1 = tw[k * step], w2 = tw[2 * k * step], w3 = tw[3 * k * step];
          if (INV) {
            v1 = cmulc(v1, w1);
            v2 = cmulc(v2, w2);
            v3 = cmulc(v3, w3);
          } else {
            v1 = cmul(v1, w1);
            v2 = cmul(v2, w2);
            v3 = cmul(v3, w3);
          }
        }
        const cpx<T> t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), d = csub(v1, v3);
        // times -i (forward) or +i (inverse)
        const cpx<T> t3 = INV ? cpx<T>{-d.y, d.x} : cpx<T>{d.y, -d.x};
        b[o] = cadd(t0, t2);
        b[o + Ns] = cadd(t1, t3);
        b[o + 2 * Ns] = csub(t0, t2);
        b[o + 3 * Ns] = csub(t1, t3);
      } else {
        cpx<T> v0 = a[j], v1 = a[j + nb];
        if (k) v1 = INV ? cmulc(v1, tw[k * step]) : cmul(v1, tw[k * step]);
        b[o] = cadd(v0, v1);
        b[o + Ns] = csub(v0, v1);
      }
    }
    __syncthreads();
    cpx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// ---------------------------------------------------------------- set-up kernels
// Twiddle tables exp(-2 pi i m / N) for both frame sides, in FP64 then rounded.
template <typename T>
__global__ void __launch_bounds__(kNT) k_twiddles(Args<T> a) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i < a.Nx) {
    double sn, cs;
    sincospi(-2.0 * i / a.Nx, &sn, &cs);
    a.twx[i] = {(T)cs, (T)sn};
    a.twdx[i] = {cs, sn};
  }
  if (i < a.Ny) {
    double sn, cs;
    sincospi(-2.0 * i / a.Ny, &sn, &cs);
    a.twy[i] = {(T)cs, (T)sn};
    a.twdy[i] = {cs, sn};
  }
}

// exp(-2 pi i m / N) for an integer m of either sign from the FP64 table of N.
__device__ __forceinline__ cpx<double> unit_root(const cpx<double>* tab, long m, int N) {
  long r = m % N;
  if (r < 0) r += N;
  return tab[r];
}

// PSF spectrum, first stage: T1[a][kx] = sum_b P[a][b] exp(-2 pi i kx (b - ck) / Nx).
template <typename T>
__global__ void __launch_bounds__(kNT) k_psf_rows(Args<T> a) {
  const int idx = blockIdx.x * kNT + threadIdx.x;
  if (idx >= a.K * a.Nh) return;
  const int r = idx / a.Nh, kx = idx % a.Nh;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < a.K; ++b) {
    const cpx<double> u = unit_root(a.twdx, (long)kx * (b - a.ck), a.Nx);
    const double v = a.psf[r * a.K + b];
    re += v * u.x;
    im += v * u.y;
  }
  a.T1[idx] = {re, im};
}

// Second stage: H[kx][ky] = sum_a T1[a][kx] exp(-2 pi i ky (a - ck) / Ny) / (Nx Ny).
template <typename T>
__global__ void __launch_bounds__(kNT) k_psf_cols(Args<T> a) {
  const long idx = (long)blockIdx.x * kNT + threadIdx.x;
  if (idx >= (long)a.Nh * a.Ny) return;
  const int kx = (int)(idx / a.Ny), ky = (int)(idx % a.Ny);
  double re = 0.0, im = 0.0;
  for (int r = 0; r < a.K; ++r) {
    const cpx<double> u = unit_root(a.twdy, (long)ky * (r - a.ck), a.Ny);
    const cpx<double> t = a.T1[r * a.Nh + kx];
    re += t.x * u.x - t.y * u.y;
    im += t.x * u.y + t.y * u.x;
  }
  const double sc = 1.0 / ((double)a.Nx * a.Ny);
  a.H[idx] = {(T)(re * sc), (T)(im * sc)};
}

// ---------------------------------------------------------------- the lens operator
// Cubic convolution kernel (Keys, a = -1/2) at distance d >= 0.
__device__ __forceinline__ double keys(double d) {
  return d <= 1.0 ? (1.5 * d - 2.5) * d * d + 1.0 : (d < 2.0 ? ((-0.5 * d + 2.5) * d - 4.0) * d + 2.0 : 0.0);
}

// Tap q of subpixel j: node (or -1) and weight with the 1/n^2 average.
// Bilinear and nearest neighbour: 4 taps, the corners (q >> 1, q & 1) of the
// cell (nearest: the fractions are stored rounded to 0 or 1).  Bicubic: 16
// taps, row offset (q >> 2) - 1 and column offset (q & 3) - 1 from the cell's
// first node, nodes outside the grid left out.
template <typename T>
__device__ __forceinline__ void tap(const Args<T>& a, long j, int q, int& node, double& wt) {
  const Sub<T> sp = a.sub[j];
  const int c = sp.cell;
  node = -1;
  wt = 0.0;
  if (c < 0) return;
  const double fx = (double)sp.fx, fy = (double)sp.fy;
  if (a.taps == 4) {
    const int dr = q >> 1, dc = q & 1;
    node = c + dr * a.ns + dc;
    wt = (dr ? fy : 1.0 - fy) * (dc ? fx : 1.0 - fx) / a.n2;
    return;
  }
  const int jr = (q >> 2) - 1, ic = (q & 3) - 1;
  const int r = c / a.ns + jr, col = c % a.ns + ic;
  if (r < 0 || r >= a.ns || col < 0 || col >= a.ns) return;
  node = r * a.ns + col;
  wt = keys(fabs(fy - jr)) * keys(fabs(fx - ic)) / a.n2;
}

// Ray trace of every subpixel (Eq. 1, Eqs. 10-11, Sec. 2.2) into the
// subpixel table (cell and fractions).
template <typename T>
__global__ void __launch_bounds__(kNT) k_trace(Args<T> a) {
  const long j = (long)blockIdx.x * kNT + threadIdx.x;
  if (j >= (long)a.J * a.n2) return;
  double g[7];
  for (int i = 0; i < 7; ++i) g[i] = a.lens[i];
  const bool valid = lens_valid(g);
  if (j == 0 && !valid) a.flags[0] = 1;
  const int pixel = (int)(j / a.n2), k = (int)(j % a.n2);
  const int r = pixel / a.nx, c = pixel % a.nx;
  int cell = -1;
  double fx = 0.0, fy = 0.0;
  if (valid) {
    const Lens L = make_lens(g);
    double x, y, bx, by;
    subpixel_xy(r, c, k / a.nsub, k % a.nsub, a.nx, a.ny, a.pix, a.nsub, x, y);
    lens_map(L, x, y, bx, by);
    const double h = 2.0 * a.R / (a.ns - 1);
    if (!grid_cell((bx + a.R) / h, (by + a.R) / h, a.ns, cell, fx, fy)) {
      cell = -1;
      fx = fy = 0.0;
    } else if (a.interp == SL_INTERP_NEAREST) {
      fx = fx >= 0.5 ? 1.0 : 0.0;
      fy = fy >= 0.5 ? 1.0 : 0.0;
    }
  }
  a.sub[j] = {cell, (T)fx, (T)fy};
}

// The table entries of one pixel.  With four taps and at most four
// subpixels (bilinear or nearest, n <= 2) the up to 16 (node, weight) pairs
// are merged per node, the weights added in (subpixel, tap) order: entry u of
// the pixel has key pixel * kpp + u.  Otherwise every (subpixel, tap) pair
// is an entry of its own, key (pixel n^2 + subpixel) taps + tap.  Returns
// the number of entries; nd/wt/key hold them.
constexpr int kMergeMax = 16;

template <typename T>
__device__ __forceinline__ bool merged(const Args<T>& a) { return a.taps == 4 && a.n2 <= 4; }

template <typename T>
__device__ int pixel_entries(const Args<T>& a, int pixel, int* nd, double* wt) {
  int np = 0;
  const long j0 = (long)pixel * a.n2;
  for (int k = 0; k < a.n2; ++k)
    for (int q = 0; q < 4; ++q) {
      int node;
      double w;
      tap(a, j0 + k, q, node, w);
      if (node < 0) continue;
      int f = -1;
      for (int u = 0; u < np; ++u)
        if (nd[u] == node) f = u;
      if (f >= 0) {
        wt[f] += w;
      } else {
        nd[np] = node;
        wt[np] = w;
        ++np;
      }
    }
  return np;
}

// Entries per node (one thread per pixel; integer atomics).
template <typename T>
__global__ void __launch_bounds__(kNT) k_count(Args<T> a) {
  const int pixel = blockIdx.x * kNT + threadIdx.x;
  if (pixel >= a.J) return;
  if (merged(a)) {
    int nd[kMergeMax];
    double wt[kMergeMax];
    const int np = pixel_entries(a, pixel, nd, wt);
    for (int u = 0; u < np; ++u) atomicAdd(&a.cnt[nd[u]], 1);
    return;
  }
  const long j0 = (long)pixel * a.n2;
  for (int k = 0; k < a.n2; ++k)
    for (int q = 0; q < a.taps; ++q) {
      int node;
      double w;
      tap(a, j0 + k, q, node, w);
      if (node >= 0) atomicAdd(&a.cnt[node], 1);
    }
}

// Exclusive scan of the entry counts into row starts, in three passes over
// tiles of 1024 nodes: the tiles' totals, their scan (one block), then each
// tile's own scan plus its start.  Integer sums: the order does not matter.
constexpr int kTile = 1024;

// Block-wide exclusive scan of one int per thread (blockDim.x = kNT); returns
// this thread's prefix and sets *total.
__device__ __forceinline__ int block_scan_excl(int v, int* total) {
  __shared__ int ws[kNT / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int incl = v;
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += u;
  }
  if (lane == kWave - 1) ws[wid] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int i = 0; i < kNT / kWave; ++i) {
    if (i < wid) before += ws[i];
    all += ws[i];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_tile_sums(Args<T> a) {
  const int i0 = blockIdx.x * kTile;
  int v = 0, hv = 0;
  for (int k = 0; k < kTile / kNT; ++k) {
    const int i = i0 + threadIdx.x * (kTile / kNT) + k;
    if (i < a.I) {
      v += a.cnt[i];
      hv += a.cnt[i] > lt_heavy<T>();
    }
  }
  int total, htotal;
  (void)block_scan_excl(v, &total);
  (void)block_scan_excl(hv, &htotal);
  if (threadIdx.x == 0) {
    a.tsum[blockIdx.x] = total;
    a.hsum[blockIdx.x] = htotal;
  }
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_tile_scan(Args<T> a) {
  const int tiles = (a.I + kTile - 1) / kTile;   // <= kNT * 4 for I <= 2^20
  int v[4], hv[4];
  int loc = 0, hloc = 0;
  for (int k = 0; k < 4; ++k) {
    const int t = threadIdx.x * 4 + k;
    v[k] = t < tiles ? a.tsum[t] : 0;
    hv[k] = t < tiles ? a.hsum[t] : 0;
    loc += v[k];
    hloc += hv[k];
  }
  int total, htotal;
  int run = block_scan_excl(loc, &total);
  int hrun = block_scan_excl(hloc, &htotal);
  for (int k = 0; k < 4; ++k) {
    const int t = threadIdx.x * 4 + k;
    if (t < tiles) {
      a.tsum[t] = run;
      a.hsum[t] = hrun;
    }
    run += v[k];
    hrun += hv[k];
  }
  if (threadIdx.x == 0) {
    a.rowptr[a.I] = total;
    a.hsum[tiles] = htotal;
  }
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_tile_write(Args<T> a) {
  const int i0 = blockIdx.x * kTile + threadIdx.x * (kTile / kNT);
  int v[kTile / kNT];
  int loc = 0, hloc = 0;
  for (int k = 0; k < kTile / kNT; ++k) {
    v[k] = i0 + k < a.I ? a.cnt[i0 + k] : 0;
    loc += v[k];
    hloc += v[k] > lt_heavy<T>();
  }
  int total, htotal;
  int run = a.tsum[blockIdx.x] + block_scan_excl(loc, &total);
  int hrun = a.hsum[blockIdx.x] + block_scan_excl(hloc, &htotal);
  for (int k = 0; k < kTile / kNT; ++k) {
    if (i0 + k < a.I) {
      a.rowptr[i0 + k] = run;
      a.cursor[i0 + k] = run;
      if (v[k] > lt_heavy<T>()) a.heavy[hrun++] = i0 + k;
    }
    run += v[k];
  }
}

// Table entries in arrival order (one thread per pixel, the entries of
// pixel_entries or of every (subpixel, tap) pair).
template <typename T>
__global__ void __launch_bounds__(kNT) k_fill(Args<T> a) {
  const int pixel = blockIdx.x * kNT + threadIdx.x;
  if (pixel >= a.J) return;
  if (merged(a)) {
    int nd[kMergeMax];
    double wt[kMergeMax];
    const int np = pixel_entries(a, pixel, nd, wt);
    for (int u = 0; u < np; ++u) {
      const int pos = atomicAdd(&a.cursor[nd[u]], 1);
      a.key[pos] = pixel * kMergeMax + u;
      a.wtmp[pos] = (T)wt[u];
    }
    return;
  }
  const long j0 = (long)pixel * a.n2;
  for (int k = 0; k < a.n2; ++k)
    for (int q = 0; q < a.taps; ++q) {
      int node;
      double w;
      tap(a, j0 + k, q, node, w);
      if (node < 0) continue;
      const int pos = atomicAdd(&a.cursor[node], 1);
      a.key[pos] = (int32_t)((j0 + k) * a.taps + q);
      a.wtmp[pos] = (T)w;
    }
}

// Each node's entries placed in ascending key order: the rank of an entry is
// the number of the node's keys below it (keys are distinct, so the order is
// unique).  k_sort: one lane per node sorts a row of at most kSortLane
// entries in registers (rows of at most kSortSmall with the shorter code);
// longer rows (about 1 % of the nodes, clustered near the critical curves) go
// to a list (a.cursor, free after k_fill; its order does not matter) that
// k_sort_long spreads one row per wave: rows of up to kSortChunk entries
// staged in the wave's LDS slice, each lane holding its (at most 16) keys in
// registers and every staged key read once and compared with all of them;
// longer rows compare from global memory.
constexpr int kSortSmall = 8;
constexpr int kSortLane = 32;
constexpr int kSortLongBlocks = 256;   // k_sort_long: 4096 waves over the list

template <typename T>
__device__ __forceinline__ void sort_row_wave(const Args<T>& a, int b, int n, int kpp, int32_t* st, int lane) {
  constexpr int kPer = kSortChunk / kWave;
  const int32_t* keys = a.key + b;
  if (n <= kSortChunk) {
    int mine[kPer], rank[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = lane + t * kWave;
      mine[t] = e < n ? keys[e] : 0x7fffffff;
      rank[t] = 0;
      if (e < n) st[e] = mine[t];
    }
    // the wave's own LDS writes precede its reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int f = 0; f < n; ++f) {
      const int kf = st[f];
#pragma unroll
      for (int t = 0; t < kPer; ++t) rank[t] += kf < mine[t];
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = lane + t * kWave;
      if (e < n) a.lt[b + rank[t]] = {mine[t] / kpp, a.wtmp[b + e]};
    }
    // every lane's reads of this slice precede the next row's writes to it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return;
  }
  for (int e = lane; e < n; e += kWave) {
    const int ke = keys[e];
    int rank = 0;
    for (int f = 0; f < n; ++f) rank += keys[f] < ke;
    a.lt[b + rank] = {ke / kpp, a.wtmp[b + e]};
  }
}

template <typename T>
__device__ __forceinline__ void sort_row_lane(const Args<T>& a, int b, int n, int kpp) {
  constexpr int C = kSortLane;
  int k[C];
#pragma unroll
  for (int t = 0; t < C; ++t) k[t] = t < n ? a.key[b + t] : 0x7fffffff;
#pragma unroll
  for (int t = 0; t < C; ++t) {
    if (t < n) {
      int rank = 0;
#pragma unroll
      for (int f = 0; f < C; ++f) rank += k[f] < k[t];   // padding keys are above every key
      a.lt[b + rank] = {k[t] / kpp, a.wtmp[b + t]};
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_sort(Args<T> a) {
  const int node = blockIdx.x * kNT + threadIdx.x;
  if (node >= a.I) return;
  const int kpp = merged(a) ? kMergeMax : a.n2 * a.taps;   // keys per pixel
  const int b = a.rowptr[node], n = a.rowptr[node + 1] - b;
  if (n <= kSortSmall) {
    int k[kSortSmall];
#pragma unroll
    for (int t = 0; t < kSortSmall; ++t) k[t] = t < n ? a.key[b + t] : 0x7fffffff;
#pragma unroll
    for (int t = 0; t < kSortSmall; ++t) {
      if (t < n) {
        int rank = 0;
#pragma unroll
        for (int f = 0; f < kSortSmall; ++f) rank += k[f] < k[t];
        a.lt[b + rank] = {k[t] / kpp, a.wtmp[b + t]};
      }
    }
  } else if (n <= kSortLane) {
    sort_row_lane(a, b, n, kpp);
  } else {
    a.cursor[atomicAdd(&a.flags[1], 1)] = node;
  }
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_sort_long(Args<T> a) {
  __shared__ int32_t stage[kNT / kWave][kSortChunk];
  const int wv = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int kpp = merged(a) ? kMergeMax : a.n2 * a.taps;
  const int nlong = a.flags[1];
  for (int i = blockIdx.x * (kNT / kWave) + wv; i < nlong; i += gridDim.x * (kNT / kWave)) {   // wave-uniform
    const int node = a.cursor[i];
    const int b = a.rowptr[node];
    sort_row_wave(a, b, a.rowptr[node + 1] - b, kpp, stage[wv], lane);
  }
}

// (L x)(pixel) in T: the subpixels' interpolated values over n^2.
template <typename T>
__device__ __forceinline__ T gather_L(const Args<T>& a, const T* __restrict__ x, int pixel) {
  T acc = 0;
  const long j0 = (long)pixel * a.n2;
  if constexpr (sizeof(T) == 4) {
    if (a.taps == 4 && a.n2 == 4) {
      // the pixel's four 12-byte records are 48 contiguous bytes, 16-byte
      // aligned (workspace and its sections are 256-byte aligned): three
      // 16-byte loads instead of twelve 4-byte ones
      const float4* q = reinterpret_cast<const float4*>(a.sub + j0);
      const float4 q0 = q[0], q1 = q[1], q2 = q[2];
      const float wv[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int c = __float_as_int(wv[3 * k]);
        if (c < 0) continue;
        const T fx = wv[3 * k + 1], fy = wv[3 * k + 2];
        acc += (1 - fy) * ((1 - fx) * x[c] + fx * x[c + 1]) + fy * ((1 - fx) * x[c + a.ns] + fx * x[c + a.ns + 1]);
      }
      return acc / (T)4;
    }
  }
  if (a.taps == 4) {
    for (int k = 0; k < a.n2; ++k) {
      const Sub<T> sp = a.sub[j0 + k];
      const int c = sp.cell;
      if (c < 0) continue;
      const T fx = sp.fx, fy = sp.fy;
      acc += (1 - fy) * ((1 - fx) * x[c] + fx * x[c + 1]) + fy * ((1 - fx) * x[c + a.ns] + fx * x[c + a.ns + 1]);
    }
  } else {
    for (int k = 0; k < a.n2; ++k) {
      const Sub<T> sp = a.sub[j0 + k];
      const int c = sp.cell;
      if (c < 0) continue;
      const double fx = (double)sp.fx, fy = (double)sp.fy;
      const int r = c / a.ns, col = c % a.ns;
      for (int jr = -1; jr <= 2; ++jr) {
        const int rr = r + jr;
        if (rr < 0 || rr >= a.ns) continue;
        T row = 0;
        for (int ic = -1; ic <= 2; ++ic) {
          const int cc = col + ic;
          if (cc >= 0 && cc < a.ns) row += (T)keys(fabs(fx - ic)) * x[rr * a.ns + cc];
        }
        acc += (T)keys(fabs(fy - jr)) * row;
      }
    }
  }
  return acc / (T)a.n2;
}

// ---------------------------------------------------------------- CGLS scalars
// alpha of iteration it = |g|^2 / |A p|^2, or 0 once the iteration has stopped.
// (every thread of the block calls it: barriers)
template <typename T>
__device__ __forceinline__ double alpha_of(const Args<T>& a, int it) {
  const double qq = block_total(part_of(a, P_QQ, it), a.nb_qq);
  if (a.done[it]) return 0.0;
  return qq > 0.0 ? a.gg[it] / qq : 0.0;
}

// ---------------------------------------------------------------- FFT passes
enum { ROW_LP = 0, ROW_D = 2, ROW_IMG = 3 };

// Two real rows packed as one complex row z = y0 + i y1 in LDS, transformed:
// their half spectra Y0[k] = (Z[k] + conj Z[N-k]) / 2 and
// Y1[k] = -i (Z[k] - conj Z[N-k]) / 2 go to dst[kx * Ny + r0] and r0 + 1.
template <typename T>
__device__ __forceinline__ void split_store(const cpx<T>* Z, cpx<T>* dst, int Nx, int Nh, int Ny, int r0, bool two) {
  for (int k = threadIdx.x; k < Nh; k += blockDim.x) {
    const cpx<T> zk = Z[k], zm = Z[(Nx - k) & (Nx - 1)];
    const T h = (T)0.5;
    cpx<T>* d = dst + (long)k * Ny + r0;
    d[0] = {h * (zk.x + zm.x), h * (zk.y - zm.y)};
    if (two) d[1] = {h * (zk.y + zm.y), h * (zm.x - zk.x)};
  }
}

// Forward row FFTs of rows r0 = 2 blockIdx.x and r0 + 1 of an image, packed
// as one complex row, split into the two half spectra.  The image row is
// L p (ROW_LP, into S), the data d (ROW_D, into E: the residual of s = 0),
// or a given image (ROW_IMG, `src`, into S).
template <typename T, int MODE>
__global__ void __launch_bounds__(kRowNT) k_rowfwd(Args<T> a, const T* __restrict__ src) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + a.Nx;
  const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
  const bool two = r1 < a.ny;
  for (int c = threadIdx.x; c < a.Nx; c += blockDim.x) {
    T v0 = 0, v1 = 0;
    if (c < a.nx) {
      const long j0 = (long)r0 * a.nx + c, j1 = j0 + a.nx;
      if (MODE == ROW_LP) {
        v0 = gather_L(a, src, (int)j0);
        if (two) v1 = gather_L(a, src, (int)j1);
      } else if (MODE == ROW_D) {
        v0 = (T)a.d[j0];
        if (two) v1 = (T)a.d[j1];
      } else {
        v0 = src[j0];
        if (two) v1 = src[j1];
      }
    }
    A[c] = {v0, v1};
  }
  __syncthreads();
  const cpx<T>* Z = fft_lds<T, false>(A, B, a.Nx, a.twx);
  split_store(Z, MODE == ROW_D ? a.E : a.S, a.Nx, a.Nh, a.Ny, r0, two);
}

enum { COL_S = 0, COL_E = 1, COL_E_UPD = 2 };

// Column kx = blockIdx.x of a half spectrum: FFT over the Ny rows (rows
// >= ny are zero), product with the PSF spectrum (conjugated for B^T), inverse
// FFT, rows < ny stored to S.  The input column is S's own (COL_S), E's
// (COL_E), or E's after the residual update of iteration it (COL_E_UPD):
// E -= alpha SQ, written back, with the |e|^2 partial of this column by
// Parseval's identity on the zero-padded real rows (weight 1 for kx = 0 and
// Nx/2, 2 otherwise, over Nx).
template <typename T, bool CONJ, int MODE>
__global__ void __launch_bounds__(kNT) k_col(Args<T> a, int it) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + a.Ny;
  const long base = (long)blockIdx.x * a.Ny;
  cpx<T>* col = a.S + base;
  const cpx<T>* Hc = a.H + base;
  // this thread's PSF spectrum values, loaded now so that their latency
  // overlaps the column's load and forward transform
  constexpr int kHr = kMaxFrame / kNT;
  cpx<T> h[kHr];
#pragma unroll
  for (int t = 0; t < kHr; ++t) {
    const int r = threadIdx.x + t * kNT;
    h[t] = r < a.Ny ? Hc[r] : cpx<T>{0, 0};
  }
  double alpha = 0.0;
  if (MODE == COL_E_UPD) {
    alpha = alpha_of(a, it);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.alpha[it] = alpha;   // the update uses the same value
  }
  double ee = 0.0;
  for (int r = threadIdx.x; r < a.Ny; r += blockDim.x) {
    cpx<T> v = {0, 0};
    if (r < a.ny) {
      if (MODE == COL_S) {
        v = col[r];
      } else {
        v = a.E[base + r];
        if (MODE == COL_E_UPD) {
          const cpx<T> q = a.SQ[base + r];
          v = {v.x - (T)alpha * q.x, v.y - (T)alpha * q.y};
          a.E[base + r] = v;
          ee += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        }
      }
    }
    A[r] = v;
  }
  if (MODE == COL_E_UPD) {
    const double wk = (blockIdx.x == 0 || blockIdx.x == a.Nx / 2) ? 1.0 : 2.0;
    put_partial(a, ee * wk / a.Nx, P_EE, it);   // contains the barrier the FFT needs
  } else {
    __syncthreads();
  }
  cpx<T>* Z = fft_lds<T, false>(A, B, a.Ny, a.twy);
#pragma unroll
  for (int t = 0; t < kHr; ++t) {
    const int r = threadIdx.x + t * kNT;
    if (r < a.Ny) Z[r] = CONJ ? cmulc(Z[r], h[t]) : cmul(Z[r], h[t]);
  }
  __syncthreads();
  cpx<T>* Y = fft_lds<T, true>(Z, Z == A ? B : A, a.Ny, a.twy);
  for (int r = threadIdx.x; r < a.ny; r += blockDim.x) col[r] = Y[r];
}

enum { OUT_Q = 0, OUT_W = 1, OUT_IMG = 2 };

// Inverse row FFTs of rows r0 = 2 blockIdx.x and r0 + 1 from their half
// spectra (the other half by conjugate symmetry, as the rows are real):
// Z[k] = Q0[k] + i Q1[k], inverse FFT, row r0 the real and row r0 + 1 the
// imaginary part.  OUT_W: w; OUT_IMG: dst.  OUT_Q: q = A p is kept in the
// spectral domain: its |q|^2 partial, then the rows cut to the image (zero
// from column nx on) and transformed forward again into SQ.
template <typename T, int OUT>
__global__ void __launch_bounds__(kRowNT) k_rowinv(Args<T> a, T* __restrict__ dst, int it) {
  extern __shared__ __align__(16) unsigned char smem[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* B = A + a.Nx;
  const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
  const bool two = r1 < a.ny;
  const int half = a.Nx / 2;
  for (int k = threadIdx.x; k < a.Nx; k += blockDim.x) {
    const bool mirror = k > half;
    const int kk = mirror ? a.Nx - k : k;
    const cpx<T>* src = a.S + (long)kk * a.Ny + r0;
    cpx<T> q0 = src[0], q1 = two ? src[1] : cpx<T>{0, 0};
    if (mirror) {
      q0.y = -q0.y;
      q1.y = -q1.y;
    }
    A[k] = {q0.x - q1.y, q0.y + q1.x};
  }
  __syncthreads();
  cpx<T>* z = fft_lds<T, true>(A, B, a.Nx, a.twx);
  if (OUT == OUT_Q) {
    double qq = 0.0;
    for (int c = threadIdx.x; c < a.Nx; c += blockDim.x) {
      if (c < a.nx) {
        const T v0 = z[c].x, v1 = two ? z[c].y : (T)0;
        z[c] = {v0, v1};
        qq += (double)v0 * (double)v0 + (double)v1 * (double)v1;
      } else {
        z[c] = {0, 0};
      }
    }
    put_partial(a, qq, P_QQ, it);   // its barrier orders the cut before the transform
    const cpx<T>* Zq = fft_lds<T, false>(z, z == A ? B : A, a.Nx, a.twx);
    split_store(Zq, a.SQ, a.Nx, a.Nh, a.Ny, r0, two);
    return;
  }
  T* out = OUT == OUT_W ? a.w : dst;
  for (int c = threadIdx.x; c < a.nx; c += blockDim.x) {
    out[(long)r0 * a.nx + c] = z[c].x;
    if (two) out[(long)r1 * a.nx + c] = z[c].y;
  }
}

// ---------------------------------------------------------------- tiled blur
// Overlap-save on 128-wide, 96-tall tiles (FP32, PSF side <= 65): output tile
// (ty, tx) owns the 32 x 64 pixels (rows x columns) from (32 ty, 64 tx); its
// input is the 96 x 128 region 32 pixels wider on every side (zero outside
// the image), on which the circular convolution equals the zero-padded one for
// the owned pixels.  One block per tile runs the whole 2-D transform in LDS:
// two real rows packed per complex row FFT (length 128), their half spectra
// (65 columns) transformed along the columns (length 96), the product with the
// tile's PSF spectrum, and back.  One launch per blur instead of three passes
// through HBM; 32-row owned blocks give 200 tiles at 640 x 640, so that most
// compute units take one.
constexpr int kTN = 128;                      // tile width (row FFT length)
constexpr int kTNY = 96;                      // tile height (column FFT length)
constexpr int kTV = 64;                       // owned columns
constexpr int kTVY = 32;                      // owned rows
constexpr int kTHalo = 32;                    // halo on every side: the PSF half-width it allows
static_assert(kTN - kTV == 2 * kTHalo && kTNY - kTVY == 2 * kTHalo, "tile = owned block + halo");
constexpr int kTH = kTN / 2 + 1;              // 65 half-spectrum columns
constexpr int kTNT = 1024;

// In-register DFTs of length 4, 8 and 16 (INV: the conjugate kernel), in
// natural order in and out.  The lengths 8 and 16 split as 2 x 4 and 4 x 4
// (Cooley-Tukey: inner DFT4s, the factor w_R^(n2 k1), outer DFTs).
template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  const cpx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), d = csub(a1, a3);
  const cpx<T> t3 = INV ? cpx<T>{-d.y, d.x} : cpx<T>{d.y, -d.x};
  a0 = cadd(t0, t2);
  a1 = cadd(t1, t3);
  a2 = csub(t0, t2);
  a3 = csub(t1, t3);
}

// v times exp(-+2 pi i e / 16) for a constant e (the sign by INV)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> w16(cpx<T> v, int e) {
  constexpr double c1 = 0.92387953251128674, s1 = 0.38268343236508977, c2 = 0.70710678118654752;
  const double cs[16] = {1, c1, c2, s1, 0, -s1, -c2, -c1, -1, -c1, -c2, -s1, 0, s1, c2, c1};
  const double sn[16] = {0, s1, c2, c1, 1, c1, c2, s1, 0, -s1, -c2, -c1, -1, -c1, -c2, -s1};
  const cpx<T> w = {(T)cs[e & 15], INV ? (T)sn[e & 15] : -(T)sn[e & 15]};
  return cmul(v, w);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cpx<T> (&v)[8]) {
  // n = 2 n1 + n2: DFT4 over n1 for each n2, twiddle w8^(n2 k1), DFT2 over n2
  dft4<T, INV>(v[0], v[2], v[4], v[6]);
  dft4<T, INV>(v[1], v[3], v[5], v[7]);
  cpx<T> o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    const cpx<T> y0 = v[2 * k1], y1 = k1 ? w16<T, INV>(v[2 * k1 + 1], 2 * k1) : v[2 * k1 + 1];
    o[k1] = cadd(y0, y1);
    o[k1 + 4] = csub(y0, y1);
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) v[m] = o[m];
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(cpx<T> (&v)[16]) {
  // n = 4 n1 + n2: DFT4 over n1 for each n2 (result k1 in slot 4 k1 + n2),
  // twiddle w16^(n2 k1), DFT4 over n2 for each k1 (result k1 + 4 k2 in slot 4 k1 + k2)
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<T, INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2) v[4 * k1 + n2] = w16<T, INV>(v[4 * k1 + n2], n2 * k1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<T, INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  cpx<T> o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = o[m];
}

// Length-128 FFTs of the tile as two Stockham stages (as in fft_lds):
// stage 1 (radix 16, span 1): butterfly j < 8 of a row reads x[j + 8 r]
// (r < 16) and writes its DFT16 to positions 16 j + m; stage 2 (radix 8,
// span 16): butterfly j < 16 reads positions j + 16 r (r < 8), turns input r
// by w^(r j) and writes its DFT8 to positions j + 16 m.  Rows and columns
// live in buffers of row stride kTLD; the intermediate goes to a scratch of
// row stride kTP with one pad element after every 16 (position e at
// e + e / 16).  With the lanes of stage 1 taking rows b and b + 8 in each
// group of 16, every LDS access of both stages meets distinct banks.
constexpr int kTLD = kTN + 1;   // 129: odd, so the transposes (lanes along rows) meet distinct banks
constexpr int kTP = kTN + kTN / 16 + 1;   // 137

__device__ __forceinline__ int p16(int b, int e) { return b * kTP + e + (e >> 4); }

// lane item wi of stage 1 -> (row b, butterfly j): in each group of 16 lanes,
// 8 take row b and 8 row b + 8; rows past the last full set of 16 (the
// Nyquist column of the half spectra) one after another
template <int NB>
__device__ __forceinline__ void stage1_map(int wi, int& b, int& j) {
  j = wi & 7;
  if (wi < (NB / 16) * 16 * 8) {
    const int g = wi >> 4, h = (wi >> 3) & 1;
    b = (g >> 3) * 16 + (g & 7) + 8 * h;
  } else {
    b = wi >> 3;
  }
}

template <typename T, bool INV, int NB>
__device__ __forceinline__ void tile_stage1(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y) {
  constexpr int ITEMS = NB * 8, U = (ITEMS + kTNT - 1) / kTNT;
  cpx<T> v[U][16];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int wi = threadIdx.x + u * kTNT;
    if (ITEMS % kTNT == 0 || wi < ITEMS) {
      int b, j;
      stage1_map<NB>(wi, b, j);
#pragma unroll
      for (int r = 0; r < 16; ++r) v[u][r] = x[b * kTLD + j + 8 * r];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int wi = threadIdx.x + u * kTNT;
    if (ITEMS % kTNT == 0 || wi < ITEMS) {
      int b, j;
      stage1_map<NB>(wi, b, j);
      dft16<T, INV>(v[u]);
      cpx<T>* o_ = y + p16(b, 16 * j);
#pragma unroll
      for (int m = 0; m < 16; ++m) o_[m] = v[u][m];
    }
  }
  __syncthreads();
}

// tw8[(r - 1) * 16 + j] = w^(r j), r = 1..7, j < 16 (LDS; lanes along j)
template <typename T, bool INV, int NB>
__device__ __forceinline__ void tile_stage2(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y, const cpx<T>* tw8) {
  constexpr int ITEMS = NB * 16, U = (ITEMS + kTNT - 1) / kTNT;
  cpx<T> v[U][8];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int wi = threadIdx.x + u * kTNT;
    if (ITEMS % kTNT == 0 || wi < ITEMS) {
      const int b = wi >> 4, j = wi & 15;
#pragma unroll
      for (int r = 0; r < 8; ++r) v[u][r] = x[p16(b, j + 16 * r)];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int wi = threadIdx.x + u * kTNT;
    if (ITEMS % kTNT == 0 || wi < ITEMS) {
      const int b = wi >> 4, j = wi & 15;
      if (j) {
#pragma unroll
        for (int r = 1; r < 8; ++r) {
          const cpx<T> w = tw8[(r - 1) * 16 + j];
          v[u][r] = INV ? cmulc(v[u][r], w) : cmul(v[u][r], w);
        }
      }
      dft8<T, INV>(v[u]);
      cpx<T>* o_ = y + b * kTLD + j;
#pragma unroll
      for (int m = 0; m < 8; ++m) o_[16 * m] = v[u][m];
    }
  }
  __syncthreads();
}

// NB length-128 FFTs in place in x (row stride kTLD), y the stage scratch.
template <typename T, bool INV, int NB>
__device__ __forceinline__ void fft_tile(cpx<T>* x, cpx<T>* y, const cpx<T>* tw8) {
  static_assert(kTN == 128, "stage list is for length 128");
  tile_stage1<T, INV, NB>(x, y);
  tile_stage2<T, INV, NB>(y, x, tw8);
}

// Column transforms (length 96, the tile height) as two Stockham stages:
// stage 1 (radix 16, span 1): butterfly j < 6 of a column reads x[j + 6 r]
// (r < 16) and writes its DFT16 to positions 16 j + m; stage 2 (radix 6,
// span 16): butterfly j < 16 reads positions j + 16 r (r < 6), turns input r
// by w96^(r j) and writes its DFT6 to positions j + 16 m.  Columns live with
// stride kTLDC, the intermediate in a scratch of stride kTPC with one pad
// element after every 16.
constexpr int kTLDC = kTNY + 1;                 // 97
constexpr int kTPC = kTNY + kTNY / 16 + 1;      // 103
constexpr int kTBuf = kTH * kTPC;               // complex elements per LDS buffer
static_assert(kTNY / 2 * kTP <= kTBuf && kTH * kTLDC <= kTBuf && kTNY / 2 * kTLD <= kTBuf, "tile buffers fit");

__device__ __forceinline__ int p16c(int b, int e) { return b * kTPC + e + (e >> 4); }

// DFT3 and DFT6 (INV: the conjugate kernel), natural order in and out; the
// length 6 splits as 3 x 2 (DFT3s, the factor w6^(n2 k1), DFT2s)
template <typename T, bool INV>
__device__ __forceinline__ void dft3(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2) {
  const T sn = INV ? (T)0.86602540378443865 : (T)-0.86602540378443865;   // sin of -+2 pi / 3
  const cpx<T> sm = cadd(a1, a2), d = csub(a1, a2);
  const cpx<T> t = {a0.x - (T)0.5 * sm.x, a0.y - (T)0.5 * sm.y};
  const cpx<T> u = {-sn * d.y, sn * d.x};   // i sn d
  a0 = cadd(a0, sm);
  a1 = cadd(t, u);
  a2 = csub(t, u);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft6(cpx<T> (&v)[6]) {
  dft3<T, INV>(v[0], v[2], v[4]);   // n2 = 0: result k1 in slot 2 k1
  dft3<T, INV>(v[1], v[3], v[5]);   // n2 = 1: result k1 in slot 2 k1 + 1
  const T h = (T)0.5, r3 = INV ? (T)0.86602540378443865 : (T)-0.86602540378443865;
  const cpx<T> w1 = {h, r3}, w2 = {-h, r3};   // w6^1, w6^2
  cpx<T> o[6];
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    const cpx<T> y0 = v[2 * k1];
    const cpx<T> y1 = k1 == 0 ? v[1] : cmul(v[2 * k1 + 1], k1 == 1 ? w1 : w2);
    o[k1] = cadd(y0, y1);
    o[k1 + 3] = csub(y0, y1);
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) v[m] = o[m];
}

// HM = 1 (2): each input times H (conj H), stored [ky][kx] (96 x 65), first.
template <typename T, bool INV, int HM>
__device__ __forceinline__ void col_stage1(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y,
                                           const cpx<T>* __restrict__ H) {
  constexpr int ITEMS = kTH * 6;
  static_assert(ITEMS <= kTNT, "one butterfly per thread");
  const int wi = threadIdx.x;
  cpx<T> v[16];
  // consecutive lanes take consecutive columns (b = wi mod 65): the reads of a
  // stage are then contiguous and its scratch writes 103 = 7 mod 32 apart
  if (wi < ITEMS) {
    const int j = wi / kTH, b = wi - j * kTH;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = x[b * kTLDC + j + 6 * r];
    if (HM) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const cpx<T> hh = H[(j + 6 * r) * kTH + b];   // Ht is [ky][kx]: lanes along kx read consecutive values
        v[r] = HM == 1 ? cmul(v[r], hh) : cmulc(v[r], hh);
      }
    }
  }
  if (wi < ITEMS) {
    const int j = wi / kTH, b = wi - j * kTH;
    dft16<T, INV>(v);
    cpx<T>* o_ = y + p16c(b, 16 * j);
#pragma unroll
    for (int m = 0; m < 16; ++m) o_[m] = v[m];
  }
  __syncthreads();
}

// tw6[(r - 1) * 16 + j] = w96^(r j), r = 1..5, j < 16 (LDS)
template <typename T, bool INV>
__device__ __forceinline__ void col_stage2(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y, const cpx<T>* tw6) {
  constexpr int ITEMS = kTH * 16, U = (ITEMS + kTNT - 1) / kTNT;
  cpx<T> v[U][6];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int wi = threadIdx.x + u * kTNT;
    if (wi < ITEMS) {
      const int b = wi >> 4, j = wi & 15;
#pragma unroll
      for (int r = 0; r < 6; ++r) v[u][r] = x[p16c(b, j + 16 * r)];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int wi = threadIdx.x + u * kTNT;
    if (wi < ITEMS) {
      const int b = wi >> 4, j = wi & 15;
      if (j) {
#pragma unroll
        for (int r = 1; r < 6; ++r) {
          const cpx<T> w = tw6[(r - 1) * 16 + j];
          v[u][r] = INV ? cmulc(v[u][r], w) : cmul(v[u][r], w);
        }
      }
      dft6<T, INV>(v[u]);
      cpx<T>* o_ = y + b * kTLDC + j;
#pragma unroll
      for (int m = 0; m < 6; ++m) o_[16 * m] = v[u][m];
    }
  }
  __syncthreads();
}

// The 65 half-spectrum columns (length 96) in place in x (stride kTLDC), y the stage scratch.
template <typename T, bool INV, int HM = 0>
__device__ __forceinline__ void fft_cols(cpx<T>* x, cpx<T>* y, const cpx<T>* tw6, const cpx<T>* __restrict__ H = nullptr) {
  static_assert(kTNY == 96, "stage list is for length 96");
  col_stage1<T, INV, HM>(x, y, H);
  col_stage2<T, INV>(y, x, tw6);
}

enum { TILE_B = 0, TILE_BT0 = 1, TILE_BT = 2 };

// First forward column stage with the unpacking of the row spectra fused in:
// column kx, row r of the half spectra is formed from packed row r / 2 of the
// row transforms in x (stride kTLD) at kx and 128 - kx (two real rows' spectra
// from one complex one); writes the stage scratch y (as col_stage1).
template <typename T>
__device__ __forceinline__ void col_stage1_unpack(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y) {
  constexpr int ITEMS = kTH * 6;
  const int wi = threadIdx.x;
  cpx<T> v[16];
  if (wi < ITEMS) {
    const int j = wi / kTH, b = wi - j * kTH;   // consecutive lanes, consecutive columns (as col_stage1)
    const int km = (kTN - b) & (kTN - 1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int rr = j + 6 * r, pr = rr >> 1;
      const cpx<T> zk = x[pr * kTLD + b], zm = x[pr * kTLD + km];
      const T h = (T)0.5;
      v[r] = (rr & 1) ? cpx<T>{h * (zk.y + zm.y), h * (zm.x - zk.x)} : cpx<T>{h * (zk.x + zm.x), h * (zk.y - zm.y)};
    }
  }
  if (wi < ITEMS) {
    const int j = wi / kTH, b = wi - j * kTH;
    dft16<T, false>(v);
    cpx<T>* o_ = y + p16c(b, 16 * j);
#pragma unroll
    for (int m = 0; m < 16; ++m) o_[m] = v[m];
  }
  __syncthreads();
}

// First inverse row stage of packed rows PR0..PR0+NPR-1 with the repacking
// fused in: packed row pr at column k is Q0[k] + i Q1[k] of the two tile rows
// 2 pr, 2 pr + 1, read from the column-major spectra x (stride kTLDC), the
// upper half by conjugate symmetry; writes the row stage scratch y (rows
// 0..NPR-1, as tile_stage1).
template <typename T, int PR0, int NPR>
__device__ __forceinline__ void row_stage1_repack(const cpx<T>* __restrict__ x, cpx<T>* __restrict__ y) {
  constexpr int ITEMS = NPR * 8;
  static_assert(ITEMS <= kTNT && NPR % 16 == 0, "one butterfly per thread, whole sets of 16 rows");
  const int wi = threadIdx.x;
  cpx<T> v[16];
  int b = 0, j = 0;
  if (wi < ITEMS) {
    stage1_map<NPR>(wi, b, j);
    const int pr = PR0 + b;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int k = j + 8 * r;
      const bool mirror = k > kTN / 2;
      const int kk = mirror ? kTN - k : k;
      cpx<T> q0 = x[kk * kTLDC + 2 * pr], q1 = x[kk * kTLDC + 2 * pr + 1];
      if (mirror) {
        q0.y = -q0.y;
        q1.y = -q1.y;
      }
      v[r] = {q0.x - q1.y, q0.y + q1.x};
    }
  }
  if (wi < ITEMS) {
    dft16<T, true>(v);
    cpx<T>* o_ = y + p16(b, 16 * j);
#pragma unroll
    for (int m = 0; m < 16; ++m) o_[m] = v[m];
  }
  __syncthreads();
}

// One tile of a blur.  TILE_B: q = B y on the owned pixels, with the block's
// |q|^2 partial.  TILE_BT0: w = B^T e0 (e0 = d).  TILE_BT: the residual
// update e_out = e_in - alpha q (alpha of iteration it; written on the owned
// pixels, recomputed on the halo), the block's |e|^2 partial, and
// w = B^T e_out.  Only the packed rows that hold owned pixels (16..31) take
// the inverse row transform.  Packed rows are kept with row stride kTLD,
// column-major half spectra with stride kTLDC.
template <typename T, int MODE>
__global__ void __launch_bounds__(kTNT) k_tile(Args<T> a, const T* __restrict__ e_in, T* __restrict__ e_out, int it) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cpx<T> tw8[7 * 16];
  __shared__ cpx<T> tw6[5 * 16];
  cpx<T>* X = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* Y = X + kTBuf;
  const int tile = xcd_item(blockIdx.x, gridDim.x);
  const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
  const int y0 = ty * kTVY - kTHalo, x0 = tx * kTV - kTHalo;   // image position of tile element (0, 0)
  if (threadIdx.x < 7 * 16) {
    const int r = threadIdx.x / 16 + 1, j = threadIdx.x & 15;
    tw8[threadIdx.x] = a.twt[(r * j) & (kTN - 1)];
    if (r <= 5) tw6[threadIdx.x] = a.twc[(r * j) % kTNY];
  }
  // load: packed row pr holds tile rows 2 pr (real part) and 2 pr + 1 (imaginary part);
  // thread t takes column t mod 128 of packed rows t / 128 + 8 u
  constexpr int LU = kTNY / 2 * kTN / kTNT;
  static_assert(LU * kTNT == kTNY / 2 * kTN, "whole packed rows per pass");
  const int c = threadIdx.x & (kTN - 1), pr0 = threadIdx.x / kTN;
  const int cc = x0 + c;
  const bool col_in = cc >= 0 && cc < a.nx;
  T v[LU][2], qv[LU][2];
#pragma unroll
  for (int u = 0; u < LU; ++u) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = y0 + 2 * (pr0 + 8 * u) + h;
      const bool in = col_in && r >= 0 && r < a.ny;
      const long j = (long)r * a.nx + cc;
      const T* src = MODE == TILE_B ? a.y : e_in;
      v[u][h] = in ? src[j] : (T)0;
      if (MODE == TILE_BT) qv[u][h] = in ? a.q[j] : (T)0;
    }
  }
  double alpha = 0.0;   // after the loads are issued: its reduction waits on other blocks' partials
  if (MODE == TILE_BT) {
    alpha = alpha_of(a, it);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.alpha[it] = alpha;   // the update uses the same value
  }
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < LU; ++u) {
    const int pr = pr0 + 8 * u;
    if (MODE == TILE_BT) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v[u][h] -= (T)alpha * qv[u][h];
        const int r = y0 + 2 * pr + h;
        const int lr = 2 * pr + h - kTHalo, lc = c - kTHalo;
        if (col_in && r >= 0 && r < a.ny && lr >= 0 && lr < kTVY && lc >= 0 && lc < kTV) {   // owned: once
          e_out[(long)r * a.nx + cc] = v[u][h];
          part += (double)v[u][h] * (double)v[u][h];
        }
      }
    }
    X[pr * kTLD + c] = {v[u][0], v[u][1]};
  }
  if (MODE == TILE_BT) put_partial(a, part, P_EE, it, tile);   // contains the barrier the FFT needs
  else __syncthreads();
  fft_tile<T, false, kTNY / 2>(X, Y, tw8);                 // row spectra in X
  col_stage1_unpack<T>(X, Y);                               // half spectra, columns: stage 1 into Y
  col_stage2<T, false>(Y, X, tw6);                          // columns (stride kTLDC) in X
  fft_cols<T, true, MODE == TILE_B ? 1 : 2>(X, Y, tw6, a.Ht);   // times the PSF spectrum, inverse columns
  constexpr int PR0 = kTHalo / 2, NPR = kTVY / 2;           // packed rows 16..31 hold the owned rows
  row_stage1_repack<T, PR0, NPR>(X, Y);
  // last inverse row stage (as tile_stage2), its owned outputs written to the image directly
  T* out = MODE == TILE_B ? a.q : a.w;
  double qq = 0.0;
  if (threadIdx.x < NPR * 16) {
    const int b = threadIdx.x >> 4, j = threadIdx.x & 15;
    cpx<T> v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = Y[p16(b, j + 16 * r)];
    if (j) {
#pragma unroll
      for (int r = 1; r < 8; ++r) v[r] = cmulc(v[r], tw8[(r - 1) * 16 + j]);
    }
    dft8<T, true>(v);
    const int r0 = y0 + 2 * (PR0 + b);   // image rows of the packed row's real and imaginary parts
#pragma unroll
    for (int m = kTHalo / 16; m < (kTHalo + kTV) / 16; ++m) {   // owned columns 32..95: m = 2..5
      const int cx = x0 + j + 16 * m;
      if (cx >= a.nx) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = r0 + h;
        if (r >= a.ny) continue;
        const T val = h ? v[m].y : v[m].x;
        out[(long)r * a.nx + cx] = val;
        if (MODE == TILE_B) qq += (double)val * (double)val;
      }
    }
  }
  if (MODE == TILE_B) put_partial(a, qq, P_QQ, it, tile);
}

// y = L p (one thread per pixel).
template <typename T>
__global__ void __launch_bounds__(kNT) k_gather(Args<T> a) {
  const int pixel = blockIdx.x * kNT + threadIdx.x;
  if (pixel < a.J) a.y[pixel] = gather_L(a, a.p, pixel);
}

// e0 = d in T.
template <typename T>
__global__ void __launch_bounds__(kNT) k_copy_d(Args<T> a) {
  const int j = blockIdx.x * kNT + threadIdx.x;
  if (j < a.J) a.e0[j] = (T)a.d[j];
}

// The tile's PSF spectrum
//   Ht[ky][kx] = sum_{a,b} P[a][b] exp(-2 pi i (ky (a - ck) / 96 + kx (b - ck) / 128)) / (128 96)
// in FP64, separably: first T1t[a][kx] over b (and the tile twiddles), then over a.
// exp(-2 pi i m / n)
__device__ __forceinline__ cpx<double> root_of(long m, int n) {
  m %= n;
  if (m < 0) m += n;
  double sn, cs;
  sincospi(-2.0 * (double)m / n, &sn, &cs);
  return {cs, sn};
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_tile_psf_rows(Args<T> a) {
  const int idx = blockIdx.x * kNT + threadIdx.x;
  if (idx < kTN) {
    const cpx<double> u = root_of(idx, kTN);
    a.twt[idx] = {(T)u.x, (T)u.y};
  }
  if (idx < kTNY) {
    const cpx<double> u = root_of(idx, kTNY);
    a.twc[idx] = {(T)u.x, (T)u.y};
  }
  if (idx >= a.K * kTH) return;
  const int r = idx / kTH, kx = idx - r * kTH;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < a.K; ++b) {
    const cpx<double> u = root_of((long)kx * (b - a.ck), kTN);
    const double v = a.psf[r * a.K + b];
    re += v * u.x;
    im += v * u.y;
  }
  a.T1t[idx] = {re, im};
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_tile_psf_cols(Args<T> a) {
  const int idx = blockIdx.x * kNT + threadIdx.x;
  if (idx >= kTH * kTNY) return;
  const int ky = idx / kTH, kx = idx - ky * kTH;   // stored [ky][kx]
  double re = 0.0, im = 0.0;
  for (int r = 0; r < a.K; ++r) {
    const cpx<double> u = root_of((long)ky * (r - a.ck), kTNY);
    const cpx<double> t = a.T1t[r * kTH + kx];
    re += t.x * u.x - t.y * u.y;
    im += t.x * u.y + t.y * u.x;
  }
  const double sc = 1.0 / ((double)kTN * kTNY);
  a.Ht[idx] = {(T)(re * sc), (T)(im * sc)};
}

// ---------------------------------------------------------------- source-side kernels
// g = L^T w over the sorted table, with its |g|^2 partial in slot `it`:
// lt_lanes lanes per node, lane l adding entries l, l + kLtG, ... in order, then
// a fixed butterfly over the group; lane 0 holds the node's value.  Each
// thread serves lt_groups node groups at once (most nodes have fewer entries than
// lanes, so a node is one dependent chain of loads: row bounds, entry, w).
// Grid-stride over the nodes (nb_lt <= kMaxParts blocks).
template <typename T>
__global__ void __launch_bounds__(kLtNT) k_lt(Args<T> a, int it) {
  constexpr int kLtU = lt_groups<T>(), kLtG = lt_lanes<T>();
  double gg = 0.0;
  const int nb_reg = a.nb_lt - a.nb_heavy;
  if ((int)blockIdx.x < a.nb_heavy) {
    // heavy nodes (the first blocks, so that their longer chains start first):
    // one wave per node, lane l adding entries l, l + 64, ... in order (four
    // loads in flight), then a fixed butterfly over the wave
    const int lane = threadIdx.x & (kWave - 1);
    const int nh = a.hsum[(a.I + kTile - 1) / kTile];
    constexpr int waves = kLtNT / kWave;
    for (int h = (int)blockIdx.x * waves + (int)threadIdx.x / kWave; h < nh; h += a.nb_heavy * waves) {
      const int node = a.heavy[h];
      const int e1 = a.rowptr[node + 1];
      int e = a.rowptr[node] + lane;
      T acc = 0;
      for (; e + 3 * kWave < e1; e += 4 * kWave) {
        const LtE<T> t0 = a.lt[e], t1 = a.lt[e + kWave], t2 = a.lt[e + 2 * kWave], t3 = a.lt[e + 3 * kWave];
        const T w0 = a.w[t0.pix], w1 = a.w[t1.pix], w2 = a.w[t2.pix], w3 = a.w[t3.pix];
        acc += t0.w * w0;
        acc += t1.w * w1;
        acc += t2.w * w2;
        acc += t3.w * w3;
      }
      for (; e < e1; e += kWave) {
        const LtE<T> tt = a.lt[e];
        acc += tt.w * a.w[tt.pix];
      }
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
      if (lane == 0) {
        a.g[node] = acc;
        gg += (double)acc * (double)acc;
      }
    }
    put_partial(a, gg, P_GG, it);
    return;
  }
  const int l = threadIdx.x & (kLtG - 1);
  constexpr int per_pass = kLtNT / kLtG;
  // node ranges in block order, so consecutive ranges go to different XCDs:
  // the long rows cluster near the critical curves, and contiguous runs of
  // ranges per XCD (as the tiles take) load one XCD with most of them
  const int rb = (int)blockIdx.x - a.nb_heavy;
  for (int n0 = rb * per_pass * kLtU; n0 < a.I; n0 += nb_reg * per_pass * kLtU) {
    // kLtU node groups per thread: their row bounds, first entries and w values in flight together
    int node[kLtU], e[kLtU], e1[kLtU];
    bool own[kLtU];   // the node is summed here (in range and not heavy)
    T acc[kLtU];
#pragma unroll
    for (int u = 0; u < kLtU; ++u) {
      node[u] = n0 + u * per_pass + threadIdx.x / kLtG;
      const bool ok = node[u] < a.I;
      const int r0 = ok ? a.rowptr[node[u]] : 0, r1 = ok ? a.rowptr[node[u] + 1] : 0;
      own[u] = ok && r1 - r0 <= lt_heavy<T>();
      e[u] = r0 + l;
      e1[u] = own[u] ? r1 : 0;
      acc[u] = 0;
    }
    LtE<T> t[kLtU];
#pragma unroll
    for (int u = 0; u < kLtU; ++u) t[u] = e[u] < e1[u] ? a.lt[e[u]] : LtE<T>{0, (T)0};
    T wv[kLtU];
#pragma unroll
    for (int u = 0; u < kLtU; ++u) wv[u] = e[u] < e1[u] ? a.w[t[u].pix] : (T)0;
#pragma unroll
    for (int u = 0; u < kLtU; ++u) {
      if (e[u] < e1[u]) acc[u] += t[u].w * wv[u];
      e[u] += kLtG;
      // the rest of the lane's entries, in order, four loads in flight
      for (; e[u] + 3 * kLtG < e1[u]; e[u] += 4 * kLtG) {
        const LtE<T> t0 = a.lt[e[u]], t1 = a.lt[e[u] + kLtG], t2 = a.lt[e[u] + 2 * kLtG], t3 = a.lt[e[u] + 3 * kLtG];
        const T w0 = a.w[t0.pix], w1 = a.w[t1.pix], w2 = a.w[t2.pix], w3 = a.w[t3.pix];
        acc[u] += t0.w * w0;
        acc[u] += t1.w * w1;
        acc[u] += t2.w * w2;
        acc[u] += t3.w * w3;
      }
      for (; e[u] < e1[u]; e[u] += kLtG) {
        const LtE<T> tt = a.lt[e[u]];
        acc[u] += tt.w * a.w[tt.pix];
      }
    }
#pragma unroll
    for (int u = 0; u < kLtU; ++u) {
#pragma unroll
      for (int o = kLtG / 2; o > 0; o >>= 1) acc[u] += __shfl_xor(acc[u], o, kLtG);
      if (own[u] && l == 0) {
        a.g[node[u]] = acc[u];
        gg += (double)acc[u] * (double)acc[u];
      }
    }
  }
  put_partial(a, gg, P_GG, it);
}

// Start: s = 0, p = g = A^T d, |g|^2 (slot n_iter holds its partials).
template <typename T>
__global__ void __launch_bounds__(kNodeNT) k_start(Args<T> a) {
  for (int i = blockIdx.x * kNodeNT + threadIdx.x; i < a.I; i += gridDim.x * kNodeNT) {
    a.s[i] = 0;
    a.p[i] = a.g[i];
  }
  const double gg = block_total(part_of(a, P_GG, a.n_iter), a.nb_lt);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.gg[0] = gg;
    a.done[0] = !(gg > 0.0);
  }
}

// End of iteration it: s += alpha p, p = g + beta p with beta = |g_new|^2 / |g|^2,
// the iterate kept and its |s|^2 partial; block 0 records the scalars of the
// next iteration.  Grid-stride over the nodes (nb_node <= kMaxParts blocks).
template <typename T>
__global__ void __launch_bounds__(kNodeNT) k_update(Args<T> a, int it) {
  // the first node's operands are loaded before the |g|^2 total, whose
  // partial loads and block reduction then hide their latency
  const int i0 = blockIdx.x * kNodeNT + threadIdx.x;
  T s0 = 0, p0 = 0, g0 = 0;
  if (i0 < a.I) {
    s0 = a.s[i0];
    p0 = a.p[i0];
    g0 = a.g[i0];
  }
  const double alpha = a.alpha[it];
  const bool moved = alpha > 0.0;
  const double gn = block_total(part_of(a, P_GG, it), a.nb_lt);
  const bool stop = !moved || !(gn > 0.0);
  const double beta = stop ? 0.0 : gn / a.gg[it];
  double ss = 0.0;
  for (int i = i0; i < a.I; i += gridDim.x * kNodeNT) {
    const bool first = i == i0;
    T s = first ? s0 : a.s[i];
    const T p = first ? p0 : a.p[i], g = first ? g0 : a.g[i];
    if (moved) {
      s += (T)alpha * p;
      a.s[i] = s;
      a.p[i] = g + (T)beta * p;
    }
    a.s_iter[(long)it * a.I + i] = s;
    ss += (double)s * (double)s;
  }
  put_partial(a, ss, P_SS, it);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.gg[it + 1] = moved ? gn : a.gg[it];
    a.done[it + 1] = a.done[it] || stop;
    a.upd[it] = moved;
  }
}

// chi^2 and sum s^2 of every iterate, statuses, the L-curve corner.
// (each wave adds the partials of some of the 2 n_iter sums, lane l taking
// partials l, l + 64, ... in order and a fixed butterfly combining the lanes;
// then thread 0 does the rest with the L-curve scratch in dynamic LDS)
template <typename T>
__global__ void __launch_bounds__(kLtNT) k_final(Args<T> a, sl_result out) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* scratch = reinterpret_cast<double*>(smem);
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  for (int j = wv; j < 2 * a.n_iter; j += kLtNT / kWave) {
    const int k = j >> 1;
    const bool ee = (j & 1) == 0;
    const double* p = part_of(a, ee ? P_EE : P_SS, k);
    const int n = ee ? a.nb_ee : a.nb_node;   // |e|^2 partials: per frequency column or per tile
    double v = 0.0;
    for (int i = lane; i < n; i += kWave) v += p[i];
    v = wave_sum(v);
    if (lane == 0) {
      if (ee)
        out.chi2[k] = v / (a.sigma * a.sigma);
      else
        out.reg[k] = v;
    }
  }
  __syncthreads();
  const bool invalid = a.flags[0] != 0;
  const bool empty = !invalid && !(a.gg[0] > 0.0);
  // the corner (every thread of the block takes part; the branch is uniform)
  const int kk = (!invalid && !empty && a.n_iter >= 4) ? lcurve_corner_block(out.reg, out.chi2, a.n_iter, scratch) : -1;
  if (threadIdx.x != 0) return;
  int cst = invalid ? SL_ST_INVALID : (empty ? SL_ST_EMPTY : SL_ST_OK);
  for (int k = 0; k < a.n_iter; ++k) {
    out.iters[k] = k + 1;
    const int st = invalid ? SL_ST_INVALID : (empty ? SL_ST_EMPTY : (a.upd[k] ? SL_ST_OK : SL_ST_BREAKDOWN));
    out.status[k] = st;
    if (cst == SL_ST_OK && st == SL_ST_BREAKDOWN) cst = SL_ST_BREAKDOWN;
  }
  int k = 0;
  if (!invalid && !empty) {
    if (a.n_iter >= 4) {
      if (kk >= 0)
        k = kk;
      else if (cst == SL_ST_OK)
        cst = SL_ST_LCURVE;
    } else if (a.n_iter > 1 && cst == SL_ST_OK) {
      cst = SL_ST_LCURVE;
    }
  }
  out.k_star[0] = k;
  out.corner_status[0] = cst;
  out.s_off[0] = 0;
  out.s_off[1] = a.I;
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_corner_copy(Args<T> a, sl_result out) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i >= a.I) return;
  const int k = out.k_star[0];
  out.s_corner[i] = (double)a.s_iter[(long)k * a.I + i];
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_zero_int(int32_t* p, long n) {
  const long i = (long)blockIdx.x * kNT + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- host side
struct Layout {
  int Nx, Ny, Nh, taps;
  long long cap;
  size_t total;
  size_t off[48];
};

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Region sizes in order; both the size query and the call use this.
static Layout make_layout(int nx, int ny, int nsub, int ns, int K, int interp, int n_iter, size_t sz,
                          bool solve) {
  Layout L{};
  const int ck = (K - 1) / 2;
  L.Nx = frame_side(nx, ck);
  L.Ny = frame_side(ny, ck);
  L.Nh = L.Nx / 2 + 1;
  L.taps = interp == SL_INTERP_BICUBIC ? 16 : 4;
  const long long J = (long long)nx * ny, n2 = (long long)nsub * nsub, I = (long long)ns * ns;
  L.cap = J * n2 * L.taps;
  const size_t c = 2 * sz;   // one complex element
  const int nb_row = (ny + 1) / 2;
  const int tiles = ((nx + kTV - 1) / kTV) * ((ny + kTVY - 1) / kTVY);
  // row blocks, column blocks, tiles, node blocks
  const int maxb = std::max(std::max(nb_row, L.Nh), std::max(tiles, kMaxParts));
  size_t sizes[48];
  int n = 0;
  sizes[n++] = c * L.Nx;                              // twx
  sizes[n++] = c * L.Ny;                              // twy
  sizes[n++] = 16 * (size_t)L.Nx;                     // twdx
  sizes[n++] = 16 * (size_t)L.Ny;                     // twdy
  sizes[n++] = c * (size_t)L.Nh * L.Ny;               // H
  sizes[n++] = c * (size_t)L.Nh * L.Ny;               // S
  sizes[n++] = 16 * (size_t)K * L.Nh;                 // T1
  if (solve) {
    sizes[n++] = (sz == 8 ? 24 : 12) * (size_t)(J * n2);   // sub
    sizes[n++] = 4 * (size_t)I;                       // cnt
    sizes[n++] = 4 * (size_t)((I + kTile - 1) / kTile);   // tsum
    sizes[n++] = 4 * (size_t)((I + kTile - 1) / kTile + 1);   // hsum
    sizes[n++] = 4 * (size_t)I;                       // heavy
    sizes[n++] = 4 * (size_t)(I + 1);                 // rowptr
    sizes[n++] = 4 * (size_t)I;                       // cursor
    sizes[n++] = 4 * (size_t)L.cap;                   // key
    sizes[n++] = sz * (size_t)L.cap;                  // wtmp
    sizes[n++] = (sz == 8 ? 16 : 8) * (size_t)L.cap;  // lt
    sizes[n++] = c * (size_t)L.Nh * L.Ny;             // E
    sizes[n++] = c * (size_t)L.Nh * L.Ny;             // SQ
    sizes[n++] = sz * (size_t)J;                      // w
    sizes[n++] = sz * (size_t)J;                      // y
    sizes[n++] = sz * (size_t)J;                      // q
    sizes[n++] = sz * (size_t)J;                      // e0
    sizes[n++] = sz * (size_t)J;                      // e1
    sizes[n++] = c * (size_t)kTH * kTNY;              // Ht
    sizes[n++] = c * (size_t)kTN;                     // twt
    sizes[n++] = c * (size_t)kTNY;                    // twc
    sizes[n++] = 16 * (size_t)K * kTH;                // T1t
    sizes[n++] = sz * (size_t)I;                      // s
    sizes[n++] = sz * (size_t)I;                      // p
    sizes[n++] = sz * (size_t)I;                      // g
    sizes[n++] = sz * (size_t)I * n_iter;             // s_iter
    sizes[n++] = 8 * (size_t)4 * (n_iter + 1) * maxb; // part
    sizes[n++] = 8 * (size_t)(n_iter + 1);            // gg
    sizes[n++] = 8 * (size_t)n_iter;                  // alpha
    sizes[n++] = 4 * (size_t)(n_iter + 1);            // done
    sizes[n++] = 4 * (size_t)n_iter;                  // upd
    sizes[n++] = 8;                                   // flags
  }
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    L.off[i] = off;
    off += align256(sizes[i]);
  }
  L.total = off;
  return L;
}

template <typename T>
static Args<T> bind(const Layout& L, unsigned char* ws, bool solve) {
  Args<T> a{};
  int i = 0;
  a.twx = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
  a.twy = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
  a.twdx = reinterpret_cast<cpx<double>*>(ws + L.off[i++]);
  a.twdy = reinterpret_cast<cpx<double>*>(ws + L.off[i++]);
  a.H = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
  a.S = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
  a.T1 = reinterpret_cast<cpx<double>*>(ws + L.off[i++]);
  if (solve) {
    a.sub = reinterpret_cast<Sub<T>*>(ws + L.off[i++]);
    a.cnt = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.tsum = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.hsum = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.heavy = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.rowptr = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.cursor = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.key = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.wtmp = reinterpret_cast<T*>(ws + L.off[i++]);
    a.lt = reinterpret_cast<LtE<T>*>(ws + L.off[i++]);
    a.E = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
    a.SQ = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
    a.w = reinterpret_cast<T*>(ws + L.off[i++]);
    a.y = reinterpret_cast<T*>(ws + L.off[i++]);
    a.q = reinterpret_cast<T*>(ws + L.off[i++]);
    a.e0 = reinterpret_cast<T*>(ws + L.off[i++]);
    a.e1 = reinterpret_cast<T*>(ws + L.off[i++]);
    a.Ht = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
    a.twt = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
    a.twc = reinterpret_cast<cpx<T>*>(ws + L.off[i++]);
    a.T1t = reinterpret_cast<cpx<double>*>(ws + L.off[i++]);
    a.s = reinterpret_cast<T*>(ws + L.off[i++]);
    a.p = reinterpret_cast<T*>(ws + L.off[i++]);
    a.g = reinterpret_cast<T*>(ws + L.off[i++]);
    a.s_iter = reinterpret_cast<T*>(ws + L.off[i++]);
    a.part = reinterpret_cast<double*>(ws + L.off[i++]);
    a.gg = reinterpret_cast<double*>(ws + L.off[i++]);
    a.alpha = reinterpret_cast<double*>(ws + L.off[i++]);
    a.done = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.upd = reinterpret_cast<int32_t*>(ws + L.off[i++]);
    a.flags = reinterpret_cast<int32_t*>(ws + L.off[i++]);
  }
  a.Nx = L.Nx;
  a.Ny = L.Ny;
  a.Nh = L.Nh;
  a.taps = L.taps;
  return a;
}

static inline unsigned nblk(long n, int nt) { return (unsigned)((n + nt - 1) / nt); }

template <typename T>
static int set_lds(size_t bytes) {
  const void* ks[] = {(const void*)k_rowfwd<T, ROW_LP>,       (const void*)k_rowfwd<T, ROW_D>,
                      (const void*)k_rowfwd<T, ROW_IMG>,      (const void*)k_col<T, false, COL_S>,
                      (const void*)k_col<T, true, COL_S>,     (const void*)k_col<T, true, COL_E>,
                      (const void*)k_col<T, true, COL_E_UPD>,
                      (const void*)k_rowinv<T, OUT_Q>,  (const void*)k_rowinv<T, OUT_W>,
                      (const void*)k_rowinv<T, OUT_IMG>};
  for (const void* k : ks) SL_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  SL_HIP(hipFuncSetAttribute((const void*)k_final<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(8 * kLcurveScratch)));
  return SL_OK;
}

// PSF spectrum and twiddles (every call).
template <typename T>
static int spectrum(const Args<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles<T>, dim3(nblk(a.Nx > a.Ny ? a.Nx : a.Ny, kNT)), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_psf_rows<T>, dim3(nblk((long)a.K * a.Nh, kNT)), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_psf_cols<T>, dim3(nblk((long)a.Nh * a.Ny, kNT)), dim3(kNT), 0, st, a);
  return check_launch("PSF spectrum");
}

// One blur of the image in flight: row pass (launched by the caller), column
// pass, inverse row pass.
template <typename T, bool CONJ, int COL, int OUT>
static void blur_tail(const Args<T>& a, T* dst, int it, hipStream_t st) {
  const size_t lx = 2 * sizeof(cpx<T>) * a.Nx, ly = 2 * sizeof(cpx<T>) * a.Ny;
  hipLaunchKernelGGL((k_col<T, CONJ, COL>), dim3(a.Nh), dim3(kNT), ly, st, a, it);
  hipLaunchKernelGGL((k_rowinv<T, OUT>), dim3(a.nb_row), dim3(kRowNT), lx, st, a, dst, it);
}

template <typename T>
static int fft_blur_impl(int transpose, int nx, int ny, const double* psf, int k, const void* in, void* out,
                         void* workspace, hipStream_t st) {
  const Layout L = make_layout(nx, ny, 1, 2, k, SL_INTERP_BILINEAR, 1, sizeof(T), false);
  Args<T> a = bind<T>(L, static_cast<unsigned char*>(workspace), false);
  a.nx = nx;
  a.ny = ny;
  a.K = k;
  a.ck = (k - 1) / 2;
  a.psf = psf;
  a.nb_row = (ny + 1) / 2;
  if (int e = set_lds<T>(2 * sizeof(cpx<T>) * (a.Nx > a.Ny ? a.Nx : a.Ny))) return e;
  if (int e = spectrum(a, st)) return e;
  hipLaunchKernelGGL((k_rowfwd<T, ROW_IMG>), dim3(a.nb_row), dim3(kRowNT), 2 * sizeof(cpx<T>) * a.Nx, st, a,
                     static_cast<const T*>(in));
  if (transpose)
    blur_tail<T, true, COL_S, OUT_IMG>(a, static_cast<T*>(out), 0, st);
  else
    blur_tail<T, false, COL_S, OUT_IMG>(a, static_cast<T*>(out), 0, st);
  return check_launch("fft blur");
}

template <typename T>
static int solve_impl(const sl_problem* pb, const double* lens, int ns, int n_iter, void* workspace,
                      sl_result* out, hipStream_t st) {
  const sl_image_grid& g = pb->img;
  const Layout L = make_layout(g.nx, g.ny, g.nsub, ns, pb->k, pb->interp, n_iter, sizeof(T), true);
  Args<T> a = bind<T>(L, static_cast<unsigned char*>(workspace), true);
  a.nx = g.nx;
  a.ny = g.ny;
  a.nsub = g.nsub;
  a.n2 = g.nsub * g.nsub;
  a.ns = ns;
  a.I = ns * ns;
  a.J = g.nx * g.ny;
  a.K = pb->k;
  a.ck = (pb->k - 1) / 2;
  a.interp = pb->interp;
  a.pix = g.pix;
  a.R = pb->half_width;
  a.sigma = pb->sigma;
  a.lens = lens;
  a.d = pb->d;
  a.psf = pb->psf;
  a.n_iter = n_iter;
  a.nb_row = (g.ny + 1) / 2;
  a.nb_node = (int)std::min<long>(nblk(a.I, kNodeNT), kMaxParts);
  a.nb_heavy = sizeof(T) == 4 ? kLtHeavyBlocks : 0;
  a.nb_lt = (int)std::min<long>(nblk((long)a.I * lt_lanes<T>(), (long)kLtNT * lt_groups<T>()), kMaxParts - a.nb_heavy) +
            a.nb_heavy;
  // FP32 with a PSF no wider than the tile's halo: the tiled blur (k_tile)
  a.tiles_x = (a.nx + kTV - 1) / kTV;
  a.tiles_y = (a.ny + kTVY - 1) / kTVY;
  const int ntiles = a.tiles_x * a.tiles_y;
  a.tiled = sizeof(T) == 4 && a.ck <= kTHalo;
  a.nb_qq = a.tiled ? ntiles : a.nb_row;
  a.nb_ee = a.tiled ? ntiles : a.Nh;
  a.max_blocks = std::max(std::max(std::max(a.nb_row, a.Nh), ntiles), std::max(a.nb_node, a.nb_lt));
  const size_t lx = 2 * sizeof(cpx<T>) * a.Nx;
  const size_t lt = 2 * sizeof(cpx<T>) * (size_t)kTBuf;
  if (int e = set_lds<T>(2 * sizeof(cpx<T>) * (a.Nx > a.Ny ? a.Nx : a.Ny))) return e;
  if constexpr (sizeof(T) == 4) {
    const void* kt[] = {(const void*)k_tile<T, TILE_B>, (const void*)k_tile<T, TILE_BT0>,
                        (const void*)k_tile<T, TILE_BT>};
    for (const void* k : kt) SL_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lt));
  }
  // counters start at zero (a fill kernel: the call may be captured in a graph)
  hipLaunchKernelGGL(k_zero_int<T>, dim3(nblk(a.I, kNT)), dim3(kNT), 0, st, a.cnt, (long)a.I);
  hipLaunchKernelGGL(k_zero_int<T>, dim3(1), dim3(kNT), 0, st, a.flags, 2L);
  if (a.tiled) {
    hipLaunchKernelGGL(k_tile_psf_rows<T>, dim3(nblk(std::max(a.K * kTH, kTN), kNT)), dim3(kNT), 0, st, a);
    hipLaunchKernelGGL(k_tile_psf_cols<T>, dim3(nblk(kTH * kTNY, kNT)), dim3(kNT), 0, st, a);
    if (int e = check_launch("tile PSF spectrum")) return e;
  } else if (int e = spectrum(a, st)) {
    return e;
  }
  const long nsubpix = (long)a.J * a.n2;
  hipLaunchKernelGGL(k_trace<T>, dim3(nblk(nsubpix, kNT)), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_count<T>, dim3(nblk(a.J, kNT)), dim3(kNT), 0, st, a);
  const unsigned tiles = nblk(a.I, kTile);
  hipLaunchKernelGGL(k_tile_sums<T>, dim3(tiles), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_tile_write<T>, dim3(tiles), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_fill<T>, dim3(nblk(a.J, kNT)), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_sort<T>, dim3(nblk(a.I, kNT)), dim3(kNT), 0, st, a);
  hipLaunchKernelGGL(k_sort_long<T>, dim3(kSortLongBlocks), dim3(kNT), 0, st, a);
  if (int e = check_launch("large solve set-up")) return e;
  if constexpr (sizeof(T) == 4) {
    if (a.tiled) {
      // g = A^T d, p = g; then per iteration y = L p, q = B y, e -= alpha q with w = B^T e, g = L^T w, s and p
      hipLaunchKernelGGL(k_copy_d<T>, dim3(nblk(a.J, kNT)), dim3(kNT), 0, st, a);
      hipLaunchKernelGGL((k_tile<T, TILE_BT0>), dim3(ntiles), dim3(kTNT), lt, st, a, (const T*)a.e0, (T*)nullptr, 0);
      hipLaunchKernelGGL(k_lt<T>, dim3(a.nb_lt), dim3(kLtNT), 0, st, a, n_iter);
      hipLaunchKernelGGL(k_start<T>, dim3(a.nb_node), dim3(kNodeNT), 0, st, a);
      for (int it = 0; it < n_iter; ++it) {
        T* ein = (it & 1) ? a.e1 : a.e0;
        T* eout = (it & 1) ? a.e0 : a.e1;
        hipLaunchKernelGGL(k_gather<T>, dim3(nblk(a.J, kNT)), dim3(kNT), 0, st, a);
        hipLaunchKernelGGL((k_tile<T, TILE_B>), dim3(ntiles), dim3(kTNT), lt, st, a, (const T*)nullptr, (T*)nullptr,
                           it);
        hipLaunchKernelGGL((k_tile<T, TILE_BT>), dim3(ntiles), dim3(kTNT), lt, st, a, (const T*)ein, eout, it);
        hipLaunchKernelGGL(k_lt<T>, dim3(a.nb_lt), dim3(kLtNT), 0, st, a, it);
        hipLaunchKernelGGL(k_update<T>, dim3(a.nb_node), dim3(kNodeNT), 0, st, a, it);
      }
      if (int e = check_launch("large solve iterations (tiled blur)")) return e;
      hipLaunchKernelGGL(k_final<T>, dim3(1), dim3(kLtNT), 8 * kLcurveScratch, st, a, *out);
      hipLaunchKernelGGL(k_corner_copy<T>, dim3(nblk(a.I, kNT)), dim3(kNT), 0, st, a, *out);
      return check_launch("large solve corner");
    }
  }
  // g = A^T d, p = g
  hipLaunchKernelGGL((k_rowfwd<T, ROW_D>), dim3(a.nb_row), dim3(kRowNT), lx, st, a, (const T*)nullptr);
  blur_tail<T, true, COL_E, OUT_W>(a, nullptr, 0, st);
  hipLaunchKernelGGL(k_lt<T>, dim3(a.nb_lt), dim3(kLtNT), 0, st, a, n_iter);
  hipLaunchKernelGGL(k_start<T>, dim3(a.nb_node), dim3(kNodeNT), 0, st, a);
  for (int it = 0; it < n_iter; ++it) {
    hipLaunchKernelGGL((k_rowfwd<T, ROW_LP>), dim3(a.nb_row), dim3(kRowNT), lx, st, a, (const T*)a.p);
    blur_tail<T, false, COL_S, OUT_Q>(a, nullptr, it, st);               // spectra of q = A p, |q|^2
    blur_tail<T, true, COL_E_UPD, OUT_W>(a, nullptr, it, st);            // e -= alpha q, |e|^2; w = B^T e
    hipLaunchKernelGGL(k_lt<T>, dim3(a.nb_lt), dim3(kLtNT), 0, st, a, it);
    hipLaunchKernelGGL(k_update<T>, dim3(a.nb_node), dim3(kNodeNT), 0, st, a, it);
  }
  if (int e = check_launch("large solve iterations")) return e;
  hipLaunchKernelGGL(k_final<T>, dim3(1), dim3(kLtNT), 8 * kLcurveScratch, st, a, *out);
  hipLaunchKernelGGL(k_corner_copy<T>, dim3(nblk(a.I, kNT)), dim3(kNT), 0, st, a, *out);
  return check_launch("large solve corner");
}

static int check_large(const sl_problem* pb, int ns, int n_iter) {
  SL_REQUIRE(pb != nullptr, "problem is NULL");
  const sl_image_grid& g = pb->img;
  SL_REQUIRE(g.nx >= 1 && g.ny >= 1 && g.nx <= kMaxImage && g.ny <= kMaxImage,
             "large solve supports images up to %d x %d (got %d x %d)", kMaxImage, kMaxImage, g.nx, g.ny);
  SL_REQUIRE(std::isfinite(g.pix) && g.pix > 0.0, "pixel size must be positive");
  SL_REQUIRE(g.nsub >= 1 && g.nsub <= SL_MAX_NSUB, "nsub %d outside [1, %d]", g.nsub, SL_MAX_NSUB);
  SL_REQUIRE(pb->k >= 1 && pb->k <= kMaxPsf && (pb->k & 1), "PSF side %d must be odd, <= %d", pb->k, kMaxPsf);
  SL_REQUIRE(std::isfinite(pb->sigma) && pb->sigma > 0.0, "sigma must be positive");
  SL_REQUIRE(std::isfinite(pb->half_width) && pb->half_width > 0.0, "half_width must be positive");
  SL_REQUIRE(pb->dtype == SL_F32 || pb->dtype == SL_F64, "unknown dtype %d", pb->dtype);
  SL_REQUIRE(pb->interp == SL_INTERP_BILINEAR || pb->interp == SL_INTERP_NEAREST || pb->interp == SL_INTERP_BICUBIC,
             "unknown interp %d", pb->interp);
  SL_REQUIRE(ns >= 2 && ns <= kMaxNs, "ns %d outside [2, %d]", ns, kMaxNs);
  SL_REQUIRE(n_iter >= 1 && n_iter <= SL_MAX_LAMBDA, "n_iter %d outside [1, %d]", n_iter, SL_MAX_LAMBDA);
  const int ck = (pb->k - 1) / 2;
  SL_REQUIRE(frame_side(g.nx, ck) <= kMaxFrame && frame_side(g.ny, ck) <= kMaxFrame,
             "FFT frame above %d for this image and PSF", kMaxFrame);
  const long long entries = (long long)g.nx * g.ny * g.nsub * g.nsub * (pb->interp == SL_INTERP_BICUBIC ? 16 : 4);
  SL_REQUIRE(entries < (1LL << 31), "too many L^T entries (%lld)", entries);
  return SL_OK;
}

static int check_blur(int dtype, int nx, int ny, int k) {
  SL_REQUIRE(dtype == SL_F32 || dtype == SL_F64, "unknown dtype %d", dtype);
  SL_REQUIRE(nx >= 1 && ny >= 1 && nx <= kMaxImage && ny <= kMaxImage, "image %d x %d outside [1, %d]", nx, ny,
             kMaxImage);
  SL_REQUIRE(k >= 1 && k <= kMaxPsf && (k & 1), "PSF side %d must be odd, <= %d", k, kMaxPsf);
  const int ck = (k - 1) / 2;
  SL_REQUIRE(frame_side(nx, ck) <= kMaxFrame && frame_side(ny, ck) <= kMaxFrame, "FFT frame above %d", kMaxFrame);
  return SL_OK;
}

}  // namespace large
}  // namespace sl

using namespace sl;
using namespace sl::large;

extern "C" {

size_t sl_fft_blur_workspace_size(int dtype, int nx, int ny, int k) {
  if (check_blur(dtype, nx, ny, k) != SL_OK) return 0;
  return make_layout(nx, ny, 1, 2, k, SL_INTERP_BILINEAR, 1, dtype == SL_F64 ? 8 : 4, false).total;
}

int sl_fft_blur(int dtype, int transpose, int nx, int ny, const double* psf, int k, const void* in, void* out,
                void* workspace, size_t workspace_bytes, void* stream) {
  if (int e = check_blur(dtype, nx, ny, k)) return e;
  SL_REQUIRE(transpose == 0 || transpose == 1, "transpose must be 0 or 1");
  SL_REQUIRE(psf && in && out && in != out, "bad device pointers");
  SL_REQUIRE(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
             "workspace must be non-NULL and 256-byte aligned");
  const size_t need = sl_fft_blur_workspace_size(dtype, nx, ny, k);
  SL_REQUIRE(workspace_bytes >= need, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  if (dtype == SL_F32) return fft_blur_impl<float>(transpose, nx, ny, psf, k, in, out, workspace, st);
  return fft_blur_impl<double>(transpose, nx, ny, psf, k, in, out, workspace, st);
}

size_t sl_solve_large_workspace_size(const sl_problem* pb, int ns, int n_iter) {
  if (check_large(pb, ns, n_iter) != SL_OK) return 0;
  const sl_image_grid& g = pb->img;
  return make_layout(g.nx, g.ny, g.nsub, ns, pb->k, pb->interp, n_iter, pb->dtype == SL_F64 ? 8 : 4, true).total;
}

int sl_solve_large(const sl_problem* pb, const double* lens, int ns, int n_iter, void* workspace,
                   size_t workspace_bytes, sl_result* out, void* stream) {
  if (int e = check_large(pb, ns, n_iter)) return e;
  SL_REQUIRE(lens && pb->d && pb->psf, "NULL device pointer");
  SL_REQUIRE(out && out->s_corner && out->s_off && out->chi2 && out->reg && out->iters && out->status &&
                 out->k_star && out->corner_status,
             "NULL result pointer");
  SL_REQUIRE(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
             "workspace must be non-NULL and 256-byte aligned");
  const size_t need = sl_solve_large_workspace_size(pb, ns, n_iter);
  SL_REQUIRE(workspace_bytes >= need, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  if (pb->dtype == SL_F32) return solve_impl<float>(pb, lens, ns, n_iter, workspace, out, st);
  return solve_impl<double>(pb, lens, ns, n_iter, workspace, out, st);
}

}  // extern "C"
