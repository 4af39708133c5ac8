// Operator-level entry points: lens tracing, L, L^T, B, B^T and H^T H.
//
// These are the building blocks of the semilinear model (Rogers & Fiege 2011,
// Sec. 2.1-2.2, Eq. 7) exposed one call per operator.  The batched solver in
// solve.hip fuses the same operators into one persistent kernel; the kernels
// here are straightforward one-thread-per-output launches over global memory,
// except B/B^T which stage input tiles and the PSF in LDS.
#include <algorithm>
#include <cstdarg>
#include <vector>

#include "common.h"

namespace sl {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

// ------------------------------------------------------------------ trace
__global__ void k_trace(const double* __restrict__ genome, int nx, int ny, double pix, int nsub,
                        int ns, double R, double* __restrict__ uv) {
  const int n2 = nsub * nsub;
  const long total = (long)nx * ny * n2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  double g[7];
  for (int i = 0; i < 7; ++i) g[i] = genome[i];
  double u = NAN, v = NAN;
  if (lens_valid(g)) {
    const Lens L = make_lens(g);
    const int j = (int)(t / n2), k = (int)(t % n2);
    const int r = j / nx, c = j % nx;
    double x, y, bx, by;
    subpixel_xy(r, c, k / nsub, k % nsub, nx, ny, pix, nsub, x, y);
    lens_map(L, x, y, bx, by);
    const double h = 2.0 * R / (ns - 1);
    const double uu = (bx + R) / h, vv = (by + R) / h;
    if (uu >= 0.0 && uu <= ns - 1 && vv >= 0.0 && vv <= ns - 1) {
      u = uu;
      v = vv;
    }
  }
  uv[2 * t] = u;
  uv[2 * t + 1] = v;
}

// ------------------------------------------------------------------ L, L^T
template <typename T>
__global__ void k_apply_L(const double* __restrict__ uv, int J, int nsub, int ns,
                          const T* __restrict__ s, T* __restrict__ img) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const int n2 = nsub * nsub;
  T acc = 0;
  for (int k = 0; k < n2; ++k) {
    const long t = (long)j * n2 + k;
    int cell;
    double fx, fy;
    if (!grid_cell(uv[2 * t], uv[2 * t + 1], ns, cell, fx, fy)) continue;
    const T tx = (T)fx, ty = (T)fy;
    acc += (1 - tx) * (1 - ty) * s[cell] + tx * (1 - ty) * s[cell + 1] + (1 - tx) * ty * s[cell + ns] +
           tx * ty * s[cell + ns + 1];
  }
  img[j] = acc / (T)n2;
}

template <typename T>
__global__ void k_apply_LT(const double* __restrict__ uv, int J, int nsub, int ns,
                           const T* __restrict__ img, T* __restrict__ s) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const int n2 = nsub * nsub;
  const T val = img[j] / (T)n2;
  for (int k = 0; k < n2; ++k) {
    const long t = (long)j * n2 + k;
    int cell;
    double fx, fy;
    if (!grid_cell(uv[2 * t], uv[2 * t + 1], ns, cell, fx, fy)) continue;
    const T tx = (T)fx, ty = (T)fy;
    atomicAdd(&s[cell], (1 - tx) * (1 - ty) * val);
    atomicAdd(&s[cell + 1], tx * (1 - ty) * val);
    atomicAdd(&s[cell + ns], (1 - tx) * ty * val);
    atomicAdd(&s[cell + ns + 1], tx * ty * val);
  }
}

// Ordered L^T (fixed summation order).  A counting sort by node of the keys
// key = 4 t + corner (t = subpixel index j n^2 + k, corner 0..3 for the
// nodes cell, cell + 1, cell + ns, cell + ns + 1), then one thread per node
// sums its terms in ascending key order, i.e. by pixel, subpixel, corner:
// the order of a sequential scatter over the pixels.
__global__ void k_lt_count(const double* __restrict__ uv, long nsubpix, int ns, int* __restrict__ cnt) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsubpix) return;
  int cell;
  double fx, fy;
  if (!grid_cell(uv[2 * t], uv[2 * t + 1], ns, cell, fx, fy)) return;
  atomicAdd(&cnt[cell], 1);
  atomicAdd(&cnt[cell + 1], 1);
  atomicAdd(&cnt[cell + ns], 1);
  atomicAdd(&cnt[cell + ns + 1], 1);
}

// Exclusive scan of cnt[0..I) into ptr[0..I] and the fill cursors cur (one block).
__global__ void __launch_bounds__(1024) k_lt_scan(const int* __restrict__ cnt, int I, int* __restrict__ ptr,
                                                  int* __restrict__ cur) {
  __shared__ int wsum[16];
  __shared__ int carry;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int i0 = 0; i0 < I; i0 += 1024) {
    const int i = i0 + tid;
    const int v = i < I ? cnt[i] : 0;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o, 64);
      if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int before = carry;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    if (i < I) {
      ptr[i] = before + incl - v;
      cur[i] = before + incl - v;
    }
    __syncthreads();
    if (tid == 1023) carry = before + incl;
    __syncthreads();
  }
  if (tid == 0) ptr[I] = carry;
}

__global__ void k_lt_fill(const double* __restrict__ uv, long nsubpix, int ns, int* __restrict__ cur,
                          int* __restrict__ keys) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsubpix) return;
  int cell;
  double fx, fy;
  if (!grid_cell(uv[2 * t], uv[2 * t + 1], ns, cell, fx, fy)) return;
  const int nd[4] = {cell, cell + 1, cell + ns, cell + ns + 1};
#pragma unroll
  for (int q = 0; q < 4; ++q) keys[atomicAdd(&cur[nd[q]], 1)] = (int)(4 * t + q);
}

template <typename T>
__global__ void k_lt_gather(const double* __restrict__ uv, int n2, int ns, const int* __restrict__ ptr,
                            int* __restrict__ keys, const T* __restrict__ img, T* __restrict__ s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns * ns) return;
  const int e0 = ptr[i], e1 = ptr[i + 1];
  // insertion sort of this node's keys (the segment belongs to this thread)
  for (int e = e0 + 1; e < e1; ++e) {
    const int k = keys[e];
    int f = e - 1;
    while (f >= e0 && keys[f] > k) {
      keys[f + 1] = keys[f];
      --f;
    }
    keys[f + 1] = k;
  }
  T acc = 0;
  for (int e = e0; e < e1; ++e) {
    const int key = keys[e];
    const long t = key >> 2;
    const int q = key & 3;
    int cell;
    double fx, fy;
    grid_cell(uv[2 * t], uv[2 * t + 1], ns, cell, fx, fy);
    const T tx = (T)fx, ty = (T)fy;
    const T val = img[t / n2] / (T)n2;
    const T w = q == 0 ? (1 - tx) * (1 - ty) : q == 1 ? tx * (1 - ty) : q == 2 ? (1 - tx) * ty : tx * ty;
    acc += w * val;
  }
  s[i] = acc;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, long n, T v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ B, B^T
// One 16x16 output tile per block; the (16+K-1)^2 input tile and the PSF are
// staged in LDS.  TRANSPOSE=false: convolution, true: correlation.
constexpr int kTile = 16;

template <typename T, bool TRANSPOSE>
__global__ void k_blur(int nx, int ny, const double* __restrict__ psf, int K,
                       const T* __restrict__ in, T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* P = reinterpret_cast<T*>(smem);
  const int ck = (K - 1) / 2;
  const int tw = kTile + K - 1;
  T* tile = P + K * K;
  const long img_off = (long)blockIdx.z * nx * ny;
  const int R0 = blockIdx.y * kTile, C0 = blockIdx.x * kTile;
  const int tid = threadIdx.y * kTile + threadIdx.x;
  for (int i = tid; i < K * K; i += kTile * kTile) P[i] = (T)psf[i];
  for (int i = tid; i < tw * tw; i += kTile * kTile) {
    const int rr = R0 - ck + i / tw, cc = C0 - ck + i % tw;
    tile[i] = (rr >= 0 && rr < ny && cc >= 0 && cc < nx) ? in[img_off + (long)rr * nx + cc] : (T)0;
  }
  __syncthreads();
  const int r = R0 + threadIdx.y, c = C0 + threadIdx.x;
  if (r >= ny || c >= nx) return;
  T acc = 0;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      // convolution reads x[r-a+ck][c-b+ck]; correlation reads z[r+a-ck][c+b-ck]
      const int tr = TRANSPOSE ? threadIdx.y + a : threadIdx.y + 2 * ck - a;
      const int tc = TRANSPOSE ? threadIdx.x + b : threadIdx.x + 2 * ck - b;
      acc += P[a * K + b] * tile[tr * tw + tc];
    }
  out[img_off + (long)r * nx + c] = acc;
}

// ------------------------------------------------------------------ H^T H
template <typename T>
__device__ __forceinline__ T node_at(const T* s, int ns, int r, int c) {
  return (r < 0 || c < 0 || r >= ns || c >= ns) ? (T)0 : s[r * ns + c];
}
template <typename T>
__device__ __forceinline__ T d2x_at(const T* s, int ns, int r, int c) {
  if (r < 0 || c < 0 || r >= ns || c >= ns) return (T)0;
  return node_at(s, ns, r, c - 1) - 2 * node_at(s, ns, r, c) + node_at(s, ns, r, c + 1);
}
template <typename T>
__device__ __forceinline__ T d2y_at(const T* s, int ns, int r, int c) {
  if (r < 0 || c < 0 || r >= ns || c >= ns) return (T)0;
  return node_at(s, ns, r - 1, c) - 2 * node_at(s, ns, r, c) + node_at(s, ns, r + 1, c);
}

template <typename T>
__global__ void k_apply_HtH(int reg, int ns, const T* __restrict__ s, T* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns * ns) return;
  if (reg == SL_H_IDENTITY) {
    out[i] = s[i];
    return;
  }
  const int r = i / ns, c = i % ns;
  out[i] = d2x_at(s, ns, r, c - 1) - 2 * d2x_at(s, ns, r, c) + d2x_at(s, ns, r, c + 1) +
           d2y_at(s, ns, r - 1, c) - 2 * d2y_at(s, ns, r, c) + d2y_at(s, ns, r + 1, c);
}

// ------------------------------------------------------------------ host helpers
static int check_grid(const sl_image_grid* img) {
  SL_REQUIRE(img != nullptr, "image grid is NULL");
  SL_REQUIRE(img->nx >= 1 && img->ny >= 1 && (long)img->nx * img->ny <= (1L << 28),
             "image size %d x %d out of range", img->nx, img->ny);
  SL_REQUIRE(std::isfinite(img->pix) && img->pix > 0.0, "pixel size must be positive");
  SL_REQUIRE(img->nsub >= 1 && img->nsub <= SL_MAX_NSUB, "nsub %d outside [1, %d]", img->nsub,
             SL_MAX_NSUB);
  return SL_OK;
}

static int check_ns(const int32_t* ns, int n_members) {
  SL_REQUIRE(n_members >= 1, "n_members must be >= 1");
  SL_REQUIRE(ns != nullptr, "ns is NULL");
  for (int m = 0; m < n_members; ++m)
    SL_REQUIRE(ns[m] >= 2 && ns[m] <= 4096, "ns[%d] = %d outside [2, 4096]", m, ns[m]);
  return SL_OK;
}

static inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
static int apply_L_impl(const double* uv, int n_members, const sl_image_grid* img, const int32_t* ns,
                        const void* s, void* out, hipStream_t st) {
  const int J = img->nx * img->ny, n2 = img->nsub * img->nsub;
  long soff = 0;
  for (int m = 0; m < n_members; ++m) {
    hipLaunchKernelGGL(k_apply_L<T>, dim3(nblocks(J, 256)), dim3(256), 0, st,
                       uv + (long)m * J * n2 * 2, J, img->nsub, ns[m], (const T*)s + soff,
                       (T*)out + (long)m * J);
    soff += (long)ns[m] * ns[m];
  }
  return check_launch("k_apply_L");
}

template <typename T>
static int apply_LT_impl(const double* uv, int n_members, const sl_image_grid* img, const int32_t* ns,
                         const void* in, void* s, hipStream_t st) {
  const int J = img->nx * img->ny, n2 = img->nsub * img->nsub;
  long total = 0;
  for (int m = 0; m < n_members; ++m) total += (long)ns[m] * ns[m];
  hipLaunchKernelGGL(k_fill<T>, dim3(nblocks(total, 256)), dim3(256), 0, st, (T*)s, total, (T)0);
  long soff = 0;
  for (int m = 0; m < n_members; ++m) {
    hipLaunchKernelGGL(k_apply_LT<T>, dim3(nblocks(J, 256)), dim3(256), 0, st,
                       uv + (long)m * J * n2 * 2, J, img->nsub, ns[m], (const T*)in + (long)m * J,
                       (T*)s + soff);
    soff += (long)ns[m] * ns[m];
  }
  return check_launch("k_apply_LT");
}

// Workspace of the ordered L^T: per member (I + 1) + I ints of row starts and
// cursors and 4 J n^2 keys; members are processed one after another, so
// the largest member sets the size.
static size_t lt_ordered_ws(const sl_image_grid* img, const int32_t* ns, int n_members) {
  long I = 0;
  for (int m = 0; m < n_members; ++m) I = std::max(I, (long)ns[m] * ns[m]);
  const long keys = 4L * img->nx * img->ny * img->nsub * img->nsub;
  return sizeof(int) * (size_t)(2 * I + 1 + I + keys);
}

template <typename T>
static int apply_LT_ordered_impl(const double* uv, int n_members, const sl_image_grid* img, const int32_t* ns,
                                 const void* in, void* s, void* ws, hipStream_t st) {
  const int J = img->nx * img->ny, n2 = img->nsub * img->nsub;
  const long nsp = (long)J * n2;
  long I_max = 0;
  for (int m = 0; m < n_members; ++m) I_max = std::max(I_max, (long)ns[m] * ns[m]);
  int* cnt = (int*)ws;
  int* ptr = cnt + I_max;
  int* cur = ptr + I_max + 1;
  int* keys = cur + I_max;
  long soff = 0;
  for (int m = 0; m < n_members; ++m) {
    const int I = ns[m] * ns[m];
    const double* uvm = uv + (long)m * nsp * 2;
    hipLaunchKernelGGL(k_fill<int>, dim3(nblocks(I, 256)), dim3(256), 0, st, cnt, (long)I, 0);
    hipLaunchKernelGGL(k_lt_count, dim3(nblocks(nsp, 256)), dim3(256), 0, st, uvm, nsp, ns[m], cnt);
    hipLaunchKernelGGL(k_lt_scan, dim3(1), dim3(1024), 0, st, cnt, I, ptr, cur);
    hipLaunchKernelGGL(k_lt_fill, dim3(nblocks(nsp, 256)), dim3(256), 0, st, uvm, nsp, ns[m], cur, keys);
    hipLaunchKernelGGL(k_lt_gather<T>, dim3(nblocks(I, 256)), dim3(256), 0, st, uvm, n2, ns[m], ptr, keys,
                       (const T*)in + (long)m * J, (T*)s + soff);
    if (int e = check_launch("ordered L^T")) return e;
    soff += I;
  }
  return SL_OK;
}

template <typename T, bool TR>
static int blur_impl(int nx, int ny, int n_images, const double* psf, int k, const void* in, void* out,
                     hipStream_t st) {
  const int tw = kTile + k - 1;
  const size_t lds = sizeof(T) * ((size_t)k * k + (size_t)tw * tw);
  hipLaunchKernelGGL((k_blur<T, TR>), dim3(nblocks(nx, kTile), nblocks(ny, kTile), n_images),
                     dim3(kTile, kTile), lds, st, nx, ny, psf, k, (const T*)in, (T*)out);
  return check_launch("k_blur");
}

}  // namespace sl

using namespace sl;

extern "C" {

const char* sl_last_error(void) { return g_err; }

const char* sl_version(void) { return "semilin 0.1 (gfx950)"; }

int sl_lens_trace(const double* lens, int n_members, const sl_image_grid* img, const int32_t* ns,
                  double half_width, double* uv, void* stream) {
  if (int e = check_grid(img)) return e;
  if (int e = check_ns(ns, n_members)) return e;
  SL_REQUIRE(lens && uv, "NULL device pointer");
  SL_REQUIRE(std::isfinite(half_width) && half_width > 0.0, "half_width must be positive");
  hipStream_t st = (hipStream_t)stream;
  const long per = (long)img->nx * img->ny * img->nsub * img->nsub;
  for (int m = 0; m < n_members; ++m)
    hipLaunchKernelGGL(k_trace, dim3(nblocks(per, 256)), dim3(256), 0, st, lens + 7L * m, img->nx,
                       img->ny, img->pix, img->nsub, ns[m], half_width, uv + 2 * per * m);
  return check_launch("k_trace");
}

int sl_apply_L(int dtype, const double* uv, int n_members, const sl_image_grid* img, const int32_t* ns,
               const void* s, void* img_out, void* stream) {
  if (int e = check_grid(img)) return e;
  if (int e = check_ns(ns, n_members)) return e;
  SL_REQUIRE(uv && s && img_out, "NULL device pointer");
  if (dtype == SL_F32) return apply_L_impl<float>(uv, n_members, img, ns, s, img_out, (hipStream_t)stream);
  if (dtype == SL_F64) return apply_L_impl<double>(uv, n_members, img, ns, s, img_out, (hipStream_t)stream);
  SL_REQUIRE(false, "unknown dtype %d", dtype);
}

int sl_apply_LT(int dtype, const double* uv, int n_members, const sl_image_grid* img, const int32_t* ns,
                const void* img_in, void* s_out, void* stream) {
  if (int e = check_grid(img)) return e;
  if (int e = check_ns(ns, n_members)) return e;
  SL_REQUIRE(uv && img_in && s_out, "NULL device pointer");
  if (dtype == SL_F32)
    return apply_LT_impl<float>(uv, n_members, img, ns, img_in, s_out, (hipStream_t)stream);
  if (dtype == SL_F64)
    return apply_LT_impl<double>(uv, n_members, img, ns, img_in, s_out, (hipStream_t)stream);
  SL_REQUIRE(false, "unknown dtype %d", dtype);
}

size_t sl_apply_LT_ordered_workspace_size(const sl_image_grid* img, const int32_t* ns, int n_members) {
  if (check_grid(img) != SL_OK || check_ns(ns, n_members) != SL_OK) return 0;
  return lt_ordered_ws(img, ns, n_members);
}

int sl_apply_LT_ordered(int dtype, const double* uv, int n_members, const sl_image_grid* img, const int32_t* ns,
                        const void* img_in, void* s_out, void* workspace, size_t workspace_bytes, void* stream) {
  if (int e = check_grid(img)) return e;
  if (int e = check_ns(ns, n_members)) return e;
  SL_REQUIRE(uv && img_in && s_out && workspace, "NULL device pointer");
  SL_REQUIRE(((uintptr_t)workspace & 3) == 0, "workspace must be 4-byte aligned");
  SL_REQUIRE(4L * img->nx * img->ny * img->nsub * img->nsub < (1L << 31), "image too large for 32-bit keys");
  const size_t need = lt_ordered_ws(img, ns, n_members);
  SL_REQUIRE(workspace_bytes >= need, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  if (dtype == SL_F32)
    return apply_LT_ordered_impl<float>(uv, n_members, img, ns, img_in, s_out, workspace, (hipStream_t)stream);
  if (dtype == SL_F64)
    return apply_LT_ordered_impl<double>(uv, n_members, img, ns, img_in, s_out, workspace, (hipStream_t)stream);
  SL_REQUIRE(false, "unknown dtype %d", dtype);
}

static int blur_args(int nx, int ny, int n_images, const double* psf, int k, const void* in, void* out) {
  SL_REQUIRE(nx >= 1 && ny >= 1 && n_images >= 1, "bad image sizes");
  SL_REQUIRE(k >= 1 && k <= SL_MAX_PSF && (k & 1), "PSF side %d must be odd and <= %d", k, SL_MAX_PSF);
  SL_REQUIRE(psf && in && out, "NULL device pointer");
  SL_REQUIRE(in != out, "in and out must differ");
  return SL_OK;
}

int sl_apply_B(int dtype, int nx, int ny, int n_images, const double* psf, int k, const void* in,
               void* out, void* stream) {
  if (int e = blur_args(nx, ny, n_images, psf, k, in, out)) return e;
  if (dtype == SL_F32) return blur_impl<float, false>(nx, ny, n_images, psf, k, in, out, (hipStream_t)stream);
  if (dtype == SL_F64) return blur_impl<double, false>(nx, ny, n_images, psf, k, in, out, (hipStream_t)stream);
  SL_REQUIRE(false, "unknown dtype %d", dtype);
}

int sl_apply_BT(int dtype, int nx, int ny, int n_images, const double* psf, int k, const void* in,
                void* out, void* stream) {
  if (int e = blur_args(nx, ny, n_images, psf, k, in, out)) return e;
  if (dtype == SL_F32) return blur_impl<float, true>(nx, ny, n_images, psf, k, in, out, (hipStream_t)stream);
  if (dtype == SL_F64) return blur_impl<double, true>(nx, ny, n_images, psf, k, in, out, (hipStream_t)stream);
  SL_REQUIRE(false, "unknown dtype %d", dtype);
}

int sl_apply_HtH(int dtype, int reg, int n_members, const int32_t* ns, const void* s, void* out,
                 void* stream) {
  if (int e = check_ns(ns, n_members)) return e;
  SL_REQUIRE(reg == SL_H_IDENTITY || reg == SL_H_CURVATURE, "unknown reg %d", reg);
  SL_REQUIRE(s && out && s != out, "bad device pointers");
  hipStream_t st = (hipStream_t)stream;
  long off = 0;
  for (int m = 0; m < n_members; ++m) {
    const int I = ns[m] * ns[m];
    if (dtype == SL_F32)
      hipLaunchKernelGGL(k_apply_HtH<float>, dim3(nblocks(I, 256)), dim3(256), 0, st, reg, ns[m],
                         (const float*)s + off, (float*)out + off);
    else if (dtype == SL_F64)
      hipLaunchKernelGGL(k_apply_HtH<double>, dim3(nblocks(I, 256)), dim3(256), 0, st, reg, ns[m],
                         (const double*)s + off, (double*)out + off);
    else
      SL_REQUIRE(false, "unknown dtype %d", dtype);
    off += I;
  }
  return check_launch("k_apply_HtH");
}

int sl_lcurve_corner(const double* reg, const double* chi2, int n, int32_t* k_star, double* kappa) {
  SL_REQUIRE(reg && chi2 && k_star, "NULL host pointer");
  SL_REQUIRE(n >= 4 && n <= SL_MAX_LAMBDA, "L-curve needs 4..%d points, got %d", SL_MAX_LAMBDA, n);
  std::vector<double> scratch(kLcurveScratch);
  const int k = lcurve_corner_impl(reg, chi2, n, kappa, scratch.data());
  SL_REQUIRE(k >= 0, "degenerate L-curve (non-positive values or fewer than 4 distinct points)");
  *k_star = k;
  return SL_OK;
}

}  // extern "C"
