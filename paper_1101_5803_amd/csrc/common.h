// Shared device/host helpers of the semilinear lens library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "semilin.h"

namespace sl {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);

#define SL_REQUIRE(cond, ...)            \
  do {                                   \
    if (!(cond)) {                       \
      ::sl::set_error(__VA_ARGS__);      \
      return SL_EINVAL;                  \
    }                                    \
  } while (0)

#define SL_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::sl::set_error("%s failed: %s", #call, hipGetErrorString(e_));             \
      return SL_EHIP;                                                             \
    }                                                                             \
  } while (0)

inline int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("launch of %s failed: %s", what, hipGetErrorString(e));
    return SL_EHIP;
  }
  return SL_OK;
}

constexpr int kWave = 64;

// ---------------------------------------------------------------- reductions
template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide FP64 sum; `scratch` holds >= blockDim.x/64 doubles of LDS.
// All threads receive the total.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += scratch[i];   // same order in every thread
  __syncthreads();
  return t;
}

// Block-wide sums of two FP64 values at once (one pair of barriers).
__device__ __forceinline__ void block_sum2(double& a, double& b, double* scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    scratch[2 * wid] = a;
    scratch[2 * wid + 1] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  for (int i = 0; i < nw; ++i) {
    ta += scratch[2 * i];
    tb += scratch[2 * i + 1];
  }
  __syncthreads();
  a = ta;
  b = tb;
}

// ---------------------------------------------------------------- lens
// Genome layout (theta_E, q, pa, gamma, gamma_pa, x0, y0).
struct Lens {
  double b, q, cp, sp, k, g1, g2, x0, y0;
};

__host__ __device__ inline bool lens_valid(const double* g) {
  for (int i = 0; i < 7; ++i)
    if (!__builtin_isfinite(g[i])) return false;
  return g[0] >= 0.0 && g[1] > 0.0 && g[1] <= 1.0;
}

__host__ __device__ inline Lens make_lens(const double* g) {
  Lens L;
  L.b = g[0];
  L.q = g[1];
  L.cp = cos(g[2]);
  L.sp = sin(g[2]);
  L.k = sqrt(fmax(0.0, 1.0 - g[1] * g[1]));
  L.g1 = g[3] * cos(2.0 * g[4]);
  L.g2 = g[3] * sin(2.0 * g[4]);
  L.x0 = g[5];
  L.y0 = g[6];
  return L;
}

// beta = theta - alpha_SIE(theta) - alpha_shear(theta) in FP64
// (thin-lens mapping, Eq. 1; SIE with core s = 0, Eqs. 10-11).
__host__ __device__ inline void lens_map(const Lens& L, double x, double y, double& bx, double& by) {
  const double dx = x - L.x0, dy = y - L.y0;
  const double xp = L.cp * dx + L.sp * dy;
  const double yp = -L.sp * dx + L.cp * dy;
  const double psi = sqrt(L.q * L.q * xp * xp + yp * yp);
  double axp = 0.0, ayp = 0.0;
  if (psi > 0.0) {
    if (L.k < 1e-4) {  // SIS limit: alpha' = b q (x', y') / psi
      axp = L.b * L.q * xp / psi;
      ayp = L.b * L.q * yp / psi;
    } else {
      const double f = L.b * L.q / L.k;
      axp = f * atan(L.k * xp / psi);
      ayp = f * atanh(L.k * yp / psi);
    }
  }
  const double ax = L.cp * axp - L.sp * ayp;
  const double ay = L.sp * axp + L.cp * ayp;
  bx = x - ax - (L.g1 * dx + L.g2 * dy);
  by = y - ay - (L.g2 * dx - L.g1 * dy);
}

// Subpixel position of pixel (r, c), subpixel (sr, sc).
__host__ __device__ inline void subpixel_xy(int r, int c, int sr, int sc, int nx, int ny, double pix,
                                            int nsub, double& x, double& y) {
  x = (c - 0.5 * (nx - 1)) * pix + ((sc + 0.5) / nsub - 0.5) * pix;
  y = (r - 0.5 * (ny - 1)) * pix + ((sr + 0.5) / nsub - 0.5) * pix;
}

// Grid cell and fractional offsets; returns false when outside the grid.
__host__ __device__ inline bool grid_cell(double u, double v, int ns, int& cell, double& fx,
                                          double& fy) {
  if (!(u >= 0.0 && u <= ns - 1 && v >= 0.0 && v <= ns - 1)) return false;
  int c0 = (int)floor(u), r0 = (int)floor(v);
  if (c0 > ns - 2) c0 = ns - 2;
  if (r0 > ns - 2) r0 = ns - 2;
  cell = r0 * ns + c0;
  fx = u - c0;
  fy = v - r0;
  return true;
}

// ---------------------------------------------------------------- L-curve (FP64)
// Not-a-knot cubic spline first/second derivatives at the knots; solves the
// n x n moment system by Gaussian elimination with partial pivoting.
// A: n*n scratch, rhs: n scratch.  Returns false on a singular system.
// The system is banded (at most two entries below and two above the
// diagonal: the two not-a-knot rows), so with partial pivoting the factors
// keep at most two entries below and four above it; the loops visit only
// those, and every entry they skip is an exact zero (the result is that of
// the full elimination).
// Row i of the system (A zeroed and M[0] = M[n - 1] = 0 beforehand): the
// not-a-knot rows 0 and n - 1, the continuity rows between.
__host__ __device__ inline void spline_fill_row(const double* t, const double* y, int n, double* A, double* M, int i) {
  if (i == 0) {
    const double h0 = t[1] - t[0], h1 = t[2] - t[1];
    A[0] = h1;
    A[1] = -(h0 + h1);
    A[2] = h0;
  } else if (i == n - 1) {
    const double ha = t[n - 2] - t[n - 3], hb = t[n - 1] - t[n - 2];
    A[(n - 1) * n + n - 3] = hb;
    A[(n - 1) * n + n - 2] = -(ha + hb);
    A[(n - 1) * n + n - 1] = ha;
  } else {
    const double hm = t[i] - t[i - 1], hp = t[i + 1] - t[i];
    A[i * n + i - 1] = hm;
    A[i * n + i] = 2.0 * (hm + hp);
    A[i * n + i + 1] = hp;
    M[i] = 6.0 * ((y[i + 1] - y[i]) / hp - (y[i] - y[i - 1]) / hm);
  }
}

// Gaussian elimination with partial pivoting and back substitution: M holds
// the second derivatives on return; false on a zero pivot.
__host__ __device__ inline bool spline_solve(int n, double* A, double* M) {
  for (int col = 0; col < n; ++col) {
    const int rlast = col + 2 < n - 1 ? col + 2 : n - 1;
    const int clast = col + 4 < n - 1 ? col + 4 : n - 1;
    int piv = col;
    for (int r = col + 1; r <= rlast; ++r)
      if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
    if (A[piv * n + col] == 0.0) return false;
    if (piv != col) {
      for (int c = col; c <= clast; ++c) {
        const double tmp = A[col * n + c];
        A[col * n + c] = A[piv * n + c];
        A[piv * n + c] = tmp;
      }
      const double tmp = M[col];
      M[col] = M[piv];
      M[piv] = tmp;
    }
    for (int r = col + 1; r <= rlast; ++r) {
      if (A[r * n + col] == 0.0) continue;   // the quotient would be 0 (the pivot is not)
      const double f = A[r * n + col] / A[col * n + col];
      for (int c = col; c <= clast; ++c) A[r * n + c] -= f * A[col * n + c];
      M[r] -= f * M[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double acc = M[r];
    const int clast = r + 4 < n - 1 ? r + 4 : n - 1;
    for (int c = r + 1; c <= clast; ++c) acc -= A[r * n + c] * M[c];
    M[r] = acc / A[r * n + r];
  }
  return true;
}

// First derivative at knot i from the second derivatives M.
__host__ __device__ inline double spline_d1_at(const double* t, const double* y, int n, const double* M, int i) {
  if (i < n - 1) {
    const double h = t[i + 1] - t[i];
    return (y[i + 1] - y[i]) / h - h * (2.0 * M[i] + M[i + 1]) / 6.0;
  }
  const double h = t[n - 1] - t[n - 2];
  return (y[n - 1] - y[n - 2]) / h + h * (M[n - 2] + 2.0 * M[n - 1]) / 6.0;
}

__host__ __device__ inline bool spline_knot_derivs(const double* t, const double* y, int n, double* A,
                                                   double* M, double* d1) {
  for (int i = 0; i < n * n; ++i) A[i] = 0.0;
  for (int i = 0; i < n; ++i) M[i] = 0.0;
  for (int i = 0; i < n; ++i) spline_fill_row(t, y, n, A, M, i);
  if (!spline_solve(n, A, M)) return false;
  for (int i = 0; i < n; ++i) d1[i] = spline_d1_at(t, y, n, M, i);
  return true;
}

// L-curve corner; scratch needs 2*SL_MAX_LAMBDA^2 + 10*SL_MAX_LAMBDA doubles.
// Returns k* >= 0, or -1 when the curve is degenerate.
__host__ __device__ inline int lcurve_corner_impl(const double* reg, const double* chi2, int n,
                                                  double* kappa_out, double* scratch) {
  if (kappa_out)
    for (int i = 0; i < n; ++i) kappa_out[i] = NAN;
  if (n < 4 || n > SL_MAX_LAMBDA) return -1;
  for (int i = 0; i < n; ++i)
    if (!(reg[i] > 0.0) || !(chi2[i] > 0.0) || !__builtin_isfinite(reg[i]) || !__builtin_isfinite(chi2[i])) return -1;
  double* X = scratch;
  double* Y = X + n;
  double* t = Y + n;
  int* keep = (int*)(t + n);                 // n ints fit in n doubles
  double* xs = t + 2 * n;
  double* ys = xs + n;
  double* A = ys + n;                         // n*n
  double* M = A + n * n;
  double* dx1 = M + n;
  double* dy1 = dx1 + n;
  double* Mx = dy1 + n;
  for (int i = 0; i < n; ++i) {
    X[i] = log10(reg[i]);
    Y[i] = log10(chi2[i]);
  }
  double total = 0.0;
  for (int i = 1; i < n; ++i) total += hypot(X[i] - X[i - 1], Y[i] - Y[i - 1]);
  int m = 0;
  keep[m] = 0;
  t[m] = 0.0;
  xs[m] = X[0];
  ys[m] = Y[0];
  ++m;
  double acc = 0.0;
  for (int i = 1; i < n; ++i) {
    acc += hypot(X[i] - X[i - 1], Y[i] - Y[i - 1]);
    if (acc - t[m - 1] <= 1e-12 * total) continue;
    keep[m] = i;
    t[m] = acc;
    xs[m] = X[i];
    ys[m] = Y[i];
    ++m;
  }
  if (m < 4) return -1;
  if (!spline_knot_derivs(t, xs, m, A, M, dx1)) return -1;
  for (int i = 0; i < m; ++i) Mx[i] = M[i];
  if (!spline_knot_derivs(t, ys, m, A, M, dy1)) return -1;
  int best = 0;
  double bestk = -1.0;
  for (int i = 0; i < m; ++i) {
    const double num = fabs(dx1[i] * M[i] - dy1[i] * Mx[i]);
    const double den = dx1[i] * dx1[i] + dy1[i] * dy1[i];
    const double kap = num / (den * sqrt(den));
    if (kappa_out) kappa_out[keep[i]] = kap;
    if (i == 0 || kap > bestk * (1.0 + 1e-12)) {
      best = i;
      bestk = kap;
    }
  }
  return keep[best];
}

constexpr int kLcurveScratch = 2 * SL_MAX_LAMBDA * SL_MAX_LAMBDA + 12 * SL_MAX_LAMBDA;

// The L-curve corner of lcurve_corner_impl computed by a whole block (every
// thread calls it; all receive the result): the logarithms, the segment
// lengths, the rows of the two spline systems, the knot derivatives and the
// curvatures one value per thread with the same operations as there; the
// running arc length with its point drop, the two eliminations (on threads 0
// and 64, in different waves, side by side) and the argmax in order.  Same
// result bit for bit; the one-thread form is a chain of dependent FP64 steps.
// sc: kLcurveScratch doubles of LDS; blocks of at least 128 + n threads.
__device__ inline int lcurve_corner_block(const double* reg, const double* chi2, int n, double* sc) {
  __shared__ int sh[4];   // validity, kept points m, the x system's solve then the result, the y system's solve
  const int tid = threadIdx.x;
  if (n < 4 || n > SL_MAX_LAMBDA) return -1;
  double* X = sc;
  double* Y = X + n;
  double* seg = Y + n;
  double* t = seg + n;
  int* keep = (int*)(t + n);
  double* xs = t + 2 * n;
  double* ys = xs + n;
  double* Mx = ys + n;
  double* My = Mx + n;
  double* dx1 = My + n;
  double* dy1 = dx1 + n;
  double* kap = dy1 + n;
  double* Ax = kap + n;
  double* Ay = Ax + n * n;   // 12 n + 2 n^2 doubles in all
  if (tid == 0) sh[0] = 1;
  __syncthreads();
  if (tid < n) {
    if (!(reg[tid] > 0.0) || !(chi2[tid] > 0.0) || !__builtin_isfinite(reg[tid]) || !__builtin_isfinite(chi2[tid]))
      sh[0] = 0;
    X[tid] = log10(reg[tid]);
    Y[tid] = log10(chi2[tid]);
  }
  __syncthreads();
  if (!sh[0]) return -1;
  if (tid >= 1 && tid < n) seg[tid] = hypot(X[tid] - X[tid - 1], Y[tid] - Y[tid - 1]);
  __syncthreads();
  if (tid == 0) {
    double total = 0.0;
    for (int i = 1; i < n; ++i) total += seg[i];
    int m = 0;
    keep[m] = 0;
    t[m] = 0.0;
    xs[m] = X[0];
    ys[m] = Y[0];
    ++m;
    double acc = 0.0;
    for (int i = 1; i < n; ++i) {
      acc += seg[i];
      if (acc - t[m - 1] <= 1e-12 * total) continue;
      keep[m] = i;
      t[m] = acc;
      xs[m] = X[i];
      ys[m] = Y[i];
      ++m;
    }
    sh[1] = m;
  }
  __syncthreads();
  const int m = sh[1];
  if (m < 4) return -1;
  for (int i = tid; i < 2 * m * m; i += blockDim.x) Ax[i] = 0.0;   // Ax and Ay
  if (tid < m) {
    Mx[tid] = 0.0;
    My[tid] = 0.0;
  }
  __syncthreads();
  if (tid < m) spline_fill_row(t, xs, m, Ax, Mx, tid);
  else if (tid >= 128 && tid < 128 + m) spline_fill_row(t, ys, m, Ay, My, tid - 128);
  __syncthreads();
  if (tid == 0) sh[2] = spline_solve(m, Ax, Mx) ? 1 : 0;
  if (tid == 64) sh[3] = spline_solve(m, Ay, My) ? 1 : 0;
  __syncthreads();
  if (!sh[2] || !sh[3]) return -1;
  __syncthreads();   // every thread has read sh[2] before thread 0 reuses it
  if (tid < m) {
    dx1[tid] = spline_d1_at(t, xs, m, Mx, tid);
    dy1[tid] = spline_d1_at(t, ys, m, My, tid);
  }
  __syncthreads();
  if (tid < m) {
    const double num = fabs(dx1[tid] * My[tid] - dy1[tid] * Mx[tid]);
    const double den = dx1[tid] * dx1[tid] + dy1[tid] * dy1[tid];
    kap[tid] = num / (den * sqrt(den));
  }
  __syncthreads();
  if (tid == 0) {
    int best = 0;
    double bestk = -1.0;
    for (int i = 0; i < m; ++i)
      if (i == 0 || kap[i] > bestk * (1.0 + 1e-12)) {
        best = i;
        bestk = kap[i];
      }
    sh[2] = keep[best];
  }
  __syncthreads();
  return sh[2];
}


}  // namespace sl
