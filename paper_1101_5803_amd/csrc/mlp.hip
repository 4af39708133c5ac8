// Surrogate MLP 7 -> 256 -> 256 -> 1 (GELU, erf form) on gfx950.
//
// Numerics: FP32 master weights; BF16 (round to nearest even) copies of the
// weights and of every layer input enter the products, which accumulate in
// FP32.  The forward 256x256 product runs on the BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16).  The backward products keep the gradient
// signals in FP32 and run on the FP32 matrix cores (v_mfma_f32_16x16x4_f32);
// the BF16-valued weights and activations enter them exactly.  Rounding an
// activation to BF16 is treated as the identity in the backward pass.
//
// Kernels of one training step (all on the caller's stream):
//   k_mlp_prep   W1 -> W1^T as BF16 (forward operand) and FP32 (backward)
//   k_mlp_fwd    layer 1 (VALU), layer 2 (MFMA), output dot product; stores
//                the activations and GELU derivatives of the batch
//   k_mlp_bwd1   output gradient, dz2, dh1 = dz2 W1^T (MFMA), dz1, and
//                per-tile partial sums of the small gradients
//   k_mlp_wgrad  gW1 = a1^T dz2 (MFMA, 32x32 tiles) and the fixed-order
//                reduction of the per-tile partials
//   k_mlp_adam   Adam with bias correction, elementwise
// Every sum has a fixed order, so results are bitwise reproducible.
#include <mutex>

#include "common.h"

namespace sl {
namespace {

constexpr int kIn = SL_MLP_IN;
constexpr int kH = SL_MLP_HID;
constexpr int kBM = 32;        // batch rows per forward / backward block
constexpr int kThr = 256;      // threads per block (4 waves)
constexpr int kMaxBatch = SL_MLP_MAX_BATCH;

// parameter offsets (floats) in the packed vector
constexpr int oW0 = 0;
constexpr int oB0 = oW0 + kIn * kH;
constexpr int oW1 = oB0 + kH;
constexpr int oB1 = oW1 + kH * kH;
constexpr int oW2 = oB1 + kH;
constexpr int oB2 = oW2 + kH;
static_assert(oB2 + 1 == SL_MLP_NPARAM, "parameter layout");

// per-tile partial sums written by k_mlp_bwd1: gW0 | gb0 | gb1 | gW2 | gb2
constexpr int pW0 = 0;
constexpr int pB0 = pW0 + kIn * kH;
constexpr int pB1 = pB0 + kH;
constexpr int pW2 = pB1 + kH;
constexpr int pB2 = pW2 + kH;
constexpr int kPart = pB2 + kH;   // gb2 sits in the first slot of its 256-wide group

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round to the nearest BF16 value, ties to even (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16r(float f) { return __uint_as_float((unsigned)bf16_bits(f) << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
// d/dz [z Phi(z)] = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct Ws {
  unsigned short* w1t_bf;   // [256 out][256 in] BF16 bits
  float* w1t_f;             // [256 out][256 in] BF16 values in FP32
  float* yhat;              // [B]
  float* g3;                // [B] dL/dy
  float* a1;                // [B][256] BF16 values of h1
  float* gz1;               // [B][256] gelu'(z1)
  float* a2;                // [B][256]
  float* gz2;               // [B][256]
  float* dz2;               // [B][256]
  float* part;              // [tiles][kPart]
  double* lossp;            // [tiles]
  double* loss;             // [1]
  float* grad;              // [NPARAM] (when the caller passes no gradient buffer)
};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t carve(int batch, unsigned char* base, Ws* w) {
  const size_t B = (size_t)(batch > 0 ? batch : 0);
  const size_t tiles = (B + kBM - 1) / kBM;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return base ? base + o : nullptr;
  };
  Ws t;
  t.w1t_bf = reinterpret_cast<unsigned short*>(take(sizeof(unsigned short) * kH * kH));
  t.w1t_f = reinterpret_cast<float*>(take(sizeof(float) * kH * kH));
  t.yhat = reinterpret_cast<float*>(take(sizeof(float) * B));
  t.g3 = reinterpret_cast<float*>(take(sizeof(float) * B));
  t.a1 = reinterpret_cast<float*>(take(sizeof(float) * B * kH));
  t.gz1 = reinterpret_cast<float*>(take(sizeof(float) * B * kH));
  t.a2 = reinterpret_cast<float*>(take(sizeof(float) * B * kH));
  t.gz2 = reinterpret_cast<float*>(take(sizeof(float) * B * kH));
  t.dz2 = reinterpret_cast<float*>(take(sizeof(float) * B * kH));
  t.part = reinterpret_cast<float*>(take(sizeof(float) * tiles * kPart));
  t.lossp = reinterpret_cast<double*>(take(sizeof(double) * tiles));
  t.loss = reinterpret_cast<double*>(take(sizeof(double)));
  t.grad = reinterpret_cast<float*>(take(sizeof(float) * SL_MLP_NPARAM));
  if (w) *w = t;
  return off;
}

// W1 [in][out] -> W1^T [out][in] in BF16 and FP32, through a 64x64 LDS tile.
// Grid 16 blocks of 256 threads.
__global__ void __launch_bounds__(kThr) k_mlp_prep(const float* __restrict__ params, unsigned short* __restrict__ wbf,
                                                   float* __restrict__ wf) {
  __shared__ float tile[64][65];
  const int ti = blockIdx.x / 4, tj = blockIdx.x % 4;   // tile rows (in) and columns (out)
  const float* W1 = params + oW1;
  for (int e = threadIdx.x; e < 64 * 64; e += kThr) {
    const int r = e / 64, c = e % 64;
    tile[r][c] = bf16r(W1[(ti * 64 + r) * kH + tj * 64 + c]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += kThr) {
    const int r = e / 64, c = e % 64;   // r: out within tile, c: in within tile
    const float v = tile[c][r];
    const int idx = (tj * 64 + r) * kH + ti * 64 + c;
    wf[idx] = v;
    wbf[idx] = (unsigned short)(__float_as_uint(v) >> 16);
  }
}

struct FwdArgs {
  const float* params;
  const float* x;
  const float* ytrue;   // training only
  int B;
  float inv_b2;         // 2 / B
  float* y;             // forward output (nullable in training)
  Ws w;
};

// One block: kBM batch rows.  Thread t owns hidden column t in layer 1; wave
// w owns output columns [64w, 64w + 64) of layer 2 as two 32x32 MFMA tiles.
template <bool TRAIN>
__global__ void __launch_bounds__(kThr) k_mlp_fwd(FwdArgs a) {
  constexpr int kPitch = kH + 8;   // BF16 elements per LDS row
  __shared__ __attribute__((aligned(16))) unsigned short A1s[kBM * kPitch];
  __shared__ float xs[kBM * kIn];
  __shared__ float yp[4][kBM];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blockIdx.x * kBM;
  const int nrow = min(kBM, a.B - row0);
  for (int e = tid; e < kBM * kIn; e += kThr) xs[e] = e < nrow * kIn ? bf16r(a.x[(size_t)row0 * kIn + e]) : 0.0f;
  __syncthreads();
  // ---- layer 1: z1 = bf16(x) bf16(W0) + b0, a1 = bf16(gelu(z1))
  {
    const int n = tid;
    float w0[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) w0[k] = bf16r(a.params[oW0 + k * kH + n]);
    const float b0 = a.params[oB0 + n];
    for (int r = 0; r < kBM; ++r) {
      float z = b0;
#pragma unroll
      for (int k = 0; k < kIn; ++k) z = fmaf(xs[r * kIn + k], w0[k], z);
      unsigned short hb = 0;
      if (r < nrow) {
        hb = bf16_bits(gelu(z));
        if (TRAIN) {
          const size_t o = (size_t)(row0 + r) * kH + n;
          a.w.a1[o] = __uint_as_float((unsigned)hb << 16);
          a.w.gz1[o] = gelu_grad(z);
        }
      }
      A1s[r * kPitch + n] = hb;
    }
  }
  __syncthreads();
  // ---- layer 2 on the BF16 matrix cores: z2 = a1 W1 (+ b1 below)
  f32x16 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;
  const int li = lane & 31, lg = lane >> 5;
  const unsigned short* brow0 = a.w.w1t_bf + (size_t)(64 * wv + li) * kH + 8 * lg;
  const unsigned short* brow1 = brow0 + 32 * kH;
  const unsigned short* arow = A1s + li * kPitch + 8 * lg;
#pragma unroll 4
  for (int kk = 0; kk < kH / 16; ++kk) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(arow + 16 * kk);
    const bf16x8 b0v = *reinterpret_cast<const bf16x8*>(brow0 + 16 * kk);
    const bf16x8 b1v = *reinterpret_cast<const bf16x8*>(brow1 + 16 * kk);
    acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b0v, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b1v, acc[1], 0, 0, 0);
  }
  // ---- epilogue: a2 = bf16(gelu(z2 + b1)); partial y over this lane's column
  // Accumulator element r of a 32x32 tile sits at row 8(r/4) + 4 lg + r%4,
  // column li.
  float ys[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) ys[r] = 0.0f;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int j = 64 * wv + 32 * t + li;
    const float b1 = a.params[oB1 + j];
    const float w2 = bf16r(a.params[oW2 + j]);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * lg + (r & 3);
      const float z = acc[t][r] + b1;
      const float h = bf16r(gelu(z));
      if (TRAIN && i < nrow) {
        const size_t o = (size_t)(row0 + i) * kH + j;
        a.w.a2[o] = h;
        a.w.gz2[o] = gelu_grad(z);
      }
      ys[r] = fmaf(h, w2, ys[r]);
    }
  }
  // sum over the 32 columns of each half-wave (lanes sharing lg)
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float v = ys[r];
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    ys[r] = v;
  }
  if (li == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) yp[wv][8 * (r >> 2) + 4 * lg + (r & 3)] = ys[r];
  }
  __syncthreads();
  if (tid < kBM) {
    double lp = 0.0;
    if (tid < nrow) {
      const float yv = ((a.params[oB2] + yp[0][tid]) + yp[1][tid]) + (yp[2][tid] + yp[3][tid]);
      const size_t b = (size_t)row0 + tid;
      if (a.y) a.y[b] = yv;
      if (TRAIN) {
        a.w.yhat[b] = yv;
        const float d = yv - a.ytrue[b];
        a.w.g3[b] = a.inv_b2 * d;
        lp = (double)d * (double)d;
      }
    }
    if (TRAIN) {
      // fixed-order sum of the 32 rows within the first wave
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) lp += __shfl_xor(lp, o, 64);
      if (tid == 0) a.w.lossp[blockIdx.x] = lp;
    }
  }
}

struct BwdArgs {
  const float* params;
  const float* x;
  int B;
  Ws w;
};

// One block: kBM batch rows.  dz2 = g3 bf16(W2) gelu'(z2); dh1 = dz2 W1^T on
// the FP32 matrix cores (wave w: output columns [64w, 64w + 64), two 16-row
// tiles); dz1 = dh1 gelu'(z1).  Writes dz2 and the tile's partial sums of
// gW0, gb0, gb1, gW2, gb2.
__global__ void __launch_bounds__(kThr) k_mlp_bwd1(BwdArgs a) {
  constexpr int kP = kH + 4;
  __shared__ float D2s[kBM * kP];
  __shared__ float xs[kBM * kIn];
  __shared__ float g3s[kBM];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blockIdx.x * kBM;
  const int nrow = min(kBM, a.B - row0);
  float* part = a.w.part + (size_t)blockIdx.x * kPart;
  for (int e = tid; e < kBM * kIn; e += kThr) xs[e] = e < nrow * kIn ? bf16r(a.x[(size_t)row0 * kIn + e]) : 0.0f;
  if (tid < kBM) g3s[tid] = tid < nrow ? a.w.g3[row0 + tid] : 0.0f;
  __syncthreads();
  {
    const int j = tid;
    const float w2 = bf16r(a.params[oW2 + j]);
    float sb1 = 0.0f, sw2 = 0.0f;
    for (int r = 0; r < kBM; ++r) {
      float d = 0.0f;
      if (r < nrow) {
        const size_t o = (size_t)(row0 + r) * kH + j;
        d = g3s[r] * w2 * a.w.gz2[o];
        a.w.dz2[o] = d;
        sw2 = fmaf(a.w.a2[o], g3s[r], sw2);
      }
      sb1 += d;
      D2s[r * kP + j] = d;
    }
    part[pB1 + j] = sb1;
    part[pW2 + j] = sw2;
    if (j == 0) {
      float s = 0.0f;
      for (int r = 0; r < kBM; ++r) s += g3s[r];
      part[pB2] = s;
    }
  }
  __syncthreads();
  // dh1[i][k] = sum_j dz2[i][j] W1[k][j]: A = D2s (rows i, inner j), B[j][k] = W1^T[j][k]
  // f32 16x16x4: A element (row l%16, inner l/16); B element (inner l/16, column l%16);
  // accumulator element r at row 4(l/16) + r, column l%16.
  const int lc = lane & 15, lq = lane >> 4;
  f32x4 acc[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][n][r] = 0.0f;
  const float* Bp = a.w.w1t_f + (size_t)lq * kH + 64 * wv + lc;
#pragma unroll 2
  for (int kk = 0; kk < kH / 4; ++kk) {
    const float a0 = D2s[lc * kP + 4 * kk + lq];
    const float a1 = D2s[(16 + lc) * kP + 4 * kk + lq];
    float bv[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) bv[n] = Bp[(size_t)(4 * kk) * kH + 16 * n];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      acc[0][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bv[n], acc[0][n], 0, 0, 0);
      acc[1][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bv[n], acc[1][n], 0, 0, 0);
    }
  }
  // dz1 = dh1 gelu'(z1); partial gb0 and gW0 of this tile
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const int k = 64 * wv + 16 * n + lc;
    float sb0 = 0.0f, sw0[kIn];
#pragma unroll
    for (int c = 0; c < kIn; ++c) sw0[c] = 0.0f;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * m + 4 * lq + r;
        float dz1 = 0.0f;
        if (i < nrow) dz1 = acc[m][n][r] * a.w.gz1[(size_t)(row0 + i) * kH + k];
        sb0 += dz1;
#pragma unroll
        for (int c = 0; c < kIn; ++c) sw0[c] = fmaf(xs[i * kIn + c], dz1, sw0[c]);
      }
    // add the four row groups (lanes lc, lc+16, lc+32, lc+48)
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      sb0 += __shfl_xor(sb0, o, 64);
#pragma unroll
      for (int c = 0; c < kIn; ++c) sw0[c] += __shfl_xor(sw0[c], o, 64);
    }
    if (lq == 0) {
      part[pB0 + k] = sb0;
#pragma unroll
      for (int c = 0; c < kIn; ++c) part[pW0 + c * kH + k] = sw0[c];
    }
  }
}

struct WgradArgs {
  int B;
  int tiles;
  Ws w;
  float* grad;
};

// Blocks 0..63: gW1 tile (32 inputs x 32 outputs) = a1^T dz2 over the batch,
// the four waves taking interleaved groups of 4 rows, summed in a fixed order.
// Blocks 64..64+kPart/256-1: fixed-order sums of the per-tile partials; block
// 64 also sums the loss.
__global__ void __launch_bounds__(kThr) k_mlp_wgrad(WgradArgs a) {
  __shared__ float red[4][32][33];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (blockIdx.x < 64) {
    const int k0 = 32 * (blockIdx.x / 8), j0 = 32 * (blockIdx.x % 8);
    const int lc = lane & 15, lq = lane >> 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][n][r] = 0.0f;
    for (int b0 = 4 * wv; b0 < a.B; b0 += 16) {
      const int b = b0 + lq;
      float av[2] = {0.0f, 0.0f}, bv[2] = {0.0f, 0.0f};
      if (b < a.B) {
        const float* a1r = a.w.a1 + (size_t)b * kH + k0 + lc;
        const float* d2r = a.w.dz2 + (size_t)b * kH + j0 + lc;
        av[0] = a1r[0];
        av[1] = a1r[16];
        bv[0] = d2r[0];
        bv[1] = d2r[16];
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m], bv[n], acc[m][n], 0, 0, 0);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wv][16 * m + 4 * lq + r][16 * n + lc] = acc[m][n][r];
    __syncthreads();
    for (int e = tid; e < 32 * 32; e += kThr) {
      const int i = e / 32, j = e % 32;
      const float v = (red[0][i][j] + red[1][i][j]) + (red[2][i][j] + red[3][i][j]);
      a.grad[oW1 + (k0 + i) * kH + j0 + j] = v;
    }
    return;
  }
  const int q = blockIdx.x - 64;
  const int c = q * kThr + tid;   // column of the partial table
  float s = 0.0f;
  for (int t = 0; t < a.tiles; ++t) s += a.w.part[(size_t)t * kPart + c];
  if (c < pB0) a.grad[oW0 + c] = s;
  else if (c < pB1) a.grad[oB0 + c - pB0] = s;
  else if (c < pW2) a.grad[oB1 + c - pB1] = s;
  else if (c < pB2) a.grad[oW2 + c - pW2] = s;
  else if (c == pB2) a.grad[oB2] = s;
  if (q == 0 && wv == 0) {
    double l = 0.0;
    for (int t = lane; t < a.tiles; t += 64) l += a.w.lossp[t];
    l = wave_sum(l);
    if (lane == 0) *a.w.loss = l / (double)a.B;
  }
}

__global__ void __launch_bounds__(kThr) k_mlp_adam(float* __restrict__ p, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g, float lr,
                                                   float c1, float c2, const double* __restrict__ loss,
                                                   float* __restrict__ loss_out) {
  // 1 - beta written out: 1.0f - 0.999f is 1.0000467e-3 in FP32, not 1e-3
  constexpr float b1 = 0.9f, omb1 = 0.1f, b2 = 0.999f, omb2 = 0.001f, eps = 1e-8f;
  const int i = blockIdx.x * kThr + threadIdx.x;
  if (i == 0 && loss_out) *loss_out = (float)*loss;
  if (i >= SL_MLP_NPARAM) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Scratch of sl_mlp_forward_noalloc: the BF16 and FP32 transposed copies of
// W1 that k_mlp_prep writes and k_mlp_fwd reads (the forward pass needs no
// other scratch, whatever the batch).  Every call rewrites all of it.
constexpr size_t kNoallocBf = sizeof(unsigned short) * kH * kH;   // 128 KiB
constexpr size_t kNoallocBytes = kNoallocBf + sizeof(float) * kH * kH;   // 384 KiB
static_assert(kNoallocBf % 256 == 0, "FP32 copy stays 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// Device address of `scratch` on the current device, looked up once per
// device with that device current (each GPU holds its own copy).
int noalloc_scratch(unsigned char** out) {
  static std::mutex mu;
  static unsigned char* ptr[64] = {nullptr};
  int dev = 0;
  SL_HIP(hipGetDevice(&dev));
  SL_REQUIRE(dev >= 0 && dev < 64, "device index %d out of range", dev);
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    SL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    SL_REQUIRE(p != nullptr, "no device address for the forward scratch");
    ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = ptr[dev];
  return SL_OK;
}

int validate(const void* params, const float* x, int batch, const void* ws) {
  SL_REQUIRE(batch >= 1 && batch <= kMaxBatch, "batch %d outside [1, %d]", batch, kMaxBatch);
  SL_REQUIRE(params && x && ws, "null pointer argument");
  return SL_OK;
}

}  // namespace
}  // namespace sl

using namespace sl;

extern "C" {

size_t sl_mlp_workspace_size(int batch) {
  if (batch < 0 || batch > kMaxBatch) {
    set_error("batch %d outside [0, %d]", batch, kMaxBatch);
    return 0;
  }
  return carve(batch, nullptr, nullptr);
}

int sl_mlp_forward(const float* params, const float* x, int batch, float* y, void* workspace, void* stream) {
  if (int rc = validate(params, x, batch, workspace)) return rc;
  SL_REQUIRE(y, "null output");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ws w;
  carve(batch, static_cast<unsigned char*>(workspace), &w);
  k_mlp_prep<<<16, kThr, 0, st>>>(params, w.w1t_bf, w.w1t_f);
  if (int rc = check_launch("k_mlp_prep")) return rc;
  FwdArgs fa{params, x, nullptr, batch, 0.0f, y, w};
  k_mlp_fwd<false><<<(batch + kBM - 1) / kBM, kThr, 0, st>>>(fa);
  return check_launch("k_mlp_fwd");
}

int sl_mlp_forward_noalloc(const float* params, const float* x, int batch, float* y, void* stream) {
  SL_REQUIRE(batch >= 1 && batch <= kMaxBatch, "batch %d outside [1, %d]", batch, kMaxBatch);
  SL_REQUIRE(params && x && y, "null pointer argument");
  unsigned char* sc = nullptr;
  if (int rc = noalloc_scratch(&sc)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ws w{};
  w.w1t_bf = reinterpret_cast<unsigned short*>(sc);
  w.w1t_f = reinterpret_cast<float*>(sc + kNoallocBf);
  k_mlp_prep<<<16, kThr, 0, st>>>(params, w.w1t_bf, w.w1t_f);
  if (int rc = check_launch("k_mlp_prep")) return rc;
  FwdArgs fa{params, x, nullptr, batch, 0.0f, y, w};
  k_mlp_fwd<false><<<(batch + kBM - 1) / kBM, kThr, 0, st>>>(fa);
  return check_launch("k_mlp_fwd");
}

int sl_mlp_train_step(float* params, float* adam_m, float* adam_v, const float* x, const float* y, int batch,
                      float lr, int t, float* grads_out, float* loss_out, void* workspace, void* stream) {
  if (int rc = validate(params, x, batch, workspace)) return rc;
  SL_REQUIRE(adam_m && adam_v && y, "null pointer argument");
  SL_REQUIRE(t >= 1, "Adam step number t = %d must be >= 1", t);
  SL_REQUIRE(std::isfinite(lr) && lr > 0.0f, "learning rate must be finite and positive");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ws w;
  carve(batch, static_cast<unsigned char*>(workspace), &w);
  const int tiles = (batch + kBM - 1) / kBM;
  float* grad = grads_out ? grads_out : w.grad;
  k_mlp_prep<<<16, kThr, 0, st>>>(params, w.w1t_bf, w.w1t_f);
  if (int rc = check_launch("k_mlp_prep")) return rc;
  FwdArgs fa{params, x, y, batch, (float)(2.0 / batch), nullptr, w};
  k_mlp_fwd<true><<<tiles, kThr, 0, st>>>(fa);
  if (int rc = check_launch("k_mlp_fwd")) return rc;
  BwdArgs ba{params, x, batch, w};
  k_mlp_bwd1<<<tiles, kThr, 0, st>>>(ba);
  if (int rc = check_launch("k_mlp_bwd1")) return rc;
  WgradArgs wa{batch, tiles, w, grad};
  k_mlp_wgrad<<<64 + kPart / kThr, kThr, 0, st>>>(wa);
  if (int rc = check_launch("k_mlp_wgrad")) return rc;
  const double c1 = 1.0 / (1.0 - std::pow(0.9, t)), c2 = 1.0 / (1.0 - std::pow(0.999, t));
  k_mlp_adam<<<(SL_MLP_NPARAM + kThr - 1) / kThr, kThr, 0, st>>>(params, adam_m, adam_v, grad, lr, (float)c1,
                                                                 (float)c2, w.loss, loss_out);
  return check_launch("k_mlp_adam");
}

}  // extern "C"
