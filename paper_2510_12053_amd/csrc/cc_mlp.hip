// Learned per-vertex warm start: feature extraction, and a 32-64-64-16 SiLU
// network whose products run on BF16 MFMA (v_mfma_f32_16x16x16_bf16) with
// FP32 accumulation.  One wave owns a tile of 16 rows; activations move
// between layers through LDS to turn the accumulator layout into the operand
// layout.  Weight gradients are accumulated per wave and reduced in a fixed
// order, so training is bit-reproducible.
//
// MFMA 16x16x16 lane layout (lane l, element i of the 4-vector):
//   A operand  A[l % 16][4 (l / 16) + i]
//   B operand  B[4 (l / 16) + i][l % 16]
//   C result   C[4 (l / 16) + i][l % 16]

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cc_device.h"
#include "cc_mlp.h"

namespace cc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);                                    // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.f / (1.f + expf(-z));
  return s * (1.f + z * (1.f - s));
}

__device__ __forceinline__ floatx4 mfma(bf16x4 a, bf16x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// B fragment of a row-major K x N bf16 matrix W for k-step s and n-tile t.
__device__ __forceinline__ bf16x4 bfrag(const uint16_t* W, int N, int s, int t, int l) {
  bf16x4 b;
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = (short)W[(16 * s + 4 * (l / 16) + i) * N + 16 * t + (l % 16)];
  return b;
}
// B fragment of W^T where W is row-major N_w x K_w: (W^T)[k][n] = W[n][k].
__device__ __forceinline__ bf16x4 bfragT(const uint16_t* W, int Kw, int s, int t, int l) {
  bf16x4 b;
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = (short)W[(16 * t + (l % 16)) * Kw + 16 * s + 4 * (l / 16) + i];
  return b;
}
// A fragment (k-step s) from a 16 x ld bf16 tile in LDS (row-major).
__device__ __forceinline__ bf16x4 afrag(const uint16_t* tile, int ld, int s, int l) {
  bf16x4 a;
#pragma unroll
  for (int i = 0; i < 4; ++i) a[i] = (short)tile[(l % 16) * ld + 16 * s + 4 * (l / 16) + i];
  return a;
}
// A fragment of tile^T (m-tile mt): (tile^T)[m][k] = tile[k][m], k = row.
__device__ __forceinline__ bf16x4 afragT(const uint16_t* tile, int ld, int mt, int l) {
  bf16x4 a;
#pragma unroll
  for (int i = 0; i < 4; ++i) a[i] = (short)tile[(4 * (l / 16) + i) * ld + 16 * mt + (l % 16)];
  return a;
}
// Accumulator (C layout) of n-tile t written into a 16 x ld bf16 LDS tile.
__device__ __forceinline__ void cstore(uint16_t* tile, int ld, int t, int l, floatx4 v) {
#pragma unroll
  for (int i = 0; i < 4; ++i) tile[(4 * (l / 16) + i) * ld + 16 * t + (l % 16)] = f2bf(v[i]);
}
__device__ __forceinline__ bf16x4 to_bf(floatx4 v) {
  bf16x4 b;
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = (short)f2bf(v[i]);
  return b;
}

struct MlpDev {
  const float* W;       // FP32 master parameters, packed (MLP_* offsets)
  const uint16_t* W1b;  // 32 x 64 bf16
  const uint16_t* W2b;  // 64 x 64
  const uint16_t* W3b;  // 64 x 16
  const float* mean;    // 16
  const float* istd;    // 16 (reciprocal standard deviations)
};


// Normalised input tile (16 rows x 16 features) -> LDS, bf16.  Rows past
// `rows` are zero.  src(row) returns the address of the row's raw features.
template <typename Src>
__device__ __forceinline__ void load_input(uint16_t* xt, int rows, const MlpDev& net, Src&& src,
                                           int l) {
  for (int e = l; e < 256; e += 64) {
    const int r = e / 16, c = e % 16;
    float v = 0.f;
    if (r < rows) v = (src(r)[c] - net.mean[c]) * net.istd[c];
    xt[r * 16 + c] = f2bf(v);
  }
}

// Forward of one 16-row tile.  On return: Z1, Z2 (pre-activations, C layout,
// 4 n-tiles each), LDS tiles a1 (16x64), a2 (16x64) of bf16 activations, and
// the output accumulator y (16 x 16, C layout, bias added).
__device__ __forceinline__ void tile_forward(const MlpDev& net, const uint16_t* xt, uint16_t* a1,
                                             uint16_t* a2, floatx4 Z1[4], floatx4 Z2[4],
                                             floatx4& y, int l) {
  const float* b1 = net.W + MLP_B1;
  const float* b2 = net.W + MLP_B2;
  const float* b3 = net.W + MLP_B3;
  const bf16x4 ax = afrag(xt, 16, 0, l);  // features 16..31 are zero padding
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
    c = mfma(ax, bfrag(net.W1b, MLP_HID, 0, t, l), c);
    const float bias = b1[16 * t + (l % 16)];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] += bias;
    Z1[t] = c;
    floatx4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = silu(c[i]);
    cstore(a1, MLP_HID, t, l, a);
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) c = mfma(afrag(a1, MLP_HID, s, l), bfrag(net.W2b, MLP_HID, s, t, l), c);
    const float bias = b2[16 * t + (l % 16)];
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] += bias;
    Z2[t] = c;
    floatx4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = silu(c[i]);
    cstore(a2, MLP_HID, t, l, a);
  }
  __syncthreads();
  floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 4; ++s) c = mfma(afrag(a2, MLP_HID, s, l), bfrag(net.W3b, MLP_OUT, s, 0, l), c);
  const float bias = b3[l % 16];
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] += bias;
  y = c;
}

// Inference: rows of raw features (stride 16) -> first 3 outputs (stride 3).
__global__ void __launch_bounds__(64 * MLP_WAVES) k_mlp_forward(MlpDev net, const float* __restrict__ X,
                                                                int B, float* __restrict__ Y) {
  __shared__ uint16_t lds[MLP_WAVES][16 * 16 + 2 * 16 * 64];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  uint16_t* xt = lds[w];
  uint16_t* a1 = xt + 256;
  uint16_t* a2 = a1 + 16 * 64;
  const int tiles = (B + 15) / 16;
  // every wave of the workgroup runs the same number of tile iterations so the
  // workgroup barriers inside tile_forward line up
  const int per = (tiles + gridDim.x * MLP_WAVES - 1) / (gridDim.x * MLP_WAVES);
  for (int it = 0; it < per; ++it) {
    const int tile = (blockIdx.x * MLP_WAVES + w) + it * gridDim.x * MLP_WAVES;
    const int r0 = tile * 16;
    const int rows = tile < tiles ? min(16, B - r0) : 0;
    load_input(xt, rows, net, [&](int r) { return X + (size_t)(r0 + r) * MLP_IN; }, l);
    __syncthreads();
    floatx4 Z1[4], Z2[4], y;
    tile_forward(net, xt, a1, a2, Z1, Z2, y, l);
    if ((l % 16) < MLP_NOUT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * (l / 16) + i;
        if (r < rows) Y[(size_t)(r0 + r) * MLP_NOUT + (l % 16)] = y[i];
      }
    }
    __syncthreads();
  }
}

// Forward + MSE + backward for the minibatch rows idx[0..B).  Each wave
// accumulates the gradient of its tiles; wave w writes its partial gradient
// to part[w * MLP_NPARAM ...] and its partial loss to lpart[w].
__global__ void __launch_bounds__(64 * MLP_WAVES) k_mlp_train(MlpDev net, const float* __restrict__ X,
                                                              const float* __restrict__ T,
                                                              const int* __restrict__ idx, int B,
                                                              float* __restrict__ part,
                                                              float* __restrict__ lpart) {
  __shared__ uint16_t lds[MLP_WAVES][16 * 16 + 2 * 16 * 64 + 16 * 64];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  uint16_t* xt = lds[w];
  uint16_t* a1 = xt + 256;
  uint16_t* a2 = a1 + 16 * 64;
  uint16_t* dz = a2 + 16 * 64;  // 16 x 64 scratch for dZ in operand layout
  const float gscale = 2.f / (float(B) * MLP_NOUT);
  floatx4 gW3[4], gW2[16], gW1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) gW3[i] = gW1[i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 16; ++i) gW2[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  float gb1[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f, loss = 0.f;
  const int tiles = (B + 15) / 16;
  const int nw = gridDim.x * MLP_WAVES;
  const int per = (tiles + nw - 1) / nw;
  for (int it = 0; it < per; ++it) {
    const int tile = (blockIdx.x * MLP_WAVES + w) + it * nw;
    const int r0 = tile * 16;
    const int rows = tile < tiles ? min(16, B - r0) : 0;
    load_input(xt, rows, net, [&](int r) { return X + (size_t)idx[r0 + r] * MLP_IN; }, l);
    __syncthreads();
    floatx4 Z1[4], Z2[4], y;
    tile_forward(net, xt, a1, a2, Z1, Z2, y, l);
    // dY (C layout): only the first 3 outputs of real rows carry loss
    floatx4 dy;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * (l / 16) + i, c = l % 16;
      float d = 0.f;
      if (r < rows && c < MLP_NOUT) {
        const float res = y[i] - T[(size_t)idx[r0 + r] * MLP_NOUT + c];
        loss += res * res;
        d = gscale * res;
      }
      dy[i] = d;
    }
    // layer 3: dW3 += A2^T dY, db3 += colsum dY, dA2 = dY W3^T
    const bf16x4 dyb = to_bf(dy);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) gW3[mt] = mfma(afragT(a2, MLP_HID, mt, l), dyb, gW3[mt]);
    gb3 += dy[0] + dy[1] + dy[2] + dy[3];
    cstore(dz, 16, 0, l, dy);
    __syncthreads();
    floatx4 dZ2[4];
    const bf16x4 ady = afrag(dz, 16, 0, l);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      floatx4 c = {0.f, 0.f, 0.f, 0.f};
      c = mfma(ady, bfragT(net.W3b, MLP_OUT, 0, t, l), c);
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] *= dsilu(Z2[t][i]);
      dZ2[t] = c;
      gb2[t] += c[0] + c[1] + c[2] + c[3];
    }
    __syncthreads();
    // layer 2: dW2 += A1^T dZ2, dA1 = dZ2 W2^T
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x4 b = to_bf(dZ2[t]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) gW2[mt * 4 + t] = mfma(afragT(a1, MLP_HID, mt, l), b, gW2[mt * 4 + t]);
      cstore(dz, MLP_HID, t, l, dZ2[t]);
    }
    __syncthreads();
    floatx4 dZ1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) c = mfma(afrag(dz, MLP_HID, s, l), bfragT(net.W2b, MLP_HID, s, t, l), c);
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] *= dsilu(Z1[t][i]);
      dZ1[t] = c;
      gb1[t] += c[0] + c[1] + c[2] + c[3];
    }
    // layer 1: dW1 (first 16 input rows) += Xn^T dZ1
    const bf16x4 ax = afragT(xt, 16, 0, l);
#pragma unroll
    for (int t = 0; t < 4; ++t) gW1[t] = mfma(ax, to_bf(dZ1[t]), gW1[t]);
    __syncthreads();
  }
  // bias sums: combine the four lane groups holding the same column
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    gb1[t] += __shfl_xor(gb1[t], 16, 64);
    gb1[t] += __shfl_xor(gb1[t], 32, 64);
    gb2[t] += __shfl_xor(gb2[t], 16, 64);
    gb2[t] += __shfl_xor(gb2[t], 32, 64);
  }
  gb3 += __shfl_xor(gb3, 16, 64);
  gb3 += __shfl_xor(gb3, 32, 64);
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
  float* P = part + (size_t)(blockIdx.x * MLP_WAVES + w) * MLP_NPARAM;
  // C layout of an (m-tile, n-tile) gradient block: row 16 mt + 4 (l/16) + i, col 16 t + l%16
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * mt + 4 * (l / 16) + i;
      P[MLP_W3 + r * MLP_OUT + (l % 16)] = gW3[mt][i];
#pragma unroll
      for (int t = 0; t < 4; ++t) P[MLP_W2 + r * MLP_HID + 16 * t + (l % 16)] = gW2[mt * 4 + t][i];
    }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * (l / 16) + i;
      P[MLP_W1 + r * MLP_HID + 16 * t + (l % 16)] = gW1[t][i];
      P[MLP_W1 + (16 + r) * MLP_HID + 16 * t + (l % 16)] = 0.f;  // padding inputs
    }
  if (l < 16) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      P[MLP_B1 + 16 * t + l] = gb1[t];
      P[MLP_B2 + 16 * t + l] = gb2[t];
    }
    P[MLP_B3 + l] = gb3;
  }
  if (l == 0) lpart[blockIdx.x * MLP_WAVES + w] = loss;
}

// Fixed-order sum of the per-wave partials: grad[p] = sum_w part[w][p].
__global__ void k_mlp_sum(const float* __restrict__ part, int nwaves, float* __restrict__ grad,
                          const float* __restrict__ lpart, float* __restrict__ loss, int B) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MLP_NPARAM) {
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += part[(size_t)w * MLP_NPARAM + p];
    grad[p] = s;
  }
  if (p == 0) {
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += lpart[w];
    loss[0] = s / (float(B) * MLP_NOUT);
  }
}

// Adam on the FP32 masters; refreshes the bf16 copies of the weight matrices.
__global__ void k_mlp_adam(float* __restrict__ W, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, float lr, float c1, float c2, uint16_t* __restrict__ W1b,
                           uint16_t* __restrict__ W2b, uint16_t* __restrict__ W3b) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mi = b1 * m[p] + (1.f - b1) * g[p];
  const float vi = b2 * v[p] + (1.f - b2) * g[p] * g[p];
  m[p] = mi;
  v[p] = vi;
  const float w = W[p] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  W[p] = w;
  if (p >= MLP_W1 && p < MLP_W1 + MLP_IN_PAD * MLP_HID) W1b[p - MLP_W1] = f2bf(w);
  else if (p >= MLP_W2 && p < MLP_W2 + MLP_HID * MLP_HID) W2b[p - MLP_W2] = f2bf(w);
  else if (p >= MLP_W3 && p < MLP_W3 + MLP_HID * MLP_OUT) W3b[p - MLP_W3] = f2bf(w);
}

__global__ void k_mlp_to_bf16(const float* __restrict__ W, uint16_t* __restrict__ W1b,
                              uint16_t* __restrict__ W2b, uint16_t* __restrict__ W3b) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  const float w = W[p];
  if (p >= MLP_W1 && p < MLP_W1 + MLP_IN_PAD * MLP_HID) W1b[p - MLP_W1] = f2bf(w);
  else if (p >= MLP_W2 && p < MLP_W2 + MLP_HID * MLP_HID) W2b[p - MLP_W2] = f2bf(w);
  else if (p >= MLP_W3 && p < MLP_W3 + MLP_HID * MLP_OUT) W3b[p - MLP_W3] = f2bf(w);
}

// Per-feature mean and 1/std over N rows (float64 sums, one block per feature).
__global__ void k_mlp_stats(const float* __restrict__ X, int N, float* __restrict__ mean,
                            float* __restrict__ istd) {
  __shared__ double red[WG];
  const int c = blockIdx.x;
  double s = 0.0, s2 = 0.0;
  for (int r = threadIdx.x; r < N; r += WG) {
    const double v = X[(size_t)r * MLP_IN + c];
    s += v;
    s2 += v * v;
  }
  const double S = block_sum<WG>(s, red);
  __syncthreads();
  const double S2 = block_sum<WG>(s2, red);
  if (threadIdx.x == 0) {
    const double mu = N > 0 ? S / N : 0.0;
    const double var = N > 0 ? fmax(S2 / N - mu * mu, 0.0) : 0.0;
    const double sd = sqrt(var);
    mean[c] = (float)mu;
    istd[c] = (float)(sd > 1e-12 ? 1.0 / sd : 1.0);
  }
}

constexpr int FEAT_G = FEAT_LANES;

// Features of free vertex j of one mesh at the predictor xt (internal order)
// with x0 the start-of-step positions, computed by G lanes that share j: the
// lanes split the neighbour list and the incident elements, then combine by
// shuffles.  The diagonal Hessian block comes from the element store of an
// element-Hessian pass at xt (estore, s_el times each element's packed
// blocks, in the step's precision T), so no projected Hessian is evaluated
// here.  Every lane of the group must call it (j may be past the free range:
// the group then contributes nothing and writes nothing).
template <int G, typename T>
__device__ __forceinline__ void features_group(const MeshView& mv, int j, int lane,
                                               const double* __restrict__ xt, const double* __restrict__ x0,
                                               double h, double E, const T* __restrict__ estore, double s_el,
                                               double ell, const int* __restrict__ nptr,
                                               const int* __restrict__ nidx,
                                               const double* __restrict__ Xr, float* __restrict__ out) {
  constexpr int D = 3;
  const int n = mv.n;
  const bool valid = j < mv.nf;
  double f[16];
  // relative predictor displacement and velocity
  double mu_[3] = {0, 0, 0};
  int a0 = 0, a1 = 0;
  if (valid) { a0 = nptr[j]; a1 = nptr[j + 1]; }
  for (int t = a0 + lane; t < a1; t += G) {
    const int k = nidx[t];
#pragma unroll
    for (int c = 0; c < D; ++c) mu_[c] += xt[c * n + k] - Xr[c * n + k];
  }
  // diagonal Hessian block and strain statistics over the star
  double Hd[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double wsum = 0, ic_m = 0, j_m = 0, jmin = 1e300, icmax = -1e300;
  int s0 = 0, s1 = 0;
  if (valid) { s0 = mv.star_ptr[j]; s1 = mv.star_ptr[j + 1]; }
  for (int t = s0 + lane; t < s1; t += G) {
    const int e = mv.star[t] >> 2, a = mv.star[t] & 3;
    double F[3][3], beta[4][3], vol;
    load_element<double, 3>(mv, e, xt, F, beta, vol);
    const T* blk = estore + ((size_t)pidx<4>(a, a) * mv.m + e) * 9;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) Hd[r][c] += (double)blk[r * 3 + c];
    double ic = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) ic += F[r][q] * F[r][q];
    ic -= 3.0;
    const double J = det<double, 3>(F);
    wsum += vol;
    ic_m += vol * ic;
    j_m += vol * (J - 1.0);
    jmin = fmin(jmin, J);
    icmax = fmax(icmax, ic);
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) mu_[c] += __shfl_xor(mu_[c], off, G);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Hd[r][c] += __shfl_xor(Hd[r][c], off, G);
      wsum += __shfl_xor(wsum, off, G);
      ic_m += __shfl_xor(ic_m, off, G);
      j_m += __shfl_xor(j_m, off, G);
      jmin = fmin(jmin, __shfl_xor(jmin, off, G));
      icmax = fmax(icmax, __shfl_xor(icmax, off, G));
    }
  }
  if (!valid || lane != 0) return;
  const double inv = a1 > a0 ? 1.0 / (a1 - a0) : 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    f[c] = ((xt[c * n + j] - Xr[c * n + j]) - mu_[c] * inv) / ell;
    f[3 + c] = (xt[c * n + j] - x0[c * n + j]) / ell;
  }
  const double mj = mv.mass[j];
  const double scale = mj + h * h * E * ell;
  const double hs = h * h / s_el;                 // h^2 H_e from the stored s_el H_e
  const int up[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int r = up[q][0], c = up[q][1];
    f[6 + q] = ((r == c ? mj : 0.0) + hs * Hd[r][c]) / scale;
  }
  f[12] = ic_m / wsum;
  f[13] = j_m / wsum;
  f[14] = jmin;
  f[15] = icmax;
#pragma unroll
  for (int q = 0; q < 16; ++q) out[q] = (float)f[q];
}

// rowmap: null -> row j (internal order), else row rowmap[j]
template <typename T>
__global__ void __launch_bounds__(WG) k_features(MeshView mv, const double* __restrict__ xt,
                                                 const double* __restrict__ x0, double h, double E,
                                                 const T* __restrict__ estore, double s_el, double ell,
                                                 const int* __restrict__ nptr, const int* __restrict__ nidx,
                                                 const double* __restrict__ Xr, float* __restrict__ out,
                                                 const int* __restrict__ rowmap) {
  const int j = blockIdx.x * (WG / FEAT_G) + threadIdx.x / FEAT_G;
  const int row = (j < mv.nf) ? (rowmap ? rowmap[j] : j) : 0;
  features_group<FEAT_G, T>(mv, j, threadIdx.x % FEAT_G, xt, x0, h, E, estore, s_el, ell, nptr, nidx, Xr,
                            out + (size_t)row * 16);
}

// x_prop = xt + corr + ds * ell * Delta on free vertices (corr: the last
// step's correction; ds = 1 the network's proposal, 0 the correction alone),
// xt on Dirichlet ones.
__global__ void k_proposal(int n, int nf, const double* __restrict__ xt, const double* __restrict__ corr,
                           const float* __restrict__ delta, double ell, double ds, double* __restrict__ xp) {
  const int v = blockIdx.x * WG + threadIdx.x;
  if (v >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    xp[c * n + v] = xt[c * n + v] +
        (v < nf ? corr[c * n + v] + (ds != 0.0 ? ds * ell * (double)delta[(size_t)v * MLP_NOUT + c] : 0.0)
                : 0.0);
}

// The proposal's base x~ + corr (free vertices; x~ on Dirichlet ones), in
// caller order n x 3.
__global__ void k_base_user(MeshView mv, const int* __restrict__ vperm, const double* __restrict__ xt,
                            const double* __restrict__ corr, double* __restrict__ xu) {
  const int v = blockIdx.x * WG + threadIdx.x;
  if (v >= mv.n) return;
  const int u = vperm[v], n = mv.n;
#pragma unroll
  for (int c = 0; c < 3; ++c) xu[u * 3 + c] = xt[c * n + v] + (v < mv.nf ? corr[c * n + v] : 0.0);
}

void launch_base_user(const MeshView& mv, const int* vperm, const double* xt, double* x_user, hipStream_t st) {
  k_base_user<<<(mv.n + WG - 1) / WG, WG, 0, st>>>(mv, vperm, xt, mv.corr, x_user);
}

// ---- launchers -----------------------------------------------------------
static MlpDev netdev(const MlpState& s) {
  MlpDev d;
  d.W = s.W; d.W1b = s.W1b; d.W2b = s.W2b; d.W3b = s.W3b; d.mean = s.mean; d.istd = s.istd;
  return d;
}

static int mlp_blocks(int B) {
  const int tiles = (B + 15) / 16;
  int blocks = (tiles + MLP_WAVES - 1) / MLP_WAVES;
  return blocks > MLP_MAX_BLOCKS ? MLP_MAX_BLOCKS : (blocks < 1 ? 1 : blocks);
}

void mlp_refresh_bf16(const MlpState& s, hipStream_t st) {
  k_mlp_to_bf16<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(s.W, s.W1b, s.W2b, s.W3b);
}

void mlp_forward(const MlpState& s, const float* X, int B, float* Y, hipStream_t st) {
  if (B <= 0) return;
  k_mlp_forward<<<mlp_blocks(B), 64 * MLP_WAVES, 0, st>>>(netdev(s), X, B, Y);
}

void mlp_gradient_into(const MlpState& s, const float* X, const float* T, const int* idx, int B, float* grad,
                       float* loss, float* part, float* lpart, hipStream_t st) {
  const int nb = mlp_blocks(B);
  k_mlp_train<<<nb, 64 * MLP_WAVES, 0, st>>>(netdev(s), X, T, idx, B, part, lpart);
  k_mlp_sum<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(part, nb * MLP_WAVES, grad, lpart, loss, B);
}

void mlp_gradient(const MlpState& s, const float* X, const float* T, const int* idx, int B, float* grad,
                  float* loss, hipStream_t st) {
  mlp_gradient_into(s, X, T, idx, B, grad, loss, s.part, s.lpart, st);
}

void mlp_adam(MlpState& s, const float* grad, float lr, hipStream_t st) {
  s.t += 1;
  const float c1 = 1.f - powf(0.9f, (float)s.t), c2 = 1.f - powf(0.999f, (float)s.t);
  k_mlp_adam<<<(MLP_NPARAM + 255) / 256, 256, 0, st>>>(s.W, grad, s.m, s.v, lr, c1, c2, s.W1b, s.W2b, s.W3b);
}

void mlp_stats(MlpState& s, const float* X, int N, hipStream_t st) {
  k_mlp_stats<<<MLP_IN, WG, 0, st>>>(X, N, s.mean, s.istd);
}

void launch_features(const MeshView& mv, const double* xt, const double* x0, double h, double E, int prec,
                     const void* estore, double s_el, double ell, const int* nptr, const int* nidx,
                     const double* Xr, float* out, const int* rowmap, hipStream_t st) {
  if (mv.nf <= 0) return;
  const int nb = (mv.nf + WG / FEAT_G - 1) / (WG / FEAT_G);
  if (prec == 0)
    k_features<double><<<nb, WG, 0, st>>>(mv, xt, x0, h, E, (const double*)estore, s_el, ell, nptr, nidx, Xr,
                                          out, rowmap);
  else
    k_features<float><<<nb, WG, 0, st>>>(mv, xt, x0, h, E, (const float*)estore, s_el, ell, nptr, nidx, Xr,
                                         out, rowmap);
}

// Training targets (x_new - x_tilde) / ell of the free vertices, caller-order
// inputs, rows rowmap[j].
__global__ void k_targets(MeshView mv, const double* __restrict__ xn, const double* __restrict__ xt,
                          double ell, const int* __restrict__ rowmap, float* __restrict__ T) {
  const int j = blockIdx.x * WG + threadIdx.x;
  if (j >= mv.nf) return;
  const int u = mv.vperm[j];
#pragma unroll
  for (int c = 0; c < 3; ++c) T[(size_t)rowmap[j] * MLP_NOUT + c] = (float)((xn[u * 3 + c] - xt[u * 3 + c]) / ell);
}

void launch_targets(const MeshView& mv, const double* xn, const double* xt, double ell, const int* rowmap,
                    float* T, hipStream_t st) {
  if (mv.nf <= 0) return;
  k_targets<<<(mv.nf + WG - 1) / WG, WG, 0, st>>>(mv, xn, xt, ell, rowmap, T);
}

void launch_proposal(int n, int nf, const double* xt, const double* corr, const float* delta, double ell,
                     double ds, double* xp, hipStream_t st) {
  k_proposal<<<(n + WG - 1) / WG, WG, 0, st>>>(n, nf, xt, corr, delta, ell, ds, xp);
}

// ---- warm start of a batch (all meshes per launch, no host round trip) ------
template <typename T>
__global__ void __launch_bounds__(WG) kb_features(const BatchItem* __restrict__ items,
                                                  const BatchCtl* __restrict__ ctl,
                                                  const int* __restrict__ boff, int nmesh,
                                                  float* __restrict__ feat) {
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const int j = (blockIdx.x - boff[mi]) * (WG / FEAT_G) + threadIdx.x / FEAT_G;
  features_group<FEAT_G, T>(mv, j, threadIdx.x % FEAT_G, it.x, it.x0, sqrt(it.mat.s_el), it.youngs,
                            (const T*)it.estore, it.mat.s_el, it.ell, it.nptr, it.nidx, it.Xr,
                            feat + (size_t)(it.feat_off + (j < mv.nf ? j : 0)) * MLP_IN);
}

__global__ void __launch_bounds__(WG) kb_proposal(const BatchItem* __restrict__ items,
                                                  const BatchCtl* __restrict__ ctl,
                                                  const int* __restrict__ boff, int nmesh,
                                                  const float* __restrict__ delta, double ds) {
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const int n = it.mv.n, nf = it.mv.nf;
  const int v = (blockIdx.x - boff[mi]) * WG + threadIdx.x;
  if (v >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    it.xtrial[c * n + v] = it.xt[c * n + v] +
        (v < nf ? it.mv.corr[c * n + v] +
                      (ds != 0.0 ? ds * it.ell * (double)delta[(size_t)(it.feat_off + v) * MLP_NOUT + c] : 0.0)
                : 0.0);
}

// Learned warm start of every mesh of the batch: features, the network, the
// proposal x~ + c + l Delta, then its energy with the accept rule (it
// replaces the predictor only at a lower step energy); then the previous
// correction alone, x~ + c, which replaces the start only below the energy
// of the start so far; where either was accepted, the gradient and residual
// test.
void batch_warm_start(BatchPlan* p, const MlpState& net, float* feat, float* delta, int rows,
                      hipStream_t s) {
  const BatchGrid g = batch_grid(p);
  BatchItem* items = batch_items_dev(p);
  BatchCtl* ctl = batch_ctl_dev(p);
  if (g.pred_blocks == 0) return;
  if (g.feat_blocks > 0) {
    // element Hessians at the predictor: the features' diagonal blocks (the
    // first iteration evaluates them again at its start)
    batch_elem_hess_x(p, s);
    if (g.prec == 0)
      kb_features<double><<<g.feat_blocks, WG, 0, s>>>(items, ctl, g.feat_off, g.nmesh, feat);
    else
      kb_features<float><<<g.feat_blocks, WG, 0, s>>>(items, ctl, g.feat_off, g.nmesh, feat);
  }
  mlp_forward(net, feat, rows, delta, s);
  kb_proposal<<<g.pred_blocks, WG, 0, s>>>(items, ctl, g.pred_off, g.nmesh, delta, 1.0);
  if (!g.line_search) batch_energy_x(p, s);   // with line search batch_begin computed it
  batch_energy_trial(p, s, 3);     // E(proposal), then the accept rule
  kb_proposal<<<g.pred_blocks, WG, 0, s>>>(items, ctl, g.pred_off, g.nmesh, delta, 0.0);
  batch_energy_trial(p, s, 5);     // E(x~ + c) against the start so far
  // gradient and residual test at an accepted proposal; a rejected one
  // leaves x, g and |g| at the predictor (r = 1 from the step start)
  batch_gradient_x(p, s, 1, 4);
}

}  // namespace cc
