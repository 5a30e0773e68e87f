// Exact perturbation basis on the GPU.
//
// With Z = H^{-1} (H the rest Hessian over free DOFs), the basis of vertex i
// is U_i[j] = Z_ji Z_ii^{-1}: [I; U_i] spans the columns of Z belonging to
// vertex i, which is U_i = -H_CC^{-1} H_Ci.  Z is formed by an in-place
// blocked Gauss-Jordan inversion of the dense H (symmetric positive definite,
// so the diagonal pivot blocks stay invertible without pivoting):
//
//   for every 64-wide block K:  P = A_KK^{-1};  R = P A_K*;  C = A_*K;
//                               A_IJ -= C_I R_J (I, J != K);  A_IK = -C_I P;
//                               A_KJ = R_J;  A_KK = P.
//
// The dense matrix is column-major-free: row-major N x N float64.

#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "cc_device.h"

namespace cc {

constexpr int GJ_B = 64;   // pivot block width
constexpr int GJ_T = 64;   // update tile (GJ_T x GJ_T outputs per workgroup)

// Dense H from the block rows (internal free order); A must be zeroed first.
template <int D>
__global__ void k_dense_from_blocks(MeshView mv, const double* __restrict__ hb, double* __restrict__ A,
                                    int N) {
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t >= mv.nnzb) return;
  const int j = mv.blkrow[t], k = mv.colidx[t];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) A[(size_t)(j * D + r) * N + k * D + c] = hb[(size_t)t * D * D + r * D + c];
}

// P = A_KK^{-1} by Gauss-Jordan in LDS (one workgroup, b <= 64); writes P to
// Pout (b x b) and a copy of the old column block C = A_*K to Cbuf (N x b).
__global__ void __launch_bounds__(WG) k_gj_pivot(double* __restrict__ A, int N, int k0, int b,
                                                 double* __restrict__ Pout, double* __restrict__ Cbuf,
                                                 int* __restrict__ bad) {
  __shared__ double M[GJ_B][GJ_B + 1];
  __shared__ double piv;
  for (int e = threadIdx.x; e < b * b; e += WG) M[e / b][e % b] = A[(size_t)(k0 + e / b) * N + k0 + e % b];
  __syncthreads();
  for (int p = 0; p < b; ++p) {
    if (threadIdx.x == 0) {
      piv = M[p][p];
      if (!(piv > 0.0)) { atomicOr(bad, 1); piv = 1.0; }
    }
    __syncthreads();
    const double ip = 1.0 / piv;
    // scale row p, then eliminate column p from the other rows (in-place GJ)
    if (threadIdx.x < b) M[p][threadIdx.x] = (threadIdx.x == p) ? ip : M[p][threadIdx.x] * ip;
    __syncthreads();
    for (int e = threadIdx.x; e < b * b; e += WG) {
      const int r = e / b, c = e % b;
      if (r == p) continue;
      const double f = M[r][p];
      if (c == p) continue;
      M[r][c] -= f * M[p][c];
    }
    __syncthreads();
    if (threadIdx.x < b && threadIdx.x != p) M[threadIdx.x][p] = -M[threadIdx.x][p] * ip;
    __syncthreads();
  }
  for (int e = threadIdx.x; e < b * b; e += WG) Pout[e] = M[e / b][e % b];
  (void)Cbuf;
}

// Copy of the old column block C = A_*K (N x b), before it is overwritten.
__global__ void __launch_bounds__(WG) k_gj_copycol(const double* __restrict__ A, int N, int k0, int b,
                                                   double* __restrict__ Cbuf) {
  const size_t total = (size_t)N * b;
  for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < total; e += (size_t)gridDim.x * WG) {
    const size_t r = e / b;
    const int c = (int)(e % b);
    Cbuf[e] = A[r * N + k0 + c];
  }
}

// Row block K: A_KJ <- P A_KJ for every column J outside the pivot block.
__global__ void __launch_bounds__(WG) k_gj_rowscale(double* __restrict__ A, int N, int k0, int b,
                                                    const double* __restrict__ P) {
  __shared__ double Ps[GJ_B][GJ_B + 1];
  __shared__ double Rs[GJ_B][GJ_B + 1];
  for (int e = threadIdx.x; e < b * b; e += WG) Ps[e / b][e % b] = P[e];
  const int c0 = blockIdx.x * GJ_B;   // column chunk
  for (int e = threadIdx.x; e < b * GJ_B; e += WG) {
    const int r = e / GJ_B, c = e % GJ_B;
    Rs[r][c] = (c0 + c < N) ? A[(size_t)(k0 + r) * N + c0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < b * GJ_B; e += WG) {
    const int r = e / GJ_B, c = e % GJ_B;
    const int col = c0 + c;
    if (col >= N || (col >= k0 && col < k0 + b)) continue;
    double s = 0.0;
    for (int q = 0; q < b; ++q) s += Ps[r][q] * Rs[q][c];
    A[(size_t)(k0 + r) * N + col] = s;
  }
}

// Rank-b update of every tile outside the pivot row/column block:
// A_IJ -= C_I R_J with C the saved old column block and R the scaled row block.
__global__ void __launch_bounds__(WG) k_gj_update(double* __restrict__ A, int N, int k0, int b,
                                                  const double* __restrict__ Cbuf) {
  __shared__ double Cs[GJ_T][GJ_B + 1];
  __shared__ double Rs[GJ_B][GJ_T + 1];
  const int ti = blockIdx.y * GJ_T, tj = blockIdx.x * GJ_T;
  for (int e = threadIdx.x; e < GJ_T * b; e += WG) {
    const int r = e / b, q = e % b;
    Cs[r][q] = (ti + r < N) ? Cbuf[(size_t)(ti + r) * b + q] : 0.0;
  }
  for (int e = threadIdx.x; e < b * GJ_T; e += WG) {
    const int q = e / GJ_T, c = e % GJ_T;
    Rs[q][c] = (tj + c < N) ? A[(size_t)(k0 + q) * N + tj + c] : 0.0;
  }
  __syncthreads();
  // 256 threads, 4 x 4 outputs each
  const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  for (int q = 0; q < b; ++q) {
    double cr[4], rc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { cr[u] = Cs[tr + u][q]; rc[u] = Rs[q][tc + u]; }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[u][w] += cr[u] * rc[w];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = ti + tr + u;
    if (r >= N || (r >= k0 && r < k0 + b)) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = tj + tc + w;
      if (c >= N || (c >= k0 && c < k0 + b)) continue;
      A[(size_t)r * N + c] -= acc[u][w];
    }
  }
}

// Column block: A_IK = -C_I P for I outside the pivot block; A_KK = P.
__global__ void __launch_bounds__(WG) k_gj_colfix(double* __restrict__ A, int N, int k0, int b,
                                                  const double* __restrict__ P,
                                                  const double* __restrict__ Cbuf) {
  __shared__ double Ps[GJ_B][GJ_B + 1];
  for (int e = threadIdx.x; e < b * b; e += WG) Ps[e / b][e % b] = P[e];
  __syncthreads();
  const int r0 = blockIdx.x * (WG / GJ_B) * 1;
  (void)r0;
  const size_t total = (size_t)N * b;
  for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < total; e += (size_t)gridDim.x * WG) {
    const int r = (int)(e / b), c = (int)(e % b);
    if (r >= k0 && r < k0 + b) {
      A[(size_t)r * N + k0 + c] = Ps[r - k0][c];
    } else {
      double s = 0.0;
      for (int q = 0; q < b; ++q) s += Cbuf[(size_t)r * b + q] * Ps[q][c];
      A[(size_t)r * N + k0 + c] = -s;
    }
  }
}

// U_i[j] = Z_ji Z_ii^{-1} for every free i and j != i, written in the dense
// internal layout (row i holds every other free vertex in ascending order).
template <int D>
__global__ void k_basis_from_inverse(const double* __restrict__ Z, int nf, double* __restrict__ Ud,
                                     float* __restrict__ Uf) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * WG + threadIdx.x;
  if (j >= nf || j == i) return;
  const int N = nf * D;
  double Zi[D][D], Zinv[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) Zi[r][c] = Z[(size_t)(i * D + r) * N + i * D + c];
  if constexpr (D == 2) {
    const double det = Zi[0][0] * Zi[1][1] - Zi[0][1] * Zi[1][0];
    Zinv[0][0] = Zi[1][1] / det; Zinv[0][1] = -Zi[0][1] / det;
    Zinv[1][0] = -Zi[1][0] / det; Zinv[1][1] = Zi[0][0] / det;
  } else {
    const double det = Zi[0][0] * (Zi[1][1] * Zi[2][2] - Zi[1][2] * Zi[2][1]) -
                       Zi[0][1] * (Zi[1][0] * Zi[2][2] - Zi[1][2] * Zi[2][0]) +
                       Zi[0][2] * (Zi[1][0] * Zi[2][1] - Zi[1][1] * Zi[2][0]);
    Zinv[0][0] = (Zi[1][1] * Zi[2][2] - Zi[1][2] * Zi[2][1]) / det;
    Zinv[0][1] = (Zi[0][2] * Zi[2][1] - Zi[0][1] * Zi[2][2]) / det;
    Zinv[0][2] = (Zi[0][1] * Zi[1][2] - Zi[0][2] * Zi[1][1]) / det;
    Zinv[1][0] = (Zi[1][2] * Zi[2][0] - Zi[1][0] * Zi[2][2]) / det;
    Zinv[1][1] = (Zi[0][0] * Zi[2][2] - Zi[0][2] * Zi[2][0]) / det;
    Zinv[1][2] = (Zi[0][2] * Zi[1][0] - Zi[0][0] * Zi[1][2]) / det;
    Zinv[2][0] = (Zi[1][0] * Zi[2][1] - Zi[1][1] * Zi[2][0]) / det;
    Zinv[2][1] = (Zi[0][1] * Zi[2][0] - Zi[0][0] * Zi[2][1]) / det;
    Zinv[2][2] = (Zi[0][0] * Zi[1][1] - Zi[0][1] * Zi[1][0]) / det;
  }
  const size_t q = (size_t)i * (nf - 1) + (j < i ? j : j - 1);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) s += Z[(size_t)(j * D + r) * N + i * D + l] * Zinv[l][c];
      Ud[q * D * D + r * D + c] = s;
      Uf[q * D * D + r * D + c] = (float)s;
    }
}

// Whole build: hb (float64 rest block rows) -> U (dense internal rows).
// A: N*N doubles, work: N*GJ_B + GJ_B*GJ_B doubles.  Returns false when a
// pivot block is not positive definite.
bool exact_basis_gpu(const MeshView& mv, const double* hb, double* A, double* work, int* bad, double* Ud,
                     float* Uf, hipStream_t s) {
  const int D = mv.D, nf = mv.nf, N = nf * D;
  (void)hipMemsetAsync(A, 0, (size_t)N * N * sizeof(double), s);
  (void)hipMemsetAsync(bad, 0, sizeof(int), s);
  if (mv.nnzb > 0) {
    const int nb = (mv.nnzb + WG - 1) / WG;
    if (D == 2) k_dense_from_blocks<2><<<nb, WG, 0, s>>>(mv, hb, A, N);
    else k_dense_from_blocks<3><<<nb, WG, 0, s>>>(mv, hb, A, N);
  }
  double* P = work;
  double* C = work + GJ_B * GJ_B;
  const int tiles = (N + GJ_T - 1) / GJ_T;
  for (int k0 = 0; k0 < N; k0 += GJ_B) {
    const int b = (N - k0) < GJ_B ? (N - k0) : GJ_B;
    const int cgrid = (int)std::min<size_t>(((size_t)N * b + WG - 1) / WG, 4096);
    k_gj_pivot<<<1, WG, 0, s>>>(A, N, k0, b, P, C, bad);
    k_gj_copycol<<<cgrid, WG, 0, s>>>(A, N, k0, b, C);
    k_gj_rowscale<<<(N + GJ_B - 1) / GJ_B, WG, 0, s>>>(A, N, k0, b, P);
    k_gj_update<<<dim3(tiles, tiles), WG, 0, s>>>(A, N, k0, b, C);
    k_gj_colfix<<<(int)(((size_t)N * b + WG - 1) / WG < 4096 ? ((size_t)N * b + WG - 1) / WG : 4096), WG, 0, s>>>(
        A, N, k0, b, P, C);
  }
  if (nf > 1) {
    const dim3 g((nf + WG - 1) / WG, nf);
    if (D == 2) k_basis_from_inverse<2><<<g, WG, 0, s>>>(A, nf, Ud, Uf);
    else k_basis_from_inverse<3><<<g, WG, 0, s>>>(A, nf, Ud, Uf);
  }
  int hbad = 0;
  (void)hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
  return hbad == 0;
}

}  // namespace cc
