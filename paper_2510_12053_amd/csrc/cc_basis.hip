// Exact perturbation basis on the GPU.
//
// With Z = H^{-1} (H the step Hessian over free DOFs), the basis of vertex i
// is U_i[j] = Z_ji Z_ii^{-1}: [I; U_i] spans the columns of Z belonging to
// vertex i, which is U_i = -H_CC^{-1} H_Ci (Method, Coordinate Condensation;
// Background, JGS2).
//
// In band order (breadth-first levels, MeshView::bvert) H is block
// tridiagonal: a block (j, k) couples vertices of the same or of adjacent
// levels.  With D_l = H_ll and B_l = H_{l,l-1} the block LDL^T factorisation
//   S_0 = D_0,  F_l = B_l S_{l-1}^{-1},  S_l = D_l - F_l B_l^T
// gives H = L diag(S) L^T with L unit lower block bidiagonal (L_{l,l-1} = F_l).
// The columns of Z that belong to level q (a "panel") then follow from
//   forward:   Y_q = I,  Y_l = -F_l Y_{l-1}            (l > q; zero above q)
//   diagonal:  Z_l = S_l^{-1} Y_l                        (l >= q)
//   backward:  X_l = Z_l - F_{l+1}^T X_{l+1}             (every l, Z_l = 0 above q)
// and X is column block q of Z = H^{-1}, from which the basis rows of level
// q's vertices are formed directly.  The cost is O(N^2 n) for levels of n
// DOFs instead of the O(N^3) of a dense inverse, the memory O(N n) besides
// the basis itself.  S_l^{-1} comes from an in-place blocked Gauss-Jordan
// inversion (SPD, so its diagonal pivot blocks need no pivoting):
//
//   for every 64-wide block K:  P = A_KK^{-1};  R = P A_K*;  C = A_*K;
//                               A_IJ -= C_I R_J (I, J != K);  A_IK = -C_I P;
//                               A_KJ = R_J;  A_KK = P.
//
// Dense matrices are row-major float64.

#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "cc_device.h"

namespace cc {

constexpr int GJ_B = 64;   // pivot block width
constexpr int GJ_T = 64;   // update tile (GJ_T x GJ_T outputs per workgroup)

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

// In-place inverse of the SPD matrix A (N x N); *bad set when a pivot is
// not positive.  work: N * GJ_B + GJ_B^2 doubles.
static void gj_inverse(double* A, int N, double* work, int* bad, hipStream_t s) {
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
    k_gj_colfix<<<cgrid, WG, 0, s>>>(A, N, k0, b, P, C);
  }
}

// C (M x N) = alpha op(A) op(B) + beta C, row-major float64, op = transpose
// when TA / TB.  64 x 64 output tiles, 4 x 4 per thread, K in steps of 16
// through LDS.  With beta = 0, C is not read.
constexpr int MM_T = 64, MM_K = 16;
template <bool TA, bool TB>
__global__ void __launch_bounds__(WG) k_dgemm(int M, int N, int K, double alpha,
                                              const double* __restrict__ A, int lda,
                                              const double* __restrict__ B, int ldb, double beta,
                                              double* __restrict__ C, int ldc) {
  __shared__ double As[MM_K][MM_T + 2];
  __shared__ double Bs[MM_K][MM_T + 2];
  const int m0 = blockIdx.y * MM_T, n0 = blockIdx.x * MM_T, tid = threadIdx.x;
  const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
  for (int k0 = 0; k0 < K; k0 += MM_K) {
#pragma unroll
    for (int u = 0; u < MM_T * MM_K / WG; ++u) {
      const int e = tid + u * WG;
      // consecutive threads walk the contiguous index of each operand
      const int ma = TA ? e % MM_T : e / MM_K, ka = TA ? e / MM_T : e % MM_K;
      const int gm = m0 + ma, gka = k0 + ka;
      double va = 0.0;
      if (gm < M && gka < K) va = TA ? A[(size_t)gka * lda + gm] : A[(size_t)gm * lda + gka];
      As[ka][ma] = va;
      const int nb = TB ? e / MM_K : e % MM_T, kb = TB ? e % MM_K : e / MM_T;
      const int gn = n0 + nb, gkb = k0 + kb;
      double vb = 0.0;
      if (gn < N && gkb < K) vb = TB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn];
      Bs[kb][nb] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < MM_K; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { a[u] = As[kk][tr + u]; b[u] = Bs[kk][tc + u]; }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] += a[u] * b[w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = m0 + tr + u;
    if (r >= M) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = n0 + tc + w;
      if (c >= N) continue;
      double* o = C + (size_t)r * ldc + c;
      *o = beta == 0.0 ? alpha * acc[u][w] : alpha * acc[u][w] + beta * *o;
    }
  }
}

static void dgemm(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                  const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const dim3 grid((N + MM_T - 1) / MM_T, (M + MM_T - 1) / MM_T);
  if (!ta && !tb) k_dgemm<false, false><<<grid, WG, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (!ta && tb) k_dgemm<false, true><<<grid, WG, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (ta && !tb) k_dgemm<true, false><<<grid, WG, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else k_dgemm<true, true><<<grid, WG, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

// dst (rows x cols, leading dimension ldd) = alpha src (leading dimension lds)
__global__ void __launch_bounds__(WG) k_scale_copy(double* __restrict__ dst, int ldd,
                                                   const double* __restrict__ src, int lds, int rows,
                                                   int cols, double alpha) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = (size_t)blockIdx.x * WG + threadIdx.x; e < total; e += (size_t)gridDim.x * WG) {
    const size_t r = e / cols, c = e % cols;
    dst[r * ldd + c] = alpha * src[r * lds + c];
  }
}

static void scale_copy(double* dst, int ldd, const double* src, int lds, int rows, int cols, double alpha,
                       hipStream_t s) {
  const size_t total = (size_t)rows * cols;
  if (total == 0) return;
  const int grid = (int)std::min<size_t>((total + WG - 1) / WG, 8192);
  k_scale_copy<<<grid, WG, 0, s>>>(dst, ldd, src, lds, rows, cols, alpha);
}

// Level blocks D_l = H_ll and B_l = H_{l,l-1} from the block rows (both zeroed
// first); lev: level of every band position, loff: first band position of
// every level, oD / oB: offsets of the levels' blocks in Dbuf / Bbuf.
template <int D>
__global__ void k_level_scatter(MeshView mv, const double* __restrict__ hb, const int* __restrict__ lev,
                                const int* __restrict__ loff, const size_t* __restrict__ oD,
                                const size_t* __restrict__ oB, double* __restrict__ Dbuf,
                                double* __restrict__ Bbuf) {
  constexpr int DD = D * D;
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t >= mv.nnzb) return;
  const int pj = mv.bpos[mv.blkrow[t]], pk = mv.bpos[mv.colidx[t]];
  const int lj = lev[pj], lk = lev[pk];
  const int nl = (loff[lj + 1] - loff[lj]) * D;
  double* dst;
  int ld, r0, c0;
  if (lk == lj) {
    dst = Dbuf + oD[lj]; ld = nl; r0 = (pj - loff[lj]) * D; c0 = (pk - loff[lj]) * D;
  } else if (lk == lj - 1) {
    dst = Bbuf + oB[lj]; ld = (loff[lk + 1] - loff[lk]) * D; r0 = (pj - loff[lj]) * D; c0 = (pk - loff[lk]) * D;
  } else {
    return;   // lk == lj + 1: the transpose of B_lk
  }
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) dst[(size_t)(r0 + r) * ld + c0 + c] = hb[(size_t)t * DD + r * D + c];
}

// Basis rows of the vertices of level q from X = column block q of Z (N x nq,
// rows in band DOF order): U_i[p] = X_p,a X_a,a^{-1} for the level's a-th
// vertex i, zero at its own position.
template <int D>
__global__ void k_basis_from_panel(const double* __restrict__ X, int nq, int q0, int nf,
                                   const int* __restrict__ bvert, double* __restrict__ Ud,
                                   float* __restrict__ Uf) {
  constexpr int DD = D * D;
  const int a = blockIdx.y;
  const int p = blockIdx.x * WG + threadIdx.x;
  if (p >= nf) return;
  const int pa = q0 + a, i = bvert[pa];
  const size_t o = ((size_t)i * nf + p) * DD;
  if (p == pa) {
#pragma unroll
    for (int r = 0; r < DD; ++r) {
      if (Ud) Ud[o + r] = 0.0;
      Uf[o + r] = 0.f;
    }
    return;
  }
  double Zi[D][D], Zinv[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) Zi[r][c] = X[(size_t)(pa * D + r) * nq + a * D + c];
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
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) acc += X[(size_t)(p * D + r) * nq + a * D + l] * Zinv[l][c];
      if (Ud) Ud[o + r * D + c] = acc;
      Uf[o + r * D + c] = (float)acc;
    }
}

int exact_basis_band(const MeshView& mv, const double* hb, const int* loff_h, int L, double* Ud, float* Uf,
                     hipStream_t s) {
  const int D = mv.D, nf = mv.nf, N = nf * D;
  if (nf < 1) return 0;
  std::vector<int> n(L), lev(nf);
  std::vector<size_t> oD(L + 1, 0), oB(L + 1, 0);
  int nmax = 0;
  for (int l = 0; l < L; ++l) {
    n[l] = (loff_h[l + 1] - loff_h[l]) * D;
    nmax = std::max(nmax, n[l]);
    for (int p = loff_h[l]; p < loff_h[l + 1]; ++p) lev[p] = l;
    oD[l + 1] = oD[l] + (size_t)n[l] * n[l];
    oB[l + 1] = oB[l] + (l > 0 ? (size_t)n[l] * n[l - 1] : 0);
  }
  double *Dbuf = nullptr, *Bbuf = nullptr, *tmp = nullptr, *P = nullptr, *Q = nullptr, *work = nullptr;
  size_t *oD_d = nullptr, *oB_d = nullptr;
  int *lev_d = nullptr, *loff_d = nullptr, *bad = nullptr;
  auto release = [&]() {
    for (void* q : {(void*)Dbuf, (void*)Bbuf, (void*)tmp, (void*)P, (void*)Q, (void*)work, (void*)oD_d,
                    (void*)oB_d, (void*)lev_d, (void*)loff_d, (void*)bad})
      if (q) (void)hipFree(q);
  };
  bool ok = hipMalloc(&Dbuf, std::max<size_t>(oD[L], 1) * 8) == hipSuccess &&
            hipMalloc(&Bbuf, std::max<size_t>(oB[L], 1) * 8) == hipSuccess &&
            hipMalloc(&tmp, (size_t)nmax * nmax * 8) == hipSuccess &&
            hipMalloc(&P, (size_t)N * nmax * 8) == hipSuccess &&
            hipMalloc(&Q, (size_t)N * nmax * 8) == hipSuccess &&
            hipMalloc(&work, ((size_t)nmax * GJ_B + GJ_B * GJ_B) * 8) == hipSuccess &&
            hipMalloc(&oD_d, (L + 1) * sizeof(size_t)) == hipSuccess &&
            hipMalloc(&oB_d, (L + 1) * sizeof(size_t)) == hipSuccess &&
            hipMalloc(&lev_d, nf * sizeof(int)) == hipSuccess &&
            hipMalloc(&loff_d, (L + 1) * sizeof(int)) == hipSuccess &&
            hipMalloc(&bad, sizeof(int)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    release();
    return 2;
  }
  (void)hipMemcpyAsync(oD_d, oD.data(), (L + 1) * sizeof(size_t), hipMemcpyHostToDevice, s);
  (void)hipMemcpyAsync(oB_d, oB.data(), (L + 1) * sizeof(size_t), hipMemcpyHostToDevice, s);
  (void)hipMemcpyAsync(lev_d, lev.data(), nf * sizeof(int), hipMemcpyHostToDevice, s);
  (void)hipMemcpyAsync(loff_d, loff_h, (L + 1) * sizeof(int), hipMemcpyHostToDevice, s);
  (void)hipMemsetAsync(Dbuf, 0, std::max<size_t>(oD[L], 1) * 8, s);
  (void)hipMemsetAsync(Bbuf, 0, std::max<size_t>(oB[L], 1) * 8, s);
  (void)hipMemsetAsync(bad, 0, sizeof(int), s);
  if (mv.nnzb > 0) {
    const int nb = (mv.nnzb + WG - 1) / WG;
    if (D == 2) k_level_scatter<2><<<nb, WG, 0, s>>>(mv, hb, lev_d, loff_d, oD_d, oB_d, Dbuf, Bbuf);
    else k_level_scatter<3><<<nb, WG, 0, s>>>(mv, hb, lev_d, loff_d, oD_d, oB_d, Dbuf, Bbuf);
  }
  // block LDL^T: S_l in place of D_l (then inverted in place), F_l in place of B_l
  for (int l = 0; l < L; ++l) {
    double* Dl = Dbuf + oD[l];
    if (l > 0) {
      double* Bl = Bbuf + oB[l];
      const double* Sprev = Dbuf + oD[l - 1];
      dgemm(false, false, n[l], n[l - 1], n[l - 1], 1.0, Bl, n[l - 1], Sprev, n[l - 1], 0.0, tmp, n[l - 1], s);
      dgemm(false, true, n[l], n[l], n[l - 1], -1.0, tmp, n[l - 1], Bl, n[l - 1], 1.0, Dl, n[l], s);
      scale_copy(Bl, n[l - 1], tmp, n[l - 1], n[l], n[l - 1], 1.0, s);
    }
    gj_inverse(Dl, n[l], work, bad, s);
  }
  int hbad = 0;
  (void)hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
  if (hbad) {
    release();
    return 1;
  }
  // panels: column block q of Z, then the basis rows of level q
  for (int q = 0; q < L; ++q) {
    const int nq = n[q];
    auto rowsP = [&](int l) { return P + (size_t)loff_h[l] * D * nq; };
    auto rowsQ = [&](int l) { return Q + (size_t)loff_h[l] * D * nq; };
    scale_copy(rowsQ(q), nq, Dbuf + oD[q], nq, nq, nq, 1.0, s);                 // Z_q = S_q^{-1}
    if (q + 1 < L) scale_copy(rowsP(q + 1), nq, Bbuf + oB[q + 1], nq, n[q + 1], nq, -1.0, s);  // Y = -F
    for (int l = q + 2; l < L; ++l)
      dgemm(false, false, n[l], nq, n[l - 1], -1.0, Bbuf + oB[l], n[l - 1], rowsP(l - 1), nq, 0.0, rowsP(l), nq, s);
    for (int l = q + 1; l < L; ++l)
      dgemm(false, false, n[l], nq, n[l], 1.0, Dbuf + oD[l], n[l], rowsP(l), nq, 0.0, rowsQ(l), nq, s);
    for (int l = L - 2; l >= 0; --l)
      dgemm(true, false, n[l], nq, n[l + 1], -1.0, Bbuf + oB[l + 1], n[l], rowsQ(l + 1), nq, l >= q ? 1.0 : 0.0,
            rowsQ(l), nq, s);
    const int sq = n[q] / D;
    if (nf > 1 && sq > 0) {
      const dim3 g((nf + WG - 1) / WG, sq);
      if (D == 2) k_basis_from_panel<2><<<g, WG, 0, s>>>(Q, nq, loff_h[q], nf, mv.bvert, Ud, Uf);
      else k_basis_from_panel<3><<<g, WG, 0, s>>>(Q, nq, loff_h[q], nf, mv.bvert, Ud, Uf);
    }
  }
  const hipError_t e = hipStreamSynchronize(s);
  release();
  return e == hipSuccess ? 0 : 2;
}

}  // namespace cc
