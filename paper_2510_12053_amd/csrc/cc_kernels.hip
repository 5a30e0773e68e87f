// gfx950 kernels of the Coordinate Condensation sweep.
//
// Data layout (internal, colour-sorted order; see cc_kernels.h):
//   positions and gradients: float64 structure-of-arrays, component c of
//     vertex v at [c*n + v];
//   element store: per packed local block p (a <= b) an array of m blocks of
//     D*D values, [(p*m + e)*D*D + r*D + s];
//   block rows of the free-free Hessian: CSR over free vertices with the
//     diagonal block first in every row, [slot*D*D + r*D + s];
//   basis: CSR over free vertices, rows sorted by internal id, [q*D*D + ...].
//
// Every reduction is a fixed-order tree (no floating-point atomics), so runs
// are bit-reproducible.

#include <math.h>

#include "cc_kernels.h"

namespace cc {

constexpr int WG = 256;

template <typename T>
__device__ __forceinline__ T csqrt(T v);
template <>
__device__ __forceinline__ float csqrt<float>(float v) { return sqrtf(v); }
template <>
__device__ __forceinline__ double csqrt<double>(double v) { return sqrt(v); }

template <typename T>
__device__ __forceinline__ T cabs(T v) { return v < T(0) ? -v : v; }

// packed index of local block (a, b), a <= b, among K local vertices
template <int K>
__host__ __device__ __forceinline__ int pidx(int a, int b) {
  return a * K - (a * (a - 1)) / 2 + (b - a);
}

template <typename T> __device__ __forceinline__ const T* dinv_of(const MeshView& mv);
template <> __device__ __forceinline__ const float* dinv_of<float>(const MeshView& mv) { return mv.dinv_f; }
template <> __device__ __forceinline__ const double* dinv_of<double>(const MeshView& mv) { return mv.dinv_d; }
template <typename T> __device__ __forceinline__ const T* vol_of(const MeshView& mv);
template <> __device__ __forceinline__ const float* vol_of<float>(const MeshView& mv) { return mv.vol_f; }
template <> __device__ __forceinline__ const double* vol_of<double>(const MeshView& mv) { return mv.vol_d; }
template <typename T> __device__ __forceinline__ const T* basis_of(const MeshView& mv);
template <> __device__ __forceinline__ const float* basis_of<float>(const MeshView& mv) { return mv.U_f; }
template <> __device__ __forceinline__ const double* basis_of<double>(const MeshView& mv) { return mv.U_d; }

// F = sum_{a>=1} (x_a - x_0) beta_a^T, differences formed in float64 then cast.
template <typename T, int D>
__device__ __forceinline__ void load_element(const MeshView& mv, int e, const double* __restrict__ x,
                                             T F[D][D], T beta[D + 1][D], T& vol) {
  const int m = mv.m, n = mv.n;
  const T* dinv = dinv_of<T>(mv);
  const int v0 = mv.ev[e];
  T Ds[D][D];
#pragma unroll
  for (int a = 1; a <= D; ++a) {
    const int va = mv.ev[a * m + e];
#pragma unroll
    for (int c = 0; c < D; ++c) Ds[c][a - 1] = T(x[c * n + va] - x[c * n + v0]);
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int q = 0; q < D; ++q) beta[a + 1][q] = dinv[(a * D + q) * m + e];
#pragma unroll
  for (int q = 0; q < D; ++q) {
    T s = T(0);
#pragma unroll
    for (int a = 1; a <= D; ++a) s += beta[a][q];
    beta[0][q] = -s;
  }
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      T s = T(0);
#pragma unroll
      for (int a = 1; a <= D; ++a) s += Ds[r][a - 1] * beta[a][q];
      F[r][q] = s;
    }
  vol = vol_of<T>(mv)[e];
}

template <typename T, int D>
__device__ __forceinline__ T det(const T F[D][D]) {
  if constexpr (D == 2) {
    return F[0][0] * F[1][1] - F[0][1] * F[1][0];
  } else {
    return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
           F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
           F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  }
}

// dJ/dF: 2D [[F11,-F10],[-F01,F00]]; 3D columns f1 x f2, f2 x f0, f0 x f1.
template <typename T, int D>
__device__ __forceinline__ void cofactor(const T F[D][D], T C[D][D]) {
  if constexpr (D == 2) {
    C[0][0] = F[1][1];
    C[0][1] = -F[1][0];
    C[1][0] = -F[0][1];
    C[1][1] = F[0][0];
  } else {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int a = (q + 1) % 3, b = (q + 2) % 3;
      C[0][q] = F[1][a] * F[2][b] - F[2][a] * F[1][b];
      C[1][q] = F[2][a] * F[0][b] - F[0][a] * F[2][b];
      C[2][q] = F[0][a] * F[1][b] - F[1][a] * F[0][b];
    }
  }
}

// First Piola-Kirchhoff stress of the stable neo-Hookean energy.
template <typename T, int D>
__device__ __forceinline__ void snh_pk1(const T F[D][D], T mu, T lam, T P[D][D]) {
  T C[D][D];
  cofactor<T, D>(F, C);
  const T J = det<T, D>(F);
  const T k = lam * (J - T(1)) - mu;
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int q = 0; q < D; ++q) P[r][q] = mu * F[r][q] + k * C[r][q];
}

template <typename T, int D>
__device__ __forceinline__ T snh_psi(const T F[D][D], T mu, T lam) {
  T f2 = T(0);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int q = 0; q < D; ++q) f2 += F[r][q] * F[r][q];
  const T J = det<T, D>(F);
  return T(0.5) * mu * (f2 - T(D)) - mu * (J - T(1)) + T(0.5) * lam * (J - T(1)) * (J - T(1));
}

// Cyclic Jacobi eigen-decomposition of a symmetric matrix S (overwritten by
// its rotated form, eigenvalues on the diagonal); V accumulates the rotations
// (columns are eigenvectors).  Each rotation zeroes S[p][q] exactly.
template <typename T, int D>
__device__ __forceinline__ void jacobi_eig(T S[D][D], T V[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) V[i][j] = (i == j) ? T(1) : T(0);
  const T eps = sizeof(T) == 4 ? T(1e-7) : T(1e-16);
  const int sweeps = (D == 2) ? 1 : (sizeof(T) == 4 ? 5 : 8);
  for (int sw = 0; sw < sweeps; ++sw) {
    bool any = false;
#pragma unroll
    for (int p = 0; p < D - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < D; ++q) {
        const T apq = S[p][q];
        const T app = S[p][p], aqq = S[q][q];
        if (cabs(apq) <= eps * eps * (cabs(app) + cabs(aqq)) || apq == T(0)) {
          S[p][q] = S[q][p] = T(0);
          continue;
        }
        any = true;
        const T theta = (aqq - app) / (T(2) * apq);
        const T t = (theta >= T(0) ? T(1) : T(-1)) / (cabs(theta) + csqrt(theta * theta + T(1)));
        const T c = T(1) / csqrt(t * t + T(1));
        const T s = t * c;
        S[p][p] = app - t * apq;
        S[q][q] = aqq + t * apq;
        S[p][q] = S[q][p] = T(0);
#pragma unroll
        for (int r = 0; r < D; ++r) {
          if (r == p || r == q) continue;
          const T arp = S[r][p], arq = S[r][q];
          S[r][p] = S[p][r] = c * arp - s * arq;
          S[r][q] = S[q][r] = s * arp + c * arq;
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
          const T vrp = V[r][p], vrq = V[r][q];
          V[r][p] = c * vrp - s * vrq;
          V[r][q] = s * vrp + c * vrq;
        }
      }
    if (!any) break;
  }
}

// Rotation-variant SVD F = U diag(sig) V^T with det U = det V = +1: V from the
// eigenvectors of F^T F (a product of rotations), then a Givens QR of F V.
// The last singular value carries the sign of det F.
template <typename T, int D>
__device__ __forceinline__ void svd_rv(const T F[D][D], T U[D][D], T V[D][D], T sig[D]) {
  T S[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) s += F[k][i] * F[k][j];
      S[i][j] = s;
    }
  jacobi_eig<T, D>(S, V);
  T B[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) s += F[i][k] * V[k][j];
      B[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) U[i][j] = (i == j) ? T(1) : T(0);
#pragma unroll
  for (int k = 0; k < D - 1; ++k)
#pragma unroll
    for (int q = k + 1; q < D; ++q) {
      const T a = B[k][k], b = B[q][k];
      const T r = csqrt(a * a + b * b);
      T c = T(1), s = T(0);
      if (r > T(0)) {
        c = a / r;
        s = b / r;
      }
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const T bp = B[k][j], bq = B[q][j];
        B[k][j] = c * bp + s * bq;
        B[q][j] = -s * bp + c * bq;
      }
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const T up = U[i][k], uq = U[i][q];
        U[i][k] = c * up + s * uq;
        U[i][q] = -s * up + c * uq;
      }
    }
#pragma unroll
  for (int k = 0; k < D; ++k) sig[k] = B[k][k];
}

// Projected stable neo-Hookean Hessian as its positive eigenpairs.  In the
// frame of F = U diag(sig) V^T the Hessian splits into the block coupling the
// diagonal entries (A_kk = mu + lam c_k^2, A_kl = lam c_k c_l + s sig_m with
// c the diagonal cofactors and s = lam (J-1) - mu) and, for every pair k < l,
// a 2x2 block on (F_kl, F_lk) with eigenvalues mu -+ s sig_m (2D: sig_m = 1)
// and eigenvectors (1, +-1)/sqrt(2).  Eigen-matrices map back as
// U E V^T.  callback(weight, Q) is invoked for each eigenpair with weight > 0.
template <typename T, int D, typename CB>
__device__ __forceinline__ void snh_projected_eigs(const T F[D][D], T mu, T lam, CB&& callback) {
  T U[D][D], V[D][D], sig[D];
  svd_rv<T, D>(F, U, V, sig);
  T J = T(1);
#pragma unroll
  for (int k = 0; k < D; ++k) J *= sig[k];
  const T s = lam * (J - T(1)) - mu;
  T A[D][D], c[D], third[D][D];
  if constexpr (D == 2) {
    c[0] = sig[1];
    c[1] = sig[0];
    third[0][1] = third[1][0] = T(1);
  } else {
    c[0] = sig[1] * sig[2];
    c[1] = sig[0] * sig[2];
    c[2] = sig[0] * sig[1];
    third[0][1] = third[1][0] = sig[2];
    third[0][2] = third[2][0] = sig[1];
    third[1][2] = third[2][1] = sig[0];
  }
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int l = 0; l < D; ++l)
      A[k][l] = (k == l) ? mu + lam * c[k] * c[k] : lam * c[k] * c[l] + s * third[k][l];
  T W[D][D];
  jacobi_eig<T, D>(A, W);
  T Q[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r) {
    const T w = A[r][r];
    if (w > T(0)) {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < D; ++k) acc += W[k][r] * U[i][k] * V[j][k];
          Q[i][j] = acc;
        }
      callback(w, Q);
    }
  }
  const T h = T(0.70710678118654752440);
#pragma unroll
  for (int k = 0; k < D - 1; ++k)
#pragma unroll
    for (int l = k + 1; l < D; ++l) {
      const T sm = third[k][l];
#pragma unroll
      for (int sgn = 0; sgn < 2; ++sgn) {
        // sgn 0: vector (1, 1), eigenvalue mu - s sig_m; sgn 1: (1, -1), mu + s sig_m
        const T w = sgn == 0 ? mu - s * sm : mu + s * sm;
        if (!(w > T(0))) continue;
        const T b = sgn == 0 ? h : -h;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) Q[i][j] = h * U[i][k] * V[j][l] + b * U[i][l] * V[j][k];
        callback(w, Q);
      }
    }
}

// ---------------------------------------------------------------------------
// Element Hessian: H_e[a,b] = scale * V_e * sum_r w_r (Q_r beta_a)(Q_r beta_b)^T
template <typename T, int D>
__global__ void __launch_bounds__(WG) k_elem_hess(MeshView mv, const double* __restrict__ x, T mu,
                                                  T lam, T scale, T* __restrict__ out) {
  constexpr int K = D + 1, DD = D * D, NB = K * (K + 1) / 2;
  const int e = blockIdx.x * WG + threadIdx.x;
  if (e >= mv.m) return;
  T F[D][D], beta[K][D], vol;
  load_element<T, D>(mv, e, x, F, beta, vol);
  T acc[NB][DD];
#pragma unroll
  for (int p = 0; p < NB; ++p)
#pragma unroll
    for (int r = 0; r < DD; ++r) acc[p][r] = T(0);
  snh_projected_eigs<T, D>(F, mu, lam, [&](T w, const T (&Q)[D][D]) {
    T y[K][D];
#pragma unroll
    for (int a = 1; a < K; ++a)
#pragma unroll
      for (int r = 0; r < D; ++r) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < D; ++q) s += Q[r][q] * beta[a][q];
        y[a][r] = s;
      }
#pragma unroll
    for (int r = 0; r < D; ++r) {
      T s = T(0);
#pragma unroll
      for (int a = 1; a < K; ++a) s += y[a][r];
      y[0][r] = -s;
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
      T wy[D];
#pragma unroll
      for (int r = 0; r < D; ++r) wy[r] = w * y[a][r];
#pragma unroll
      for (int b = a; b < K; ++b)
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
          for (int s = 0; s < D; ++s) acc[pidx<K>(a, b)][r * D + s] += wy[r] * y[b][s];
    }
  });
  const T f = scale * vol;
  const int m = mv.m;
#pragma unroll
  for (int p = 0; p < NB; ++p)
#pragma unroll
    for (int r = 0; r < DD; ++r) out[((size_t)p * m + e) * DD + r] = f * acc[p][r];
}

// Block rows: every slot sums its element contributions (fixed order), plus
// the mass on the diagonal.
template <typename T, int D>
__global__ void __launch_bounds__(WG) k_assemble(MeshView mv, const T* __restrict__ est, T w_in,
                                                 T* __restrict__ hb) {
  constexpr int K = D + 1, DD = D * D;
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t >= mv.nnzb) return;
  T acc[DD];
#pragma unroll
  for (int r = 0; r < DD; ++r) acc[r] = T(0);
  const int m = mv.m;
  for (int c = mv.cptr[t]; c < mv.cptr[t + 1]; ++c) {
    const int pk = mv.centry[c];
    const int e = pk >> 4, a = (pk >> 2) & 3, b = pk & 3;
    if (a <= b) {
      const T* blk = est + ((size_t)pidx<K>(a, b) * m + e) * DD;
#pragma unroll
      for (int r = 0; r < DD; ++r) acc[r] += blk[r];
    } else {
      const T* blk = est + ((size_t)pidx<K>(b, a) * m + e) * DD;
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = 0; s < D; ++s) acc[r * D + s] += blk[s * D + r];
    }
  }
  const int j = mv.blkrow[t];
  if (mv.colidx[t] == j) {
    const T mj = w_in * T(mv.mass[j]);
#pragma unroll
    for (int r = 0; r < D; ++r) acc[r * D + r] += mj;
  }
#pragma unroll
  for (int r = 0; r < DD; ++r) hb[(size_t)t * DD + r] = acc[r];
}

template <int WGS>
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = WGS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// Free-vertex gradient in float64: G lanes per vertex share its star.
template <int D, int G>
__global__ void __launch_bounds__(WG) k_gradient(MeshView mv, const double* __restrict__ x,
                                                 const double* __restrict__ xt, Material mat,
                                                 double* __restrict__ g,
                                                 double* __restrict__ partials) {
  __shared__ double red[WG];
  const int lane = threadIdx.x % G;
  const int j = blockIdx.x * (WG / G) + threadIdx.x / G;
  const int n = mv.n;
  double acc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) acc[c] = 0.0;
  if (j < mv.nf) {
    for (int t = mv.star_ptr[j] + lane; t < mv.star_ptr[j + 1]; t += G) {
      const int pk = mv.star[t];
      const int e = pk >> 2, a = pk & 3;
      double F[D][D], beta[D + 1][D], vol, P[D][D];
      load_element<double, D>(mv, e, x, F, beta, vol);
      snh_pk1<double, D>(F, mat.mu, mat.lam, P);
#pragma unroll
      for (int r = 0; r < D; ++r) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) s += P[r][q] * beta[a][q];
        acc[r] += vol * s;
      }
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] += __shfl_xor(acc[c], off, G);
  double gsq = 0.0;
  if (j < mv.nf && lane == 0) {
    const double mj = mv.mass[j];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double gj = mat.w_in * mj * (x[c * n + j] - xt[c * n + j]) +
                        mat.s_el * (acc[c] - mj * mat.grav[c]);
      g[c * n + j] = gj;
      gsq += gj * gj;
    }
  }
  const double tot = block_sum<WG>(gsq, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <typename T, int D>
__device__ __forceinline__ bool chol(const T M[D][D], T L[D][D]) {
  T tr = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) tr += M[i][i];
  const T tol = T(1e-12) * tr;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    T s = M[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    ok = ok && (s > tol);
    const T ljj = csqrt(s > T(0) ? s : T(1));
    L[j][j] = ljj;
#pragma unroll
    for (int i = j + 1; i < D; ++i) {
      T t = M[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / ljj;
    }
#pragma unroll
    for (int i = 0; i < j; ++i) L[i][j] = T(0);
  }
  return ok;
}

// X = M^{-1} B for the Cholesky factor L of M (B, X: D x D, column-wise).
template <typename T, int D>
__device__ __forceinline__ void chol_solve(const T L[D][D], const T B[D][D], T X[D][D]) {
#pragma unroll
  for (int col = 0; col < D; ++col) {
    T y[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T s = B[i][col];
#pragma unroll
      for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
      y[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = D - 1; i >= 0; --i) {
      T s = y[i];
#pragma unroll
      for (int k = i + 1; k < D; ++k) s -= L[k][i] * X[k][col];
      X[i][col] = s / L[i][i];
    }
  }
}

__device__ __forceinline__ int find_slot(const MeshView& mv, int64_t sp0, int64_t sp1, int i, int k) {
  if (mv.dense_supp) {
    if (k == i || k >= mv.nf) return -1;
    return (int)(sp0 + (k < i ? k : k - 1));
  }
  int64_t lo = sp0, hi = sp1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (mv.sidx[mid] < k) lo = mid + 1; else hi = mid;
  }
  return (lo < sp1 && mv.sidx[lo] == k) ? (int)lo : -1;
}

// Per-vertex condensation: A_i = H_iC U_i, Ht_i = U_i^T H_CC U_i, then
// K_i = (H_ii - A Ht^{-1} A^T)^{-1} and L_i = A Ht^{-1} (CC), with the
// coordinate-descent and JGS2 forms as special cases.  G lanes per vertex.
// Contribution of support row j to A_i (when row j holds block (j, i)) and to
// Ht_i (blocks (j, k) with k in the support); Uk(k) returns U_i[k] or null.
template <typename T, int D, typename LookupU>
__device__ __forceinline__ void accum_row(const MeshView& mv, int i, int j, const T* Uj,
                                          const T* __restrict__ hb, LookupU&& Uk_of, T* A, T* Ht) {
  constexpr int DD = D * D;
  for (int t = mv.rowptr[j]; t < mv.rowptr[j + 1]; ++t) {
    const int k = mv.colidx[t];
    const T* H = hb + (size_t)t * DD;
    if (k == i) {
      // A += H_ji^T U_j
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = 0; s < D; ++s) {
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < D; ++l) acc += H[l * D + r] * Uj[l * D + s];
          A[r * D + s] += acc;
        }
      continue;
    }
    const T* Uk = Uk_of(k);
    if (!Uk) continue;
    T Hl[DD], M[DD];
#pragma unroll
    for (int r = 0; r < DD; ++r) Hl[r] = H[r];
#pragma unroll
    for (int r = 0; r < D; ++r)   // M = H_jk U_k
#pragma unroll
      for (int s = 0; s < D; ++s) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < D; ++l) acc += Hl[r * D + l] * Uk[l * D + s];
        M[r * D + s] = acc;
      }
#pragma unroll
    for (int r = 0; r < D; ++r)   // Ht += U_j^T M
#pragma unroll
      for (int s = 0; s < D; ++s) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < D; ++l) acc += Uj[l * D + r] * M[l * D + s];
        Ht[r * D + s] += acc;
      }
  }
}

// Small solves of one vertex from the reduced A_i and Ht_i; writes K_i, L_i.
template <typename T, int D>
__device__ void cc_finish(const MeshView& mv, int method, int i, bool empty, const T* A,
                          const T* Ht, const T* __restrict__ hb, T* __restrict__ KL,
                          unsigned long long* __restrict__ fb) {
  constexpr int DD = D * D;
  T Hii[D][D], Kout[D][D], Lout[D][D], Lc[D][D], I[D][D];
  const T* hd = hb + (size_t)mv.rowptr[i] * DD;
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int s = 0; s < D; ++s) {
      Hii[r][s] = hd[r * D + s];
      I[r][s] = (r == s) ? T(1) : T(0);
      Lout[r][s] = T(0);
      Kout[r][s] = T(0);
    }
  const bool ok_ii = chol<T, D>(Hii, Lc);
  if (!ok_ii) atomicAdd(&fb[2], 1ull);
  T Kcd[D][D];
  if (ok_ii) chol_solve<T, D>(Lc, I, Kcd);
  else
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int s = 0; s < D; ++s) Kcd[r][s] = T(0);
  bool use_cd = true;
  if (method == 1) {  // Coordinate Condensation
    T Htm[D][D], Lt[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int s = 0; s < D; ++s) Htm[r][s] = Ht[r * D + s];
    const bool ok_t = !empty && chol<T, D>(Htm, Lt);
    if (!ok_t) {
      atomicAdd(&fb[0], 1ull);
    } else {
      T At[D][D], Z[D][D], M[D][D], Lm[D][D];
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = 0; s < D; ++s) At[r][s] = A[s * D + r];
      chol_solve<T, D>(Lt, At, Z);  // Z = Ht^{-1} A^T
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = 0; s < D; ++s) {
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < D; ++l) acc += A[r * D + l] * Z[l][s];
          M[r][s] = Hii[r][s] - acc;  // H_ii - S
        }
      if (chol<T, D>(M, Lm)) {
        chol_solve<T, D>(Lm, I, Kout);
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
          for (int s = 0; s < D; ++s) Lout[r][s] = Z[s][r];  // L = A Ht^{-1} = Z^T
        use_cd = false;
      } else {
        atomicAdd(&fb[1], 1ull);
      }
    }
  } else if (method == 2) {  // JGS2 as printed: (H_ii + Ht)^{-1} (g_i + U^T g_C)
    T M[D][D], Lm[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int s = 0; s < D; ++s) M[r][s] = Hii[r][s] + Ht[r * D + s];
    if (!empty && chol<T, D>(M, Lm)) {
      chol_solve<T, D>(Lm, I, Kout);
#pragma unroll
      for (int r = 0; r < D; ++r) Lout[r][r] = T(-1);
      use_cd = false;
    } else {
      atomicAdd(&fb[0], 1ull);
    }
  }
  if (use_cd) {
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int s = 0; s < D; ++s) {
        Kout[r][s] = Kcd[r][s];
        Lout[r][s] = T(0);
      }
  }
  T* o = KL + (size_t)i * 2 * DD;
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int s = 0; s < D; ++s) {
      o[r * D + s] = Kout[r][s];
      o[DD + r * D + s] = Lout[r][s];
    }
}

// Generic condensation kernel: G lanes per vertex, basis and support from
// global memory (binary search for the support slot of a neighbour).
template <typename T, int D, int G>
__global__ void __launch_bounds__(WG) k_cc_prep(MeshView mv, int method, int v0, int v1,
                                                const T* __restrict__ hb, T* __restrict__ KL,
                                                unsigned long long* __restrict__ fb) {
  constexpr int DD = D * D;
  const T* Ub = basis_of<T>(mv);
  const int lane = threadIdx.x % G;
  const int i = v0 + blockIdx.x * (WG / G) + threadIdx.x / G;
  const bool active = i < v1;
  T A[DD], Ht[DD];
#pragma unroll
  for (int r = 0; r < DD; ++r) A[r] = Ht[r] = T(0);
  int64_t sp0 = 0, sp1 = 0;
  if (active && method != 0) {
    sp0 = mv.sptr[i];
    sp1 = mv.sptr[i + 1];
    for (int64_t q = sp0 + lane; q < sp1; q += G) {
      const int j = mv.sidx[q];
      T Uj[DD];
#pragma unroll
      for (int r = 0; r < DD; ++r) Uj[r] = Ub[q * DD + r];
      accum_row<T, D>(mv, i, j, Uj, hb, [&](int k) -> const T* {
        const int qk = find_slot(mv, sp0, sp1, i, k);
        return qk < 0 ? nullptr : Ub + (size_t)qk * DD;
      }, A, Ht);
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
    for (int r = 0; r < DD; ++r) {
      A[r] += __shfl_xor(A[r], off, G);
      Ht[r] += __shfl_xor(Ht[r], off, G);
    }
  if (!active || lane != 0) return;
  cc_finish<T, D>(mv, method, i, sp1 == sp0, A, Ht, hb, KL, fb);
}

// Exact-basis condensation: one workgroup per vertex; the vertex's dense
// basis row U_i (every other free vertex) is staged in LDS, so the H_jk U_k
// products read U_k from LDS while the block rows stream from global memory.
template <typename T, int D>
__global__ void __launch_bounds__(WG) k_cc_prep_dense(MeshView mv, int method, int v0,
                                                      const T* __restrict__ hb, T* __restrict__ KL,
                                                      unsigned long long* __restrict__ fb) {
  constexpr int DD = D * D;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Us = reinterpret_cast<T*>(smem_raw);
  __shared__ T red[WG / 64][2 * DD];
  const T* Ub = basis_of<T>(mv);
  const int i = v0 + blockIdx.x;
  const int cnt = mv.nf - 1;
  const int64_t sp0 = mv.sptr[i];
  for (int q = threadIdx.x; q < cnt * DD; q += WG) Us[q] = Ub[sp0 * DD + q];
  __syncthreads();
  T A[DD], Ht[DD];
#pragma unroll
  for (int r = 0; r < DD; ++r) A[r] = Ht[r] = T(0);
  if (method != 0) {
    for (int a = threadIdx.x; a < cnt; a += WG) {
      const int j = a < i ? a : a + 1;
      T Uj[DD];
#pragma unroll
      for (int r = 0; r < DD; ++r) Uj[r] = Us[a * DD + r];
      accum_row<T, D>(mv, i, j, Uj, hb, [&](int k) -> const T* {
        return Us + (size_t)(k < i ? k : k - 1) * DD;
      }, A, Ht);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int r = 0; r < DD; ++r) {
      A[r] += __shfl_xor(A[r], off, 64);
      Ht[r] += __shfl_xor(Ht[r], off, 64);
    }
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) {
#pragma unroll
    for (int r = 0; r < DD; ++r) {
      red[w][r] = A[r];
      red[w][DD + r] = Ht[r];
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int r = 0; r < DD; ++r) {
    T a = T(0), h = T(0);
#pragma unroll
    for (int ww = 0; ww < WG / 64; ++ww) {
      a += red[ww][r];
      h += red[ww][DD + r];
    }
    A[r] = a;
    Ht[r] = h;
  }
  cc_finish<T, D>(mv, method, i, cnt == 0, A, Ht, hb, KL, fb);
}


// dx_i = -K_i (g_i - L_i U_i^T g_C); written to d (Jacobi) or added to x
// (coloured sweep).  G lanes per vertex share its support.
template <typename T, int D, int G>
__global__ void __launch_bounds__(WG) k_cc_update(MeshView mv, int method, int v0, int v1,
                                                  const T* __restrict__ KL,
                                                  const double* __restrict__ g,
                                                  double* __restrict__ out, int accumulate) {
  constexpr int DD = D * D;
  const T* Ub = basis_of<T>(mv);
  const int lane = threadIdx.x % G;
  const int i = v0 + blockIdx.x * (WG / G) + threadIdx.x / G;
  const bool active = i < v1;
  const int n = mv.n;
  T b[D];
#pragma unroll
  for (int c = 0; c < D; ++c) b[c] = T(0);
  if (active && method != 0) {
    const int64_t sp0 = mv.sptr[i], sp1 = mv.sptr[i + 1];
    for (int64_t q = sp0 + lane; q < sp1; q += G) {
      const int j = mv.sidx[q];
      T gj[D];
#pragma unroll
      for (int c = 0; c < D; ++c) gj[c] = T(g[c * n + j]);
#pragma unroll
      for (int r = 0; r < D; ++r) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < D; ++l) acc += Ub[q * DD + l * D + r] * gj[l];
        b[r] += acc;
      }
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < D; ++c) b[c] += __shfl_xor(b[c], off, G);
  if (!active || lane != 0) return;
  const T* kl = KL + (size_t)i * 2 * DD;
  T gt[D];
#pragma unroll
  for (int r = 0; r < D; ++r) {
    T lb = T(0);
#pragma unroll
    for (int l = 0; l < D; ++l) lb += kl[DD + r * D + l] * b[l];
    gt[r] = T(g[r * n + i] - double(lb));
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < D; ++l) acc += kl[r * D + l] * gt[l];
    if (accumulate) out[r * n + i] -= double(acc);
    else out[r * n + i] = -double(acc);
  }
}

// Step energy: blocks [0, nbe) sum element energies, the rest the free-vertex
// inertia and gravity terms; one partial per block.
template <int D>
__global__ void __launch_bounds__(WG) k_energy(MeshView mv, const double* __restrict__ x,
                                               const double* __restrict__ xt, Material mat,
                                               int nbe, double* __restrict__ partials) {
  __shared__ double red[WG];
  double v = 0.0;
  const int n = mv.n;
  if ((int)blockIdx.x < nbe) {
    const int e = blockIdx.x * WG + threadIdx.x;
    if (e < mv.m) {
      double F[D][D], beta[D + 1][D], vol;
      load_element<double, D>(mv, e, x, F, beta, vol);
      v = mat.s_el * vol * snh_psi<double, D>(F, mat.mu, mat.lam);
    }
  } else {
    const int j = (blockIdx.x - nbe) * WG + threadIdx.x;
    if (j < mv.nf) {
      const double mj = mv.mass[j];
      double in = 0.0, gr = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double dx = x[c * n + j] - xt[c * n + j];
        in += dx * dx;
        gr += mat.grav[c] * x[c * n + j];
      }
      v = mat.w_in * 0.5 * mj * in - mat.s_el * mj * gr;
    }
  }
  const double tot = block_sum<WG>(v, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(WG) k_reduce(const double* __restrict__ partials, int n,
                                               double* __restrict__ out) {
  __shared__ double red[WG];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += WG) v += partials[i];
  const double tot = block_sum<WG>(v, red);
  if (threadIdx.x == 0) out[0] = tot;
}

__global__ void k_axpy(int count, const double* __restrict__ x, const double* __restrict__ d,
                       double alpha, double* __restrict__ out) {
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t < count) out[t] = x[t] + alpha * d[t];
}

template <int D>
__global__ void k_predict(MeshView mv, const int* __restrict__ vperm,
                          const double* __restrict__ xu, const double* __restrict__ vu,
                          const double* __restrict__ xbc, double h, int quasi,
                          double* __restrict__ x, double* __restrict__ xt,
                          double* __restrict__ x0, int* __restrict__ bad) {
  const int v = blockIdx.x * WG + threadIdx.x;
  if (v >= mv.n) return;
  const int u = vperm[v], n = mv.n;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double xp = xu[u * D + c], vp = vu[u * D + c];
    ok = ok && isfinite(xp) && isfinite(vp);
    x0[c * n + v] = xp;
    double xh;
    if (v < mv.nf) {
      xh = quasi ? xp : xp + h * vp;
    } else {
      xh = xbc ? xbc[u * D + c] : xp;
      ok = ok && isfinite(xh);
    }
    xt[c * n + v] = xh;
    x[c * n + v] = xh;
  }
  if (!ok) atomicOr(bad, 1);
}

template <int D>
__global__ void k_finalize(MeshView mv, const int* __restrict__ vperm, const double* __restrict__ x,
                           const double* __restrict__ x0, double h, int quasi,
                           double* __restrict__ xu, double* __restrict__ vu) {
  const int v = blockIdx.x * WG + threadIdx.x;
  if (v >= mv.n) return;
  const int u = vperm[v], n = mv.n;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double xn = x[c * n + v];
    xu[u * D + c] = xn;
    vu[u * D + c] = quasi ? 0.0 : (xn - x0[c * n + v]) / h;
  }
}

template <int D>
__global__ void k_gather_user(MeshView mv, const int* __restrict__ vinv, const double* __restrict__ src,
                              double* __restrict__ dst) {
  const int u = blockIdx.x * WG + threadIdx.x;
  if (u >= mv.n) return;
  const int v = vinv[u];
#pragma unroll
  for (int c = 0; c < D; ++c) dst[c * mv.n + v] = src[u * D + c];
}

template <int D>
__global__ void k_scatter_user(MeshView mv, const int* __restrict__ vperm, const double* __restrict__ src,
                               double* __restrict__ dst, int free_only) {
  const int v = blockIdx.x * WG + threadIdx.x;
  if (v >= mv.n) return;
  const int u = vperm[v];
  const bool keep = !free_only || v < mv.nf;
#pragma unroll
  for (int c = 0; c < D; ++c) dst[u * D + c] = keep ? src[c * mv.n + v] : 0.0;
}

// Parity probe: element gradients (float64 or T) and the full (un-packed)
// Hessian blocks in caller element order.
template <typename T, int D>
__global__ void k_probe_elem(MeshView mv, const double* __restrict__ x, const int* __restrict__ eperm,
                             const T* __restrict__ est, T mu, T lam, double* __restrict__ ge,
                             double* __restrict__ He) {
  constexpr int K = D + 1, DD = D * D;
  const int e = blockIdx.x * WG + threadIdx.x;
  if (e >= mv.m) return;
  const int eu = eperm[e];
  T F[D][D], beta[K][D], vol, P[D][D];
  load_element<T, D>(mv, e, x, F, beta, vol);
  snh_pk1<T, D>(F, mu, lam, P);
  for (int a = 0; a < K; ++a)
    for (int r = 0; r < D; ++r) {
      T s = T(0);
      for (int q = 0; q < D; ++q) s += P[r][q] * beta[a][q];
      ge[((size_t)eu * K + a) * D + r] = double(vol * s);
    }
  const int m = mv.m;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      const int p = a <= b ? pidx<K>(a, b) : pidx<K>(b, a);
      const T* blk = est + ((size_t)p * m + e) * DD;
      for (int r = 0; r < D; ++r)
        for (int s = 0; s < D; ++s)
          He[(((size_t)eu * K + a) * K + b) * DD + r * D + s] =
              double(a <= b ? blk[r * D + s] : blk[s * D + r]);
    }
}

// ---------------------------------------------------------------------------
static inline int nblocks(long long n, int per) { return (int)((n + per - 1) / per); }

#define CC_DISPATCH_D(D_, ...)                     \
  do {                                             \
    if ((D_) == 2) { constexpr int D = 2; __VA_ARGS__; } \
    else { constexpr int D = 3; __VA_ARGS__; }     \
  } while (0)

void launch_predict(const MeshView& mv, const int* vperm, const double* x_user, const double* v_user,
                    const double* x_bc, double h, int quasi, double* x, double* xt, double* x0,
                    int* bad, hipStream_t s) {
  CC_DISPATCH_D(mv.D, k_predict<D><<<nblocks(mv.n, WG), WG, 0, s>>>(mv, vperm, x_user, v_user, x_bc,
                                                                   h, quasi, x, xt, x0, bad));
}

void launch_finalize(const MeshView& mv, const int* vperm, const double* x, const double* x0,
                     double h, int quasi, double* x_user, double* v_user, hipStream_t s) {
  CC_DISPATCH_D(mv.D, k_finalize<D><<<nblocks(mv.n, WG), WG, 0, s>>>(mv, vperm, x, x0, h, quasi,
                                                                    x_user, v_user));
}

void launch_elem_hess(const MeshView& mv, int prec, const double* x, const Material& mat,
                      double scale, void* estore, hipStream_t s) {
  if (mv.m == 0) return;
  const int nb = nblocks(mv.m, WG);
  if (prec == 0)
    CC_DISPATCH_D(mv.D, k_elem_hess<double, D><<<nb, WG, 0, s>>>(mv, x, mat.mu, mat.lam, scale,
                                                                (double*)estore));
  else
    CC_DISPATCH_D(mv.D, k_elem_hess<float, D><<<nb, WG, 0, s>>>(mv, x, (float)mat.mu,
                                                               (float)mat.lam, (float)scale,
                                                               (float*)estore));
}

void launch_assemble(const MeshView& mv, int prec, const void* estore, const Material& mat,
                     void* hb, hipStream_t s) {
  if (mv.nnzb == 0) return;
  const int nb = nblocks(mv.nnzb, WG);
  if (prec == 0)
    CC_DISPATCH_D(mv.D, k_assemble<double, D><<<nb, WG, 0, s>>>(mv, (const double*)estore,
                                                               mat.w_in, (double*)hb));
  else
    CC_DISPATCH_D(mv.D, k_assemble<float, D><<<nb, WG, 0, s>>>(mv, (const float*)estore,
                                                              (float)mat.w_in, (float*)hb));
}

constexpr int GRAD_G = 8;

int reduce_partials_capacity(const MeshView& mv) {
  const int a = nblocks(mv.nf, WG / GRAD_G);
  const int b = nblocks(mv.m, WG) + nblocks(mv.nf, WG);
  return (a > b ? a : b) + 1;
}

void launch_gradient(const MeshView& mv, const double* x, const double* xt, const Material& mat,
                     double* g, double* partials, int* nparts, hipStream_t s) {
  const int nb = nblocks(mv.nf, WG / GRAD_G);
  *nparts = nb;
  if (nb == 0) return;
  CC_DISPATCH_D(mv.D, k_gradient<D, GRAD_G><<<nb, WG, 0, s>>>(mv, x, xt, mat, g, partials));
}

template <typename T, int D>
static void prep_g(const MeshView& mv, int method, int v0, int v1, const void* hb, void* KL,
                   unsigned long long* fb, int G, hipStream_t s) {
  const int cnt = v1 - v0;
  if (G == 64)
    k_cc_prep<T, D, 64><<<nblocks(cnt, WG / 64), WG, 0, s>>>(mv, method, v0, v1, (const T*)hb,
                                                             (T*)KL, fb);
  else
    k_cc_prep<T, D, 16><<<nblocks(cnt, WG / 16), WG, 0, s>>>(mv, method, v0, v1, (const T*)hb,
                                                             (T*)KL, fb);
}

static int support_lanes(const MeshView& mv) {
  if (mv.dense_supp) return 64;
  const double avg = mv.nf > 0 ? double(mv.nnzb) / mv.nf : 0.0;  // proxy: row length
  (void)avg;
  return 16;
}

constexpr size_t DENSE_LDS_LIMIT = 64 * 1024;

template <typename T, int D>
static bool prep_dense(const MeshView& mv, int method, int v0, int v1, const void* hb, void* KL,
                       unsigned long long* fb, hipStream_t s) {
  const size_t lds = (size_t)(mv.nf - 1) * D * D * sizeof(T);
  if (!mv.dense_supp || mv.nf < 2 || lds > DENSE_LDS_LIMIT) return false;
  k_cc_prep_dense<T, D><<<v1 - v0, WG, lds, s>>>(mv, method, v0, (const T*)hb, (T*)KL, fb);
  return true;
}

void launch_cc_prep(const MeshView& mv, int prec, int method, int v0, int v1, const void* hb,
                    void* KL, unsigned long long* fb, hipStream_t s) {
  if (v1 <= v0) return;
  bool done = false;
  if (prec == 0) CC_DISPATCH_D(mv.D, done = prep_dense<double, D>(mv, method, v0, v1, hb, KL, fb, s));
  else CC_DISPATCH_D(mv.D, done = prep_dense<float, D>(mv, method, v0, v1, hb, KL, fb, s));
  if (done) return;
  const int G = support_lanes(mv);
  if (prec == 0) CC_DISPATCH_D(mv.D, prep_g<double, D>(mv, method, v0, v1, hb, KL, fb, G, s));
  else CC_DISPATCH_D(mv.D, prep_g<float, D>(mv, method, v0, v1, hb, KL, fb, G, s));
}

template <typename T, int D>
static void update_g(const MeshView& mv, int method, int v0, int v1, const void* KL, const double* g,
                     double* out, int acc, int G, hipStream_t s) {
  const int cnt = v1 - v0;
  if (G == 64)
    k_cc_update<T, D, 64><<<nblocks(cnt, WG / 64), WG, 0, s>>>(mv, method, v0, v1, (const T*)KL, g,
                                                               out, acc);
  else
    k_cc_update<T, D, 16><<<nblocks(cnt, WG / 16), WG, 0, s>>>(mv, method, v0, v1, (const T*)KL, g,
                                                               out, acc);
}

void launch_cc_update(const MeshView& mv, int prec, int method, int v0, int v1, const void* KL,
                      const double* g, double* x_or_d, int accumulate, hipStream_t s) {
  if (v1 <= v0) return;
  const int G = support_lanes(mv);
  if (prec == 0)
    CC_DISPATCH_D(mv.D, update_g<double, D>(mv, method, v0, v1, KL, g, x_or_d, accumulate, G, s));
  else
    CC_DISPATCH_D(mv.D, update_g<float, D>(mv, method, v0, v1, KL, g, x_or_d, accumulate, G, s));
}

void launch_energy(const MeshView& mv, const double* x, const double* xt, const Material& mat,
                   double* partials, int* nparts, hipStream_t s) {
  const int nbe = nblocks(mv.m, WG), nbv = nblocks(mv.nf, WG);
  *nparts = nbe + nbv;
  if (nbe + nbv == 0) return;
  CC_DISPATCH_D(mv.D, k_energy<D><<<nbe + nbv, WG, 0, s>>>(mv, x, xt, mat, nbe, partials));
}

void launch_reduce(const double* partials, int n, double* out, hipStream_t s) {
  k_reduce<<<1, WG, 0, s>>>(partials, n, out);
}

void launch_axpy(int count, const double* x, const double* d, double alpha, double* out,
                 hipStream_t s) {
  if (count <= 0) return;
  k_axpy<<<nblocks(count, WG), WG, 0, s>>>(count, x, d, alpha, out);
}

void launch_probe_element(const MeshView& mv, int prec, const double* x_user, const int* vperm_inv,
                          const int* eperm, double* xi_tmp, const Material& mat, double* ge,
                          double* He, hipStream_t s) {
  (void)x_user;
  (void)vperm_inv;
  // xi_tmp holds internal-order positions; the caller gathered them already.
  // estore scratch follows the positions in the same allocation.
  const int nb = nblocks(mv.m, WG);
  double* est = xi_tmp + (size_t)mv.D * mv.n;
  launch_elem_hess(mv, prec, xi_tmp, mat, 1.0, est, s);
  if (prec == 0)
    CC_DISPATCH_D(mv.D, k_probe_elem<double, D><<<nb, WG, 0, s>>>(mv, xi_tmp, eperm, (const double*)est,
                                                                 mat.mu, mat.lam, ge, He));
  else
    CC_DISPATCH_D(mv.D, k_probe_elem<float, D><<<nb, WG, 0, s>>>(mv, xi_tmp, eperm, (const float*)est,
                                                                (float)mat.mu, (float)mat.lam, ge, He));
}

void launch_gather_user(const MeshView& mv, const int* vperm_inv, const double* src_user,
                        double* dst_int, hipStream_t s) {
  CC_DISPATCH_D(mv.D, k_gather_user<D><<<nblocks(mv.n, WG), WG, 0, s>>>(mv, vperm_inv, src_user, dst_int));
}

void launch_scatter_user(const MeshView& mv, const int* vperm, const double* src_int,
                         double* dst_user, int free_only, hipStream_t s) {
  CC_DISPATCH_D(mv.D, k_scatter_user<D><<<nblocks(mv.n, WG), WG, 0, s>>>(mv, vperm, src_int, dst_user,
                                                                        free_only));
}

}  // namespace cc
