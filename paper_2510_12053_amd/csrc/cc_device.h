// Device helpers shared by the single-mesh and batched kernels (gfx950).
#pragma once
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
// Global-memory view of a pointer read from a struct in memory (those are
// generic, so their loads would be FLAT, which also count against the LDS
// wait counter and stall LDS reads behind outstanding global loads).
template <typename T>
using gmem_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ const gmem_t<T>* gptr(const T* p) { return (const gmem_t<T>*)p; }
template <typename T>
__device__ __forceinline__ gmem_t<T>* gptr_w(T* p) { return (gmem_t<T>*)p; }

template <typename T> __device__ __forceinline__ const T* basis_of(const MeshView& mv);
template <> __device__ __forceinline__ const float* basis_of<float>(const MeshView& mv) { return mv.U_f; }
template <> __device__ __forceinline__ const double* basis_of<double>(const MeshView& mv) { return mv.U_d; }

// beta_a, F = sum_{a>=1} (x_a - x_0) beta_a^T and the rest volume of element
// e from its edge matrix Ds = [x_a - x_0].
template <typename T, int D>
__device__ __forceinline__ void element_from_edges(const MeshView& mv, int e, const T Ds[D][D],
                                                   T F[D][D], T beta[D + 1][D], T& vol);

// F = sum_{a>=1} (x_a - x_0) beta_a^T, differences formed in float64 then cast.
template <typename T, int D>
__device__ __forceinline__ void load_element(const MeshView& mv, int e, const double* __restrict__ x,
                                             T F[D][D], T beta[D + 1][D], T& vol) {
  const int m = mv.m, n = mv.n;
  const int v0 = mv.ev[e];
  T Ds[D][D];
#pragma unroll
  for (int a = 1; a <= D; ++a) {
    const int va = mv.ev[a * m + e];
#pragma unroll
    for (int c = 0; c < D; ++c) Ds[c][a - 1] = T(x[c * n + va] - x[c * n + v0]);
  }
  element_from_edges<T, D>(mv, e, Ds, F, beta, vol);
}

// The same at the positions x + alpha d, each formed as the trial-point
// update forms it, so the values equal those of a stored x + alpha d.
template <typename T, int D>
__device__ __forceinline__ void load_element_along(const MeshView& mv, int e, const double* __restrict__ x,
                                                   const double* __restrict__ d, double alpha,
                                                   T F[D][D], T beta[D + 1][D], T& vol) {
  const int m = mv.m, n = mv.n;
  const int v0 = mv.ev[e];
  T Ds[D][D];
#pragma unroll
  for (int a = 1; a <= D; ++a) {
    const int va = mv.ev[a * m + e];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double pa = x[c * n + va] + alpha * d[c * n + va];
      const double p0 = x[c * n + v0] + alpha * d[c * n + v0];
      Ds[c][a - 1] = T(pa - p0);
    }
  }
  element_from_edges<T, D>(mv, e, Ds, F, beta, vol);
}

template <typename T, int D>
__device__ __forceinline__ void element_from_edges(const MeshView& mv, int e, const T Ds[D][D],
                                                   T F[D][D], T beta[D + 1][D], T& vol) {
  const int m = mv.m;
  const T* dinv = dinv_of<T>(mv);
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
        // stop rotating a pair once it is below the rounding of its diagonal
        if (cabs(apq) <= eps * (cabs(app) + cabs(aqq)) || apq == T(0)) {
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
// The singular value of smallest magnitude carries the sign of det F.
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
  // With det F < 0 the negative value belongs to the smallest |sig| (then
  // U V^T is the rotation nearest to F): move it there by negating two
  // columns of U, which keeps det U = +1.
  if (sig[D - 1] < T(0)) {
    int km = D - 1;
#pragma unroll
    for (int k = 0; k < D - 1; ++k)
      if (cabs(sig[k]) < cabs(sig[km])) km = k;
    if (km != D - 1) {
      sig[D - 1] = -sig[D - 1];
      sig[km] = -sig[km];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        U[i][D - 1] = -U[i][D - 1];
        U[i][km] = -U[i][km];
      }
    }
  }
}

// Projected material Hessian as its positive eigenpairs.  In the frame of
// F = U diag(sig) V^T (rotation-variant: U, V rotations, the smallest sig may
// be negative) both materials split the same way: a D x D block coupling the
// diagonal entries, A_kk = a + lam c_k^2, A_kl = lam c_k c_l + s sig_m (c the
// diagonal cofactors, sig_m the remaining singular value, 1 in 2D), and for
// every pair k < l a flip (vector (1, 1)/sqrt(2) on (F_kl, F_lk)) with
// eigenvalue a - s sig_m and a twist ((1, -1)/sqrt(2)) with a + s sig_m - t_kl.
//   stable neo-Hookean: a = mu,   s = lam (J-1) - mu, t_kl = 0;
//   Fixed Corotational: a = 2 mu, s = lam (J-1),      t_kl = 4 mu / (sig_k + sig_l)
// (the as-rigid-as-possible part has eigenvalue 2 mu everywhere except on the
// twists, where the polar rotation turns with the element; t_kl is taken as 0
// where sig_k + sig_l = 0 and the rotation has no derivative).  Eigen-matrices
// map back as U E V^T.
//
// callback(w, Q, P, same) adds w vec(Q) vec(P)^T to the projected Hessian:
// once per eigenpair with weight w > 0 (P is Q, same = true), or, when the
// scaling block A is positive definite (its projection is A itself, and no
// eigen-solve is needed), once per k with Q = u_k v_k^T and
// P = sum_l A_kl u_l v_l^T (w = 1, same = false).
template <typename T, int D, typename CB>
__device__ __forceinline__ void projected_eigs(const T F[D][D], T mu, T lam, int model, CB&& callback) {
  T U[D][D], V[D][D], sig[D];
  svd_rv<T, D>(F, U, V, sig);
  T J = T(1);
#pragma unroll
  for (int k = 0; k < D; ++k) J *= sig[k];
  const bool fcr = model == MAT_FCR;
  const T a0 = fcr ? T(2) * mu : mu;
  const T s = fcr ? lam * (J - T(1)) : lam * (J - T(1)) - mu;
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
      A[k][l] = (k == l) ? a0 + lam * c[k] * c[k] : lam * c[k] * c[l] + s * third[k][l];
  // positive definite by Sylvester's criterion (leading principal minors)
  bool pd = A[0][0] > T(0) && A[0][0] * A[1][1] - A[0][1] * A[1][0] > T(0);
  if constexpr (D == 3) pd = pd && det<T, 3>(A) > T(0);
  T Q[D][D];
  if (pd) {
    T P[D][D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
          Q[i][j] = U[i][k] * V[j][k];
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < D; ++l) acc += A[k][l] * U[i][l] * V[j][l];
          P[i][j] = acc;
        }
      callback(T(1), Q, P, false);
    }
  } else {
    T W[D][D];
    jacobi_eig<T, D>(A, W);
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
        callback(w, Q, Q, true);
      }
    }
  }
  const T h = T(0.70710678118654752440);
#pragma unroll
  for (int k = 0; k < D - 1; ++k)
#pragma unroll
    for (int l = k + 1; l < D; ++l) {
      const T sm = third[k][l];
      const T den = sig[k] + sig[l];
      const T tw = (fcr && den != T(0)) ? T(4) * mu / den : T(0);
#pragma unroll
      for (int sgn = 0; sgn < 2; ++sgn) {
        // sgn 0: flip (1, 1), eigenvalue a - s sig_m; sgn 1: twist (1, -1), a + s sig_m - t_kl
        const T w = sgn == 0 ? a0 - s * sm : a0 + s * sm - tw;
        if (!(w > T(0))) continue;
        const T b = sgn == 0 ? h : -h;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) Q[i][j] = h * U[i][k] * V[j][l] + b * U[i][l] * V[j][k];
        callback(w, Q, Q, true);
      }
    }
}

// Fixed Corotational energy density mu |F - R|^2 + lam/2 (J-1)^2 with R = U V^T
// the rotation nearest to F, and its first Piola-Kirchhoff stress
// 2 mu (F - R) + lam (J-1) cof(F).
template <typename T, int D>
__device__ __forceinline__ T fcr_psi(const T F[D][D], T mu, T lam) {
  T U[D][D], V[D][D], sig[D];
  svd_rv<T, D>(F, U, V, sig);
  T q = T(0);
#pragma unroll
  for (int k = 0; k < D; ++k) q += (sig[k] - T(1)) * (sig[k] - T(1));
  const T J = det<T, D>(F);
  return mu * q + T(0.5) * lam * (J - T(1)) * (J - T(1));
}

template <typename T, int D>
__device__ __forceinline__ void fcr_pk1(const T F[D][D], T mu, T lam, T P[D][D]) {
  T U[D][D], V[D][D], sig[D], C[D][D];
  svd_rv<T, D>(F, U, V, sig);
  cofactor<T, D>(F, C);
  const T k = lam * (det<T, D>(F) - T(1));
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      T R = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) R += U[r][j] * V[q][j];
      P[r][q] = T(2) * mu * (F[r][q] - R) + k * C[r][q];
    }
}

template <typename T, int D>
__device__ __forceinline__ T material_psi(const T F[D][D], T mu, T lam, int model) {
  return model == MAT_FCR ? fcr_psi<T, D>(F, mu, lam) : snh_psi<T, D>(F, mu, lam);
}

template <typename T, int D>
__device__ __forceinline__ void material_pk1(const T F[D][D], T mu, T lam, int model, T P[D][D]) {
  if (model == MAT_FCR)
    fcr_pk1<T, D>(F, mu, lam, P);
  else
    snh_pk1<T, D>(F, mu, lam, P);
}

// ---------------------------------------------------------------------------
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

// Basis row of vertex i as blocks [sp0, sp1) of U: CSR rows for sparse bases,
// nf blocks in band order (own block zero) for dense ones.
__device__ __forceinline__ void supp_range(const MeshView& mv, int i, int64_t& sp0, int64_t& sp1) {
  if (mv.dense_supp) {
    sp0 = (int64_t)i * mv.nf;
    sp1 = sp0 + mv.nf;
  } else {
    sp0 = mv.sptr[i];
    sp1 = mv.sptr[i + 1];
  }
}

// Vertex (internal id) of block q of the row starting at sp0.
__device__ __forceinline__ int supp_vertex(const MeshView& mv, int64_t q, int64_t sp0) {
  return mv.dense_supp ? mv.bvert[q - sp0] : mv.sidx[q];
}

// Block of vertex k in row i (blocks [sp0, sp1)), or -1 when k is not in supp(i).
__device__ __forceinline__ int64_t find_slot(const MeshView& mv, int64_t sp0, int64_t sp1, int i, int k) {
  if (mv.dense_supp) {
    if (k == i || k >= mv.nf) return -1;
    return sp0 + mv.bpos[k];
  }
  int64_t lo = sp0, hi = sp1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (mv.sidx[mid] < k) lo = mid + 1; else hi = mid;
  }
  return (lo < sp1 && mv.sidx[lo] == k) ? lo : -1;
}

// Per-vertex condensation: A_i = H_iC U_i, Ht_i = U_i^T H_CC U_i, then
// K_i = (H_ii - A Ht^{-1} A^T)^{-1} and L_i = A Ht^{-1} (CC), with the
// coordinate-descent and JGS2 forms as special cases.  G lanes per vertex.
// Contribution of support row j to A_i (when row j holds block (j, i)) and to
// U <- R_j U with R_j the vertex's rotation (corotated basis block).
template <typename T, int D>
__device__ __forceinline__ void rotate_block(const double* __restrict__ rot, int j, T* U) {
  T Rj[D * D], out[D * D];
#pragma unroll
  for (int r = 0; r < D * D; ++r) Rj[r] = T(rot[(size_t)j * D * D + r]);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) acc += Rj[r * D + l] * U[l * D + c];
      out[r * D + c] = acc;
    }
#pragma unroll
  for (int r = 0; r < D * D; ++r) U[r] = out[r];
}

// Ht_i (blocks (j, k) with k in the support); Uk_of(k, Uk) fills U_i[k] and
// returns true, or returns false when k is outside the support.
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
    T Uk[DD];
    if (!Uk_of(k, Uk)) continue;
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


__device__ __forceinline__ int block_mesh(const int* __restrict__ boff, int nmesh, int b) {
  int lo = 0, hi = nmesh;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace cc
