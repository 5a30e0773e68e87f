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

#include <algorithm>
#include <vector>

#include "cc_device.h"

namespace cc {

// Element Hessian: H_e[a,b] = scale * V_e * sum_r w_r (Q_r beta_a)(Q_r beta_b)^T
// H selects the output blocks: 0 all of them, 1 the first half of the packed
// blocks, 2 the second half (the element's eigensystem is formed either way).
template <typename T, int D, int H>
__device__ __forceinline__ void elem_hess_body(const MeshView& mv, int e, const double* __restrict__ x,
                                               T mu, T lam, int model, T scale, T* __restrict__ out) {
  constexpr int K = D + 1, DD = D * D, NB = K * (K + 1) / 2;
  auto keep = [](int p) { return H == 0 || (H == 1 ? p < NB / 2 : p >= NB / 2); };
  if (e >= mv.m) return;
  T F[D][D], beta[K][D], vol;
  load_element<T, D>(mv, e, x, F, beta, vol);
  T acc[NB][DD];
#pragma unroll
  for (int p = 0; p < NB; ++p)
#pragma unroll
    for (int r = 0; r < DD; ++r) acc[p][r] = T(0);
  // y[a] = Q beta_a and z[a] = P beta_a (the vertex-a rows of the mode's
  // matrices); block (a, b) gains w y[a] z[b]^T
  auto rows = [&](const T (&M)[D][D], T (&y)[K][D]) {
#pragma unroll
    for (int a = 1; a < K; ++a)
#pragma unroll
      for (int r = 0; r < D; ++r) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < D; ++q) s += M[r][q] * beta[a][q];
        y[a][r] = s;
      }
#pragma unroll
    for (int r = 0; r < D; ++r) {
      T s = T(0);
#pragma unroll
      for (int a = 1; a < K; ++a) s += y[a][r];
      y[0][r] = -s;
    }
  };
  projected_eigs<T, D>(F, mu, lam, model, [&](T w, const T (&Q)[D][D], const T (&P)[D][D], bool same) {
    T y[K][D], z[K][D];
    rows(Q, y);
    if (same) {
#pragma unroll
      for (int a = 0; a < K; ++a)
#pragma unroll
        for (int r = 0; r < D; ++r) z[a][r] = y[a][r];
    } else {
      rows(P, z);
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
      T wy[D];
#pragma unroll
      for (int r = 0; r < D; ++r) wy[r] = w * y[a][r];
#pragma unroll
      for (int b = a; b < K; ++b)
        if (keep(pidx<K>(a, b)))
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int s = 0; s < D; ++s) acc[pidx<K>(a, b)][r * D + s] += wy[r] * z[b][s];
    }
  });
  const T f = scale * vol;
  const int m = mv.m;
#pragma unroll
  for (int p = 0; p < NB; ++p)
    if (keep(p))
#pragma unroll
      for (int r = 0; r < DD; ++r) out[((size_t)p * m + e) * DD + r] = f * acc[p][r];
}

// Element and assembly kernels run one thread per element / block slot in
// 64-thread workgroups: a few thousand elements then spread over most CUs
// instead of a few dozen (the per-element work is a long serial chain).
// In float64 the element kernel gives each workgroup of EWG elements two
// waves, each accumulating half of the output blocks: one wave holding all
// ten 3x3 float64 accumulators spills registers.
constexpr int EWG = 64;
template <typename T> constexpr int elem_threads() { return sizeof(T) == 8 ? 2 * EWG : EWG; }

// Element index of slot idx: idx itself, or entry idx of a list of ecount
// elements (past its end: m, which the body skips).
__device__ __forceinline__ int elem_of(const MeshView& mv, int idx, const int* elist, int ecount) {
  if (elist == nullptr) return idx;
  return idx < ecount ? elist[idx] : mv.m;
}

template <typename T, int D>
__device__ __forceinline__ void elem_hess_split(const MeshView& mv, int e0, const double* __restrict__ x,
                                                T mu, T lam, int model, T scale, T* __restrict__ out,
                                                const int* elist = nullptr, int ecount = 0) {
  if constexpr (sizeof(T) == 8) {
    const int e = elem_of(mv, e0 + threadIdx.x % EWG, elist, ecount);
    if (threadIdx.x < EWG) elem_hess_body<T, D, 1>(mv, e, x, mu, lam, model, scale, out);
    else elem_hess_body<T, D, 2>(mv, e, x, mu, lam, model, scale, out);
  } else {
    elem_hess_body<T, D, 0>(mv, elem_of(mv, e0 + threadIdx.x, elist, ecount), x, mu, lam, model, scale, out);
  }
}
constexpr int LS_WIDTH = 8;   // backtracking halvings evaluated per launch

template <typename T, int D, bool FCR>
__global__ void __launch_bounds__(elem_threads<T>()) k_elem_hess(MeshView mv, const double* __restrict__ x,
                                                                 T mu, T lam, int model, T scale,
                                                                 T* __restrict__ out, const int* elist,
                                                                 int ecount) {
  elem_hess_split<T, D>(mv, blockIdx.x * EWG, x, mu, lam, FCR ? model : MAT_SNH, scale, out, elist, ecount);
}

// Block rows: every slot sums its element contributions (fixed order), plus
// the mass on the diagonal.
// The BandRec of block slot t (row j) of a dense-basis mesh, when t is an
// upper slot: w R_j^T H_jk R_k and the band position of k.
template <typename T, int D>
__device__ __forceinline__ void band_rec_write(const MeshView& mv, int t, int j, const T* blk) {
  constexpr int DD = D * D;
  const int qp = mv.hq_slot[t];
  if (qp < 0) return;
  const int k = mv.colidx[t];
  const T w = k == j ? T(0.5) : T(1);
  T b[DD];
#pragma unroll
  for (int r = 0; r < DD; ++r) b[r] = w * blk[r];
  if (mv.rot != nullptr) {
    T Rj[DD], Rk[DD], tmp[DD];
#pragma unroll
    for (int r = 0; r < DD; ++r) {
      Rj[r] = T(mv.rot[(size_t)j * DD + r]);
      Rk[r] = T(mv.rot[(size_t)k * DD + r]);
    }
#pragma unroll
    for (int r = 0; r < D; ++r)               // tmp = B R_k
#pragma unroll
      for (int c = 0; c < D; ++c) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < D; ++l) acc += b[r * D + l] * Rk[l * D + c];
        tmp[r * D + c] = acc;
      }
#pragma unroll
    for (int r = 0; r < D; ++r)               // b = R_j^T tmp
#pragma unroll
      for (int c = 0; c < D; ++c) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < D; ++l) acc += Rj[l * D + r] * tmp[l * D + c];
        b[r * D + c] = acc;
      }
  }
  auto* rec = reinterpret_cast<BandRec<T, D>*>(mv.hq) + qp;
#pragma unroll
  for (int r = 0; r < DD; ++r) rec->h[r] = b[r];
  rec->pos = mv.bpos[k];
}

template <typename T, int D>
__device__ __forceinline__ void assemble_body(const MeshView& mv, int tt, const T* __restrict__ est,
                                              T w_in, T* __restrict__ hb, const int* slist = nullptr,
                                              int scount = 0) {
  constexpr int K = D + 1, DD = D * D;
  if (tt >= (slist ? scount : mv.nnzb)) return;
  // slots row by row in caller order of the rows: neighbouring threads then
  // read the blocks of neighbouring elements (a colour's list keeps that order)
  const int t = slist ? slist[tt] : (mv.aorder ? mv.aorder[tt] : tt);
  T acc[DD];
#pragma unroll
  for (int r = 0; r < DD; ++r) acc[r] = T(0);
  const int m = mv.m;
  // Contributions are summed in list order (so results are reproducible bit
  // for bit), with the blocks of four consecutive entries loaded before any
  // is added: a diagonal slot gathers one block per incident element, and a
  // chain of dependent index and block loads would set its time.
  const int c1 = mv.cptr[t + 1];
  int c = mv.cptr[t];
  for (; c + 4 <= c1; c += 4) {
    T v[4][DD];
    bool tr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pk = mv.centry[c + q];
      const int e = pk >> 4, a = (pk >> 2) & 3, b = pk & 3;
      tr[q] = a > b;
      const T* blk = est + ((size_t)pidx<K>(tr[q] ? b : a, tr[q] ? a : b) * m + e) * DD;
#pragma unroll
      for (int r = 0; r < DD; ++r) v[q][r] = blk[r];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int s = 0; s < D; ++s) acc[r * D + s] += tr[q] ? v[q][s * D + r] : v[q][r * D + s];
  }
  for (; c < c1; ++c) {
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
  if (mv.hq != nullptr) band_rec_write<T, D>(mv, t, j, acc);
}

template <typename T, int D>
__global__ void __launch_bounds__(EWG) k_band_copy(MeshView mv, const T* __restrict__ hb) {
  const int t = blockIdx.x * EWG + threadIdx.x;
  if (t < mv.nnzb) band_rec_write<T, D>(mv, t, mv.blkrow[t], hb + (size_t)t * D * D);
}

template <typename T, int D>
__global__ void __launch_bounds__(EWG) k_assemble(MeshView mv, const T* __restrict__ est, T w_in,
                                                  T* __restrict__ hb, const int* slist, int scount) {
  assemble_body<T, D>(mv, blockIdx.x * EWG + threadIdx.x, est, w_in, hb, slist, scount);
}

// Vertex of gradient slot idx: the free vertices in caller order, so that
// neighbouring lane groups walk overlapping element stars (nf: no vertex).
__device__ __forceinline__ int grad_vertex(const MeshView& mv, int idx) {
  if (idx >= mv.nf) return mv.nf;
  return mv.sorder ? mv.sorder[idx] : idx;
}

// Free-vertex gradient in float64: G lanes per vertex share its star.
// Returns g_j . g_j on the group's first lane, 0 elsewhere.
template <int D, int G, bool FCR>
__device__ __forceinline__ double gradient_body(const MeshView& mv, int j, int lane,
                                                const double* __restrict__ x,
                                                const double* __restrict__ xt, const Material& mat,
                                                double* __restrict__ g) {
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
      material_pk1<double, D>(F, mat.mu, mat.lam, FCR ? mat.model : MAT_SNH, P);
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
  return gsq;
}

template <int D, int G, bool FCR>
__global__ void __launch_bounds__(WG) k_gradient(MeshView mv, const double* __restrict__ x,
                                                 const double* __restrict__ xt, Material mat,
                                                 double* __restrict__ g,
                                                 double* __restrict__ partials) {
  __shared__ double red[WG];
  const double gsq = gradient_body<D, G, FCR>(mv, grad_vertex(mv, blockIdx.x * (WG / G) + threadIdx.x / G),
                                         threadIdx.x % G, x, xt, mat, g);
  const double tot = block_sum<WG>(gsq, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Vertex of thread slot idx in [0, v1 - v0): a whole-mesh sweep visits the
// free vertices in caller order, so neighbouring slots share rows of H (the
// colour-sorted internal order scatters them over the mesh); a colour sweep
// takes its colour's range.
__device__ __forceinline__ int sweep_vertex(const MeshView& mv, int v0, int v1, int idx) {
  return (v0 == 0 && v1 == mv.nf && mv.sorder) ? mv.sorder[idx] : v0 + idx;
}

// Workgroups are dealt to the 8 XCDs in turn; renumber block b of nb so that
// the blocks one XCD runs cover a contiguous range (one L2 per XCD).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Generic condensation kernel: G lanes per vertex, basis and support from
// global memory.  The support position of a neighbour comes from the slot map
// when the mesh has one, else from a binary search in the support row.
// With `stage` non-null (the same for the whole workgroup) each vertex group
// owns cap * D * D values of it: a support row of up to cap blocks is copied
// there with contiguous loads (and rotated once for a corotated basis), so the
// U_i[k] lookups of the slot-map path read LDS instead of scattered global
// blocks.
template <typename T, int D, int G>
__device__ __forceinline__ void prep_body(const MeshView& mv, int method, int i, bool active, int lane,
                                          const T* __restrict__ hb, T* __restrict__ KL,
                                          unsigned long long* __restrict__ fb,
                                          T* __restrict__ stage = nullptr, int cap = 0) {
  constexpr int DD = D * D;
  const T* Ub = basis_of<T>(mv);
  T A[DD], Ht[DD];
#pragma unroll
  for (int r = 0; r < DD; ++r) A[r] = Ht[r] = T(0);
  int64_t sp0 = 0, sp1 = 0;
  if (active && method != 0) supp_range(mv, i, sp0, sp1);
  const T* Us = nullptr;   // staged, rotated support row of vertex i
  if (stage) {
    const bool st = active && method != 0 && mv.smap && sp1 - sp0 <= cap;
    T* my = stage + (size_t)(threadIdx.x / G) * cap * DD;
    if (st)
      for (int e = lane; e < (int)(sp1 - sp0) * DD; e += G) my[e] = Ub[sp0 * DD + e];
    __syncthreads();
    if (mv.rot) {
      if (st)
        for (int q = lane; q < (int)(sp1 - sp0); q += G) {
          T b[DD];
#pragma unroll
          for (int r = 0; r < DD; ++r) b[r] = my[q * DD + r];
          rotate_block<T, D>(mv.rot, mv.sidx[sp0 + q], b);
#pragma unroll
          for (int r = 0; r < DD; ++r) my[q * DD + r] = b[r];
        }
      __syncthreads();
    }
    if (st) Us = my;
  }
  if (active && method != 0 && mv.smap) {
    // Sparse support with a slot map: the blocks (j, k), k >= j, of row j
    // whose column lies in supp(i) come with k's support position, so the
    // loads of H_jk and U_i[k] do not wait on a search.  H is symmetric, so
    // with W = sum_{k > j} H_jk U_i[k] + 1/2 H_jj U_i[j] and
    // Y = sum_j U_i[j]^T W, Ht = Y + Y^T (formed after the lane reduction).
    const int nw = mv.smap_words;
    for (int64_t q = sp0 + lane; q < sp1; q += G) {
      const int a = (int)(q - sp0);
      const uint32_t* sm = mv.smap + (size_t)q * (nw + 1);
      const int t0 = (int)sm[0];
      T Uj[DD], W[DD];
      if (Us) {
#pragma unroll
        for (int r = 0; r < DD; ++r) Uj[r] = Us[(q - sp0) * DD + r];
      } else {
#pragma unroll
        for (int r = 0; r < DD; ++r) Uj[r] = Ub[q * DD + r];
        if (mv.rot) rotate_block<T, D>(mv.rot, mv.sidx[q], Uj);
      }
#pragma unroll
      for (int r = 0; r < DD; ++r) W[r] = T(0);
      for (int w = 0; w < nw; ++w) {
        const uint32_t word = sm[1 + w];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int code = (word >> (8 * b)) & 255;
          if (code == SMAP_SKIP) continue;
          const T* H = hb + (size_t)(t0 + 4 * w + b) * DD;
          T Hl[DD];
#pragma unroll
          for (int r = 0; r < DD; ++r) Hl[r] = H[r];
          if (code == SMAP_SELF) {            // block (j, i): A += H_ji^T U_i[j]
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
              for (int c = 0; c < D; ++c) {
                T acc = T(0);
#pragma unroll
                for (int l = 0; l < D; ++l) acc += Hl[l * D + r] * Uj[l * D + c];
                A[r * D + c] += acc;
              }
            continue;
          }
          T Uk[DD];
          if (Us) {
#pragma unroll
            for (int r = 0; r < DD; ++r) Uk[r] = Us[code * DD + r];
          } else {
            const int64_t qk = sp0 + code;
#pragma unroll
            for (int r = 0; r < DD; ++r) Uk[r] = Ub[qk * DD + r];
            if (mv.rot) rotate_block<T, D>(mv.rot, mv.sidx[qk], Uk);
          }
          if (code == a)                      // diagonal block: half weight (exact)
#pragma unroll
            for (int r = 0; r < DD; ++r) Uk[r] *= T(0.5);
#pragma unroll
          for (int r = 0; r < D; ++r)         // W += H_jk U_i[k]
#pragma unroll
            for (int c = 0; c < D; ++c) {
              T acc = W[r * D + c];
#pragma unroll
              for (int l = 0; l < D; ++l) acc += Hl[r * D + l] * Uk[l * D + c];
              W[r * D + c] = acc;
            }
        }
      }
#pragma unroll
      for (int r = 0; r < D; ++r)             // Y += U_i[j]^T W
#pragma unroll
        for (int c = 0; c < D; ++c) {
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < D; ++l) acc += Uj[l * D + r] * W[l * D + c];
          Ht[r * D + c] += acc;
        }
    }
  } else if (active && method != 0) {
    for (int64_t q = sp0 + lane; q < sp1; q += G) {
      const int j = supp_vertex(mv, q, sp0);
      if (j == i) continue;                   // the zero own block of a dense row
      T Uj[DD];
#pragma unroll
      for (int r = 0; r < DD; ++r) Uj[r] = Ub[q * DD + r];
      if (mv.rot) rotate_block<T, D>(mv.rot, j, Uj);
      accum_row<T, D>(mv, i, j, Uj, hb, [&](int k, T* Uk) -> bool {
        const int64_t qk = find_slot(mv, sp0, sp1, i, k);
        if (qk < 0) return false;
#pragma unroll
        for (int r = 0; r < DD; ++r) Uk[r] = Ub[(size_t)qk * DD + r];
        if (mv.rot) rotate_block<T, D>(mv.rot, k, Uk);
        return true;
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
  if (mv.smap) {                              // Ht = Y + Y^T
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int c = r; c < D; ++c) {
        const T y = Ht[r * D + c] + Ht[c * D + r];
        Ht[r * D + c] = y;
        Ht[c * D + r] = y;
      }
  }
  cc_finish<T, D>(mv, method, i, sp1 == sp0, A, Ht, hb, KL, fb);
}

template <typename T, int D, int G>
__global__ void __launch_bounds__(WG) k_cc_prep(MeshView mv, int method, int v0, int v1,
                                                const T* __restrict__ hb, T* __restrict__ KL,
                                                unsigned long long* __restrict__ fb, int cap) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int idx = xcd_block(blockIdx.x, gridDim.x) * (WG / G) + threadIdx.x / G;
  const bool act = idx < v1 - v0;
  prep_body<T, D, G>(mv, method, act ? sweep_vertex(mv, v0, v1, idx) : v0, act, threadIdx.x % G, hb, KL,
                     fb, cap > 0 ? reinterpret_cast<T*>(smem_raw) : nullptr, cap);
}

// Exact-basis condensation of TV vertices per workgroup (Method, Eqs. block
// and schur: A_i = H_iC U_i, Ht_i = U_i^T H_CC U_i, b_i = U_i^T g_C; with
// corotation every U_i[j] is R_j U_i[j], Eq. rotation).
//
// The basis rows are stored in band order (MeshView::bvert), in which every
// block (j, k) of H with k after j has k within band_w positions of j.  H is
// symmetric, so with X_jk = U_j^T H''_jk U_k, H''_jk = R_j^T H_jk R_k,
//   Ht = sum_{j,k} X_jk = Y + Y^T,  Y = sum_j U_j^T W_j,
//   W_j = sum_{k >= j} w_jk H''_jk U_k  (w = 1/2 on the diagonal block),
// and only the upper blocks are read, from the BandRec list hq (rotated and
// weighted there once per Hessian, not once per basis row).  The workgroup
// walks the band in chunks of CH positions, one thread per row j of the
// chunk; row j needs U at positions [j, j + band_w], so the TV rows live in
// an LDS ring of R >= CH + band_w positions, refilled one chunk ahead: the
// global loads of chunk c + 1's new positions are issued before chunk c's
// products and stored after them.  A ring slot holds the TV blocks of one
// position contiguously, padded to an odd number of words, so a block read
// is one address and constant offsets, and the threads of a wave, which
// take consecutive positions (whose columns are, on structured grids,
// consecutive too), hit distinct banks.  Every H block serves the TV rows of
// the workgroup from registers.
// A_i = sum_k H_ik R_k U_i[k] comes from row i in global memory (one wave
// per vertex; the row was just streamed through L2).
//
// With g given (Jacobi sweeps), b_i = U_i^T (R^T g)_C is also accumulated
// from the staged rows and stored in bout (component-major, stride n); the
// finish kernel then writes the direction itself.
template <typename T, int D>
__device__ __forceinline__ void band_load(const MeshView& mv, const T* __restrict__ Ub, int row, int pos,
                                          T (&blk)[D * D]) {
  constexpr int DD = D * D;
  const auto* src = gptr(Ub) + ((size_t)row * mv.nf + pos) * DD;
#pragma unroll
  for (int r = 0; r < DD; ++r) blk[r] = src[r];
}

// Raw buffer resource over `bytes` bytes at p (offsets past the end read
// as zero).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// A BandRec as raw dwords, loaded 16 bytes at a time from byte offset off.
template <typename T, int D>
struct RecWords {
  static constexpr int N = sizeof(BandRec<T, D>) / 4;
  uint32_t w[N];
  __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
#pragma unroll
    for (int c = 0; c < N / 4; ++c) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16u * c, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) w[4 * c + e] = v[e];
    }
  }
  __device__ __forceinline__ T h(int r) const {
    if constexpr (sizeof(T) == 4) {
      return __builtin_bit_cast(float, w[r]);
    } else {
      return __builtin_bit_cast(double, (uint64_t)w[2 * r] | ((uint64_t)w[2 * r + 1] << 32));
    }
  }
  __device__ __forceinline__ int pos() const { return (int)w[D * D * sizeof(T) / 4]; }
};

// Sum over the 64 lanes of a wave, valid in lane 63: rotations within each
// row of 16 lanes leave the row sum in every lane of the row, then two row
// broadcasts add rows 0-1 into row 3 (DPP, no LDS traffic).
__device__ __forceinline__ float dpp_step(float x, int y) { return x + __builtin_bit_cast(float, y); }
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROWS, 0xf, false);
  return dpp_step(x, y);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xf, false);
  return x + __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}
template <typename T>
__device__ __forceinline__ T wave_sum63(T x) {
  x = dpp_add<0x128, 0xf>(x);   // row_ror:8
  x = dpp_add<0x124, 0xf>(x);   // row_ror:4
  x = dpp_add<0x122, 0xf>(x);   // row_ror:2
  x = dpp_add<0x121, 0xf>(x);   // row_ror:1
  x = dpp_add<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return x;
}

template <int W> struct UnitVec;
template <> struct UnitVec<1> { typedef uint32_t type; };
template <> struct UnitVec<2> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <> struct UnitVec<4> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

// The TV blocks of one ring slot in registers, read and written one access
// unit at a time (ring_slot_unit).
template <typename T, int D, int TV>
struct SlotRegs {
  static constexpr int UW = ring_slot_unit(TV, D, (int)sizeof(T)) / 4;   // words per unit
  static constexpr int NW = (TV * D * D * (int)sizeof(T) / 4 + UW - 1) / UW * UW;   // data words, whole units
  typedef typename UnitVec<UW>::type unit_t;
  uint32_t w[NW];
  __device__ __forceinline__ void load(const uint32_t* slot) {
    const unit_t* src = reinterpret_cast<const unit_t*>(slot);
#pragma unroll
    for (int c = 0; c < NW / UW; ++c) {
      const unit_t u = src[c];
      if constexpr (UW == 1) {
        w[c] = u;
      } else {
#pragma unroll
        for (int e = 0; e < UW; ++e) w[c * UW + e] = u[e];
      }
    }
  }
  __device__ __forceinline__ void store(uint32_t* slot) const {
    unit_t* dst = reinterpret_cast<unit_t*>(slot);
#pragma unroll
    for (int c = 0; c < NW / UW; ++c) {
      unit_t u;
      if constexpr (UW == 1) {
        u = w[c];
      } else {
#pragma unroll
        for (int e = 0; e < UW; ++e) u[e] = w[c * UW + e];
      }
      dst[c] = u;
    }
  }
  __device__ __forceinline__ T get(int idx) const {        // idx = v * D*D + r
    if constexpr (sizeof(T) == 4) {
      return __builtin_bit_cast(float, w[idx]);
    } else {
      return __builtin_bit_cast(double, (uint64_t)w[2 * idx] | ((uint64_t)w[2 * idx + 1] << 32));
    }
  }
  __device__ __forceinline__ void set(int idx, T x) {
    if constexpr (sizeof(T) == 4) {
      w[idx] = __builtin_bit_cast(uint32_t, x);
    } else {
      const uint64_t b = __builtin_bit_cast(uint64_t, x);
      w[2 * idx] = (uint32_t)b;
      w[2 * idx + 1] = (uint32_t)(b >> 32);
    }
  }
};

template <typename T, int D, int TV, int CH>
__device__ __forceinline__ void prep_band_body(const MeshView& mv, int method, int i0, int nv,
                                               const T* __restrict__ hb, T* __restrict__ KL, T* smem,
                                               const double* __restrict__ g, double* __restrict__ bout) {
  constexpr int DD = D * D, NW = CH / 64, NR = DD + D, SLW = ring_slot_words(TV, D, sizeof(T));
  const int nf = mv.nf, n = mv.n, bw = mv.band_w;
  const int R = min(nf, CH + bw);                   // ring length (band_ring)
  // position pos >= p0 (the current chunk's start) lives in slot
  // (pos - p0 + p0 % R) mod R; pos - p0 < CH + bw, so one conditional
  // subtraction of R reduces it
  auto wrap = [&](int t) { return (int)min((unsigned)t, (unsigned)(t - R)); };
  uint32_t* ring = reinterpret_cast<uint32_t*>(smem);              // [R][SLW] words
  T* red = reinterpret_cast<T*>(ring + (size_t)R * SLW);          // [NW][TV][NR]
  const T* Ub = basis_of<T>(mv);
  constexpr uint32_t RB = sizeof(BandRec<T, D>);
  const __amdgpu_buffer_rsrc_t hrs = buf_rsrc(mv.hq, (uint32_t)((size_t)mv.qmax * nf * RB));
  const int tid = threadIdx.x;
  int rows[TV];
#pragma unroll
  for (int v = 0; v < TV; ++v) rows[v] = i0 + (v < nv ? v : 0);
  auto put = [&](int pos, T (&blk)[TV][DD]) {
    SlotRegs<T, D, TV> sr;
#pragma unroll
    for (int v = 0; v < TV; ++v)
#pragma unroll
      for (int r = 0; r < DD; ++r) sr.set(v * DD + r, blk[v][r]);
    sr.store(ring + (size_t)pos * SLW);            // pos: a slot
  };
  // one buffer resource per basis row (a dense basis can pass 4 GiB, one
  // row cannot), so a block's offset is pos * D*D * sizeof(T)
  __amdgpu_buffer_rsrc_t urs[TV];
#pragma unroll
  for (int v = 0; v < TV; ++v)
    urs[v] = buf_rsrc(Ub + (size_t)rows[v] * nf * DD, (uint32_t)((size_t)nf * DD * sizeof(T)));
  auto fetch = [&](int pos, T (&blk)[TV][DD]) {
    const uint32_t off = (uint32_t)pos * (uint32_t)(DD * sizeof(T));
#pragma unroll
    for (int v = 0; v < TV; ++v)
#pragma unroll
      for (int r = 0; r < DD; ++r) {
        if constexpr (sizeof(T) == 4) {
          blk[v][r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(urs[v], off + 4u * r, 0, 0));
        } else {
          const auto u = __builtin_amdgcn_raw_buffer_load_b64(urs[v], off + 8u * r, 0, 0);
          blk[v][r] = __builtin_bit_cast(double, u);
        }
      }
  };
  int lo = R;                                       // first fill: positions [0, R) in slots [0, R)
  for (int pos = tid; pos < lo; pos += CH) {
    T blk[TV][DD];
    fetch(pos, blk);
    put(pos, blk);
  }
  int lo_slot = 0;                                  // lo % R
  int p0_slot = 0;                                  // p0 % R
  __syncthreads();
  T Y[TV][DD], Bv[TV][D];
#pragma unroll
  for (int v = 0; v < TV; ++v) {
#pragma unroll
    for (int r = 0; r < DD; ++r) Y[v][r] = T(0);
#pragma unroll
    for (int r = 0; r < D; ++r) Bv[v][r] = T(0);
  }
  for (int p0 = 0; p0 < nf; p0 += CH) {
    // chunk p0 + CH needs positions up to p0 + 2 CH + bw: prefetch them
    const int nhi = min(nf, p0 + 2 * CH + bw);
    const int ppos = lo + tid;
    const bool pf = ppos < nhi;
    T pre[TV][DD];
    if (pf) fetch(ppos, pre);
    const int p = p0 + tid;
    const int cshift = p0_slot - p0;                // slot = wrap(pos + cshift)
    if (p < nf) {
      const int cnt = gptr(mv.bq_cnt)[p];
      T W[TV][DD];
      // W_j = sum_q H''_{j,q} U_{k(q)}.  Record 0 is the diagonal block
      // (always present), applied with the row's own U_j, which the Y update
      // below needs anyway, so that it costs no ring read of its own.  With
      // three or four float32 rows U_j is read first and the diagonal product
      // sets W (no clearing of the accumulators, which the compiler emits
      // twice around the loop's guard; three rows then hold two waves per
      // SIMD instead of three, which their LDS ring allows anyway on the
      // meshes whose band sends them there); with fewer rows, whose occupancy
      // the extra live registers would cut, W is cleared and the diagonal
      // block comes last.  The other upper blocks run in a software pipeline unrolled by
      // two: block q + 1 (its H and column) is loaded while block q's LDS
      // reads and products run.  Records past the row's count are zero
      // padding or past the end of the buffer (read as zero) and are never
      // used.
      constexpr bool own_first = sizeof(T) == 4 && TV >= 3;
      auto product = [&](const RecWords<T, D>& rc, const SlotRegs<T, D, TV>& sr, bool first) {
#pragma unroll
        for (int v = 0; v < TV; ++v) {
          T U[DD];
#pragma unroll
          for (int r = 0; r < DD; ++r) U[r] = sr.get(v * DD + r);
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
              T acc = first ? rc.h(r * D) * U[c] : W[v][r * D + c] + rc.h(r * D) * U[c];
#pragma unroll
              for (int l = 1; l < D; ++l) acc += rc.h(r * D + l) * U[l * D + c];
              W[v][r * D + c] = acc;
            }
        }
      };
      auto consume = [&](const RecWords<T, D>& rc) {
        SlotRegs<T, D, TV> sr;
        sr.load(ring + (size_t)wrap(rc.pos() + cshift) * SLW);
        product(rc, sr, false);
      };
      const uint32_t step = (uint32_t)nf * RB;
      uint32_t off = (uint32_t)p * RB;
      RecWords<T, D> rd, ra, rb;
      SlotRegs<T, D, TV> sj;
      rd.fetch(hrs, off);                           // the diagonal block
      off += step;
      ra.fetch(hrs, off);
      if constexpr (own_first) {
        sj.load(ring + (size_t)wrap(p + cshift) * SLW);
        product(rd, sj, true);
      } else {
#pragma unroll
        for (int v = 0; v < TV; ++v)
#pragma unroll
          for (int r = 0; r < DD; ++r) W[v][r] = T(0);
      }
      int q = 1;
      for (; q + 1 < cnt; q += 2) {
        rb.fetch(hrs, off + step);
        consume(ra);
        ra.fetch(hrs, off + 2 * step);
        consume(rb);
        off += 2 * step;
      }
      if (q < cnt) consume(ra);
      T gj[D];
      if (g != nullptr) {
        const int j = gptr(mv.bvert)[p];
        double gd[D];
#pragma unroll
        for (int c = 0; c < D; ++c) gd[c] = gptr(g)[(size_t)c * n + j];
        if (mv.rot != nullptr) {              // R_j^T g_j
          const auto* Rj = gptr(mv.rot) + (size_t)j * DD;
#pragma unroll
          for (int c = 0; c < D; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < D; ++l) acc += Rj[l * D + c] * gd[l];
            gj[c] = T(acc);
          }
        } else {
#pragma unroll
          for (int c = 0; c < D; ++c) gj[c] = T(gd[c]);
        }
      }
      if constexpr (!own_first) {
        sj.load(ring + (size_t)wrap(p + cshift) * SLW);
        product(rd, sj, false);
      }
#pragma unroll
      for (int v = 0; v < TV; ++v) {
        T Uj[DD];
#pragma unroll
        for (int r = 0; r < DD; ++r) Uj[r] = sj.get(v * DD + r);
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
          for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) Y[v][r * D + c] += Uj[l * D + r] * W[v][l * D + c];
        if (g != nullptr)
#pragma unroll
          for (int r = 0; r < D; ++r) {
            T acc = T(0);
#pragma unroll
            for (int l = 0; l < D; ++l) acc += Uj[l * D + r] * gj[l];
            Bv[v][r] += acc;
          }
      }
    }
    __syncthreads();                                // chunk p0's ring reads are done
    if (pf) put(wrap(lo_slot + tid), pre);
    if (nhi > lo) {
      lo_slot = wrap(lo_slot + (nhi - lo));
      lo = nhi;
    }
    p0_slot = wrap(p0_slot + CH);
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < TV; ++v) {
#pragma unroll
    for (int r = 0; r < DD; ++r) Y[v][r] = wave_sum63(Y[v][r]);
#pragma unroll
    for (int r = 0; r < D; ++r) Bv[v][r] = wave_sum63(Bv[v][r]);
  }
  const int w = tid / 64, l = tid % 64;
  if (l == 63)
#pragma unroll
    for (int v = 0; v < TV; ++v) {
#pragma unroll
      for (int r = 0; r < DD; ++r) red[(w * TV + v) * NR + r] = Y[v][r];
#pragma unroll
      for (int r = 0; r < D; ++r) red[(w * TV + v) * NR + DD + r] = Bv[v][r];
    }
  __syncthreads();
  T* tot = smem;                                    // the ring is free now: [TV][NR]
  if (tid < TV * NR) {
    T acc = T(0);
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) acc += red[ww * TV * NR + tid];
    tot[tid] = acc;
  }
  __syncthreads();
  // one wave per row (rows w, w + NW, ... when the chunk has fewer waves
  // than rows)
  for (int v = w; v < nv; v += NW) {
    const int i = i0 + v;
    T A[DD];
#pragma unroll
    for (int r = 0; r < DD; ++r) A[r] = T(0);
    const int q1 = gptr(mv.rowptr)[i + 1];
    for (int q = gptr(mv.rowptr)[i] + 1 + l; q < q1; q += 64) {
      const int k = gptr(mv.colidx)[q];
      T Uk[DD];
      band_load<T, D>(mv, Ub, i, gptr(mv.bpos)[k], Uk);
      if (mv.rot != nullptr) rotate_block<T, D>(mv.rot, k, Uk);
      const auto* H = gptr(hb) + (size_t)q * DD;
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) {
          T acc = T(0);
#pragma unroll
          for (int t = 0; t < D; ++t) acc += H[r * D + t] * Uk[t * D + c];
          A[r * D + c] += acc;
        }
    }
#pragma unroll
    for (int r = 0; r < DD; ++r) A[r] = wave_sum63(A[r]);
    if (l != 63) continue;
    // A and Ht go to the vertex's K, L slots; dm_finish_body turns them into
    // K and L with one thread per vertex.  b_i = U_i^T (R^T g)_C, the
    // corotated basis's U_i^T g_C.
    const T* Yt = tot + v * NR;
    auto* out = gptr_w(KL) + (size_t)i * 2 * DD;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        out[r * D + c] = A[r * D + c];
        out[DD + r * D + c] = Yt[r * D + c] + Yt[c * D + r];
      }
    if (bout != nullptr)
#pragma unroll
      for (int r = 0; r < D; ++r) gptr_w(bout)[(size_t)r * mv.n + i] = double(Yt[DD + r]);
  }
}

// With dout given, dout holds b_i on entry and receives dx_i = -K (g_i - L b_i)
// (the arithmetic of update_body).
template <typename T, int D>
__device__ __forceinline__ void dm_finish_body(const MeshView& mv, int method, int i,
                                               const T* __restrict__ hb, T* __restrict__ KL,
                                               unsigned long long* __restrict__ fb,
                                               const double* __restrict__ g, double* __restrict__ dout,
                                               const double* x = nullptr, double* xtrial = nullptr) {
  constexpr int DD = D * D;
  T A[DD], Ht[DD];
  const T* in = KL + (size_t)i * 2 * DD;
#pragma unroll
  for (int r = 0; r < DD; ++r) {
    A[r] = in[r];
    Ht[r] = in[DD + r];
  }
  cc_finish<T, D>(mv, method, i, mv.nf <= 1, A, Ht, hb, KL, fb);
  if (dout == nullptr) return;
  const int n = mv.n;
  const T* kl = KL + (size_t)i * 2 * DD;
  T b[D], gt[D];
#pragma unroll
  for (int c = 0; c < D; ++c) b[c] = T(dout[(size_t)c * n + i]);
#pragma unroll
  for (int r = 0; r < D; ++r) {
    T lb = T(0);
#pragma unroll
    for (int l = 0; l < D; ++l) lb += kl[DD + r * D + l] * b[l];
    gt[r] = T(g[(size_t)r * n + i] - double(lb));
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < D; ++l) acc += kl[r * D + l] * gt[l];
    dout[(size_t)r * n + i] = -double(acc);
    // the trial point x + d of this vertex (Jacobi: the batched path's axpy;
    // coloured sweep: x and xtrial are the same running state, moved in place)
    if (xtrial != nullptr) xtrial[(size_t)r * n + i] = x[(size_t)r * n + i] - double(acc);
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(WG) k_cc_dm_finish(MeshView mv, int method, int v0, int v1,
                                                     const T* __restrict__ hb, T* __restrict__ KL,
                                                     unsigned long long* __restrict__ fb,
                                                     const double* __restrict__ g, double* __restrict__ dout,
                                                     double* __restrict__ xmove) {
  const int i = v0 + blockIdx.x * WG + threadIdx.x;
  if (i < v1) dm_finish_body<T, D>(mv, method, i, hb, KL, fb, g, dout, xmove, xmove);
}

template <typename T, int D, int TV, int CH>
__global__ void __launch_bounds__(CH) k_cc_prep_band(MeshView mv, int method, int v0, int v1,
                                                      const T* __restrict__ hb, T* __restrict__ KL,
                                                      const double* __restrict__ g, double* __restrict__ bout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int i0 = v0 + blockIdx.x * TV;
  prep_band_body<T, D, TV, CH>(mv, method, i0, min(TV, v1 - i0), hb, KL, reinterpret_cast<T*>(smem_raw), g,
                               bout);
}


// dx_i = -K_i (g_i - L_i U_i^T g_C); written to d (Jacobi) or added to x
// (coloured sweep).  G lanes per vertex share its support.
template <typename T, int D, int G>
__device__ __forceinline__ void update_body(const MeshView& mv, int method, int i, bool active,
                                            int lane, const T* __restrict__ KL,
                                            const double* __restrict__ g, double* __restrict__ out,
                                            int accumulate) {
  constexpr int DD = D * D;
  const T* Ub = basis_of<T>(mv);
  const int n = mv.n;
  T b[D];
#pragma unroll
  for (int c = 0; c < D; ++c) b[c] = T(0);
  if (active && method != 0) {
    int64_t sp0, sp1;
    supp_range(mv, i, sp0, sp1);
    for (int64_t q = sp0 + lane; q < sp1; q += G) {
      const int j = supp_vertex(mv, q, sp0);
      T gj[D];
#pragma unroll
      for (int c = 0; c < D; ++c) gj[c] = T(g[c * n + j]);
      if (mv.rot) {                               // (R_j U)^T g_j = U^T (R_j^T g_j)
        T t[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < D; ++l) acc += T(mv.rot[(size_t)j * DD + l * D + c]) * gj[l];
          t[c] = acc;
        }
#pragma unroll
        for (int c = 0; c < D; ++c) gj[c] = t[c];
      }
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

template <typename T, int D, int G>
__global__ void __launch_bounds__(WG) k_cc_update(MeshView mv, int method, int v0, int v1,
                                                  const T* __restrict__ KL,
                                                  const double* __restrict__ g,
                                                  double* __restrict__ out, int accumulate) {
  const int i = v0 + blockIdx.x * (WG / G) + threadIdx.x / G;
  update_body<T, D, G>(mv, method, i, i < v1, threadIdx.x % G, KL, g, out, accumulate);
}

// Step energy: blocks [0, nbe) sum element energies, the rest the free-vertex
// inertia and gravity terms; one partial per block.
// Block b < nbe sums element energies, the others free-vertex terms.
template <int D, bool FCR>
__device__ __forceinline__ double energy_body(const MeshView& mv, int b, int nbe,
                                              const double* __restrict__ x,
                                              const double* __restrict__ xt, const Material& mat) {
  double v = 0.0;
  const int n = mv.n;
  if (b < nbe) {
    const int e = b * WG + threadIdx.x;
    if (e < mv.m) {
      double F[D][D], beta[D + 1][D], vol;
      load_element<double, D>(mv, e, x, F, beta, vol);
      v = mat.s_el * vol * material_psi<double, D>(F, mat.mu, mat.lam, FCR ? mat.model : MAT_SNH);
    }
  } else {
    const int j = (b - nbe) * WG + threadIdx.x;
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
  return v;
}

// energy_body at the positions x + alpha d (formed as the trial-point update
// forms them), block for block.
template <int D, bool FCR>
__device__ __forceinline__ double energy_body_along(const MeshView& mv, int b, int nbe,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ d, double alpha,
                                                    const double* __restrict__ xt,
                                                    const Material& mat) {
  double v = 0.0;
  const int n = mv.n;
  if (b < nbe) {
    const int e = b * WG + threadIdx.x;
    if (e < mv.m) {
      double F[D][D], beta[D + 1][D], vol;
      load_element_along<double, D>(mv, e, x, d, alpha, F, beta, vol);
      v = mat.s_el * vol * material_psi<double, D>(F, mat.mu, mat.lam, FCR ? mat.model : MAT_SNH);
    }
  } else {
    const int j = (b - nbe) * WG + threadIdx.x;
    if (j < mv.nf) {
      const double mj = mv.mass[j];
      double in = 0.0, gr = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double p = x[c * n + j] + alpha * d[c * n + j];
        const double dx = p - xt[c * n + j];
        in += dx * dx;
        gr += mat.grav[c] * p;
      }
      v = mat.w_in * 0.5 * mj * in - mat.s_el * mj * gr;
    }
  }
  return v;
}

template <int D, bool FCR>
__global__ void __launch_bounds__(WG) k_energy(MeshView mv, const double* __restrict__ x,
                                               const double* __restrict__ xt, Material mat,
                                               int nbe, double* __restrict__ partials) {
  __shared__ double red[WG];
  const double v = energy_body<D, FCR>(mv, blockIdx.x, nbe, x, xt, mat);
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
                           const double* __restrict__ xt, const double* __restrict__ x0, double h, int quasi,
                           double* __restrict__ xu, double* __restrict__ vu) {
  const int v = blockIdx.x * WG + threadIdx.x;
  if (v >= mv.n) return;
  const int u = vperm[v], n = mv.n;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double xn = x[c * n + v];
    xu[u * D + c] = xn;
    vu[u * D + c] = quasi ? 0.0 : (xn - x0[c * n + v]) / h;
    if (mv.corr) mv.corr[c * n + v] = v < mv.nf ? xn - xt[c * n + v] : 0.0;
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
                             const T* __restrict__ est, T mu, T lam, int model, double* __restrict__ ge,
                             double* __restrict__ He) {
  constexpr int K = D + 1, DD = D * D;
  const int e = blockIdx.x * WG + threadIdx.x;
  if (e >= mv.m) return;
  const int eu = eperm[e];
  T F[D][D], beta[K][D], vol, P[D][D];
  load_element<T, D>(mv, e, x, F, beta, vol);
  material_pk1<T, D>(F, mu, lam, model, P);
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

// Material-dependent kernels come in two builds: FCR = false compiles the
// stable neo-Hookean path alone (its register budget untouched by the
// Fixed Corotational SVD); FCR = true follows each mesh's model at run time.
#define CC_DISPATCH_MAT(any_fcr, ...)                          \
  do {                                                         \
    if (any_fcr) { constexpr bool FCR = true; __VA_ARGS__; }   \
    else { constexpr bool FCR = false; __VA_ARGS__; }          \
  } while (0)

void launch_predict(const MeshView& mv, const int* vperm, const double* x_user, const double* v_user,
                    const double* x_bc, double h, int quasi, double* x, double* xt, double* x0,
                    int* bad, hipStream_t s) {
  CC_DISPATCH_D(mv.D, k_predict<D><<<nblocks(mv.n, WG), WG, 0, s>>>(mv, vperm, x_user, v_user, x_bc,
                                                                   h, quasi, x, xt, x0, bad));
}

void launch_finalize(const MeshView& mv, const int* vperm, const double* x, const double* xt, const double* x0,
                     double h, int quasi, double* x_user, double* v_user, hipStream_t s) {
  CC_DISPATCH_D(mv.D, k_finalize<D><<<nblocks(mv.n, WG), WG, 0, s>>>(mv, vperm, x, xt, x0, h, quasi,
                                                                    x_user, v_user));
}

void launch_elem_hess_list(const MeshView& mv, int prec, const double* x, const Material& mat,
                           double scale, void* estore, hipStream_t s, const int* elist, int count) {
  if (count <= 0) return;
  const int nb = nblocks(count, EWG);
  if (prec == 0)
    CC_DISPATCH_MAT(mat.model == MAT_FCR,
                    CC_DISPATCH_D(mv.D, k_elem_hess<double, D, FCR><<<nb, elem_threads<double>(), 0, s>>>(
                                            mv, x, mat.mu, mat.lam, mat.model, scale, (double*)estore, elist,
                                            count)));
  else
    CC_DISPATCH_MAT(mat.model == MAT_FCR,
                    CC_DISPATCH_D(mv.D, k_elem_hess<float, D, FCR><<<nb, elem_threads<float>(), 0, s>>>(
                                            mv, x, (float)mat.mu, (float)mat.lam, mat.model, (float)scale,
                                            (float*)estore, elist, count)));
}

void launch_elem_hess(const MeshView& mv, int prec, const double* x, const Material& mat,
                      double scale, void* estore, hipStream_t s) {
  launch_elem_hess_list(mv, prec, x, mat, scale, estore, s, nullptr, mv.m);
}

void launch_assemble(const MeshView& mv, int prec, const void* estore, const Material& mat,
                     void* hb, hipStream_t s) {
  launch_assemble_list(mv, prec, estore, mat, hb, s, nullptr, mv.nnzb);
}

void launch_band_copy(const MeshView& mv, int prec, const void* hb, hipStream_t s) {
  if (mv.hq == nullptr || mv.nnzb <= 0) return;
  const int nb = nblocks(mv.nnzb, EWG);
  if (prec == 0) CC_DISPATCH_D(mv.D, k_band_copy<double, D><<<nb, EWG, 0, s>>>(mv, (const double*)hb));
  else CC_DISPATCH_D(mv.D, k_band_copy<float, D><<<nb, EWG, 0, s>>>(mv, (const float*)hb));
}

void launch_assemble_list(const MeshView& mv, int prec, const void* estore, const Material& mat, void* hb,
                          hipStream_t s, const int* slist, int count) {
  if (count <= 0) return;
  const int nb = nblocks(count, EWG);
  if (prec == 0)
    CC_DISPATCH_D(mv.D, k_assemble<double, D><<<nb, EWG, 0, s>>>(mv, (const double*)estore, mat.w_in,
                                                               (double*)hb, slist, count));
  else
    CC_DISPATCH_D(mv.D, k_assemble<float, D><<<nb, EWG, 0, s>>>(mv, (const float*)estore, (float)mat.w_in,
                                                              (float*)hb, slist, count));
}

constexpr int GRAD_G = 16;   // lanes per vertex of the gradient: a 3D star holds about 24 elements

int reduce_partials_capacity(const MeshView& mv) {
  // energy partials followed by gradient partials (kb_energy_grad)
  const int a = nblocks(mv.nf, WG / GRAD_G);
  const int b = nblocks(mv.m, WG) + nblocks(mv.nf, WG);
  return a + b + 1;
}

void launch_gradient(const MeshView& mv, const double* x, const double* xt, const Material& mat,
                     double* g, double* partials, int* nparts, hipStream_t s) {
  const int nb = nblocks(mv.nf, WG / GRAD_G);
  *nparts = nb;
  if (nb == 0) return;
  CC_DISPATCH_MAT(mat.model == MAT_FCR,
                  CC_DISPATCH_D(mv.D, k_gradient<D, GRAD_G, FCR><<<nb, WG, 0, s>>>(mv, x, xt, mat, g, partials)));
}

// LDS of the staged support rows per workgroup: 32 KB keeps five 256-thread
// workgroups per CU.  Longer rows are read from global memory instead.
constexpr size_t SPARSE_STAGE_MAX = 32 * 1024;

static int sparse_stage_cap(int supp, int G, int D, int prec) {
  const size_t bytes = (size_t)(WG / G) * supp * D * D * (prec == 0 ? 8 : 4);
  return supp > 0 && bytes <= SPARSE_STAGE_MAX ? supp : 0;
}

static size_t sparse_stage_bytes(int cap, int G, int D, int prec) {
  return (size_t)(WG / G) * cap * D * D * (prec == 0 ? 8 : 4);
}

template <typename T, int D>
static void prep_g(const MeshView& mv, int method, int v0, int v1, const void* hb, void* KL,
                   unsigned long long* fb, int G, hipStream_t s) {
  const int cnt = v1 - v0;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const int cap = sparse_stage_cap(mv.smap ? mv.smap_supp : 0, G, D, prec);
  const size_t lds = sparse_stage_bytes(cap, G, D, prec);
  if (G == 64)
    k_cc_prep<T, D, 64><<<nblocks(cnt, WG / 64), WG, lds, s>>>(mv, method, v0, v1, (const T*)hb,
                                                               (T*)KL, fb, cap);
  else
    k_cc_prep<T, D, 16><<<nblocks(cnt, WG / 16), WG, lds, s>>>(mv, method, v0, v1, (const T*)hb,
                                                               (T*)KL, fb, cap);
}

static int support_lanes(const MeshView& mv) {
  if (mv.dense_supp) return 64;
  const double avg = mv.nf > 0 ? double(mv.nnzb) / mv.nf : 0.0;  // proxy: row length
  (void)avg;
  return 16;
}

static size_t g_lds_limit = 64 * 1024;

void set_lds_limit(size_t bytes) { g_lds_limit = bytes; }

int band_ring(int nf, int band_w, int ch) {
  if (nf <= 0) return 0;
  return std::min(nf, ch + band_w);
}

// Resident waves per SIMD that the registers of the dense condensation allow
// (gfx950 builds of prep_band_body, 3D: float32 228 / 182 / 122 / 79 VGPRs
// for 4 / 3 / 2 / 1 rows, float64 226 / 149 for 2 / 1 rows)
static int dense_reg_waves(int prec, int tv) {
  if (prec == 0) return tv >= 2 ? 2 : 3;
  return tv >= 3 ? 2 : tv == 2 ? 4 : 6;
}

size_t dense_lds_bytes(int tv, int ring, int D, int prec, int ch) {
  const size_t S = prec == 0 ? 8 : 4;
  // ring slots (ring_slot_words), then the per-wave partial sums
  return (size_t)ring * ring_slot_words(tv, D, (int)S) * 4 + (size_t)(ch / 64) * tv * (D * D + D) * S;
}

// float64 keeps at most two rows per workgroup (the register file of 2
// waves/SIMD holds the accumulators of two float64 rows, four float32 ones).
// Among chunks that leave as many waves resident, the smallest wins: more,
// shorter workgroups fill the last round of a launch better.  With the rows
// chosen automatically, the most rows that still let two workgroups share a
// CU come first (one workgroup's barriers and ring fill then overlap the
// other's products); only when no row count allows two does one per CU do.
DenseCfg dense_config(const int* nf, const int* band_w, int count, int D, int prec, int cap, int chunk) {
  DenseCfg best;
  const int top = std::min(prec == 0 ? 2 : 4, cap > 0 ? cap : 4);
  for (int pass = cap > 0 ? 1 : 0; pass < 2 && best.tv == 0; ++pass)
    for (int tv = top; tv >= 1 && best.tv == 0; --tv) {
      int best_waves = 0;
      for (int ch : {128, 256, BWG}) {
        if (chunk > 0 && ch != chunk) continue;
        int ring = 0;
        for (int m = 0; m < count; ++m) ring = std::max(ring, band_ring(nf[m], band_w[m], ch));
        if (ring <= 0) continue;
        const size_t lds = dense_lds_bytes(tv, ring, D, prec, ch);
        if (lds > g_lds_limit || (pass == 0 && 2 * lds > g_lds_limit)) continue;
        const int waves = std::min((int)(g_lds_limit / lds) * (ch / 64), 4 * dense_reg_waves(prec, tv));
        if (waves > best_waves) {
          best_waves = waves;
          best.tv = tv;
          best.ch = ch;
          best.lds = lds;
        }
      }
    }
  return best;
}

#define CC_DISPATCH_TVCH(tv, ch, ...)                                                 \
  switch ((tv) * 1000 + (ch)) {                                                       \
    case 1128: { constexpr int TV = 1, CH = 128; __VA_ARGS__; } break;                \
    case 2128: { constexpr int TV = 2, CH = 128; __VA_ARGS__; } break;                \
    case 3128: { constexpr int TV = 3, CH = 128; __VA_ARGS__; } break;                \
    case 4128: { constexpr int TV = 4, CH = 128; __VA_ARGS__; } break;                \
    case 1256: { constexpr int TV = 1, CH = 256; __VA_ARGS__; } break;                \
    case 2256: { constexpr int TV = 2, CH = 256; __VA_ARGS__; } break;                \
    case 3256: { constexpr int TV = 3, CH = 256; __VA_ARGS__; } break;                \
    case 4256: { constexpr int TV = 4, CH = 256; __VA_ARGS__; } break;                \
    case 1512: { constexpr int TV = 1, CH = 512; __VA_ARGS__; } break;                \
    case 2512: { constexpr int TV = 2, CH = 512; __VA_ARGS__; } break;                \
    case 3512: { constexpr int TV = 3, CH = 512; __VA_ARGS__; } break;                \
    default: { constexpr int TV = 4, CH = 512; __VA_ARGS__; } break;                  \
  }

// True when the mesh's dense basis can be streamed through the LDS ring in
// this precision (float64 needs the float64 copy of the basis).
static bool band_ok(const MeshView& mv, int prec) {
  if (!mv.dense_supp || mv.hq == nullptr || mv.nf < 2) return false;
  if (prec == 0 && mv.U_d == nullptr) return false;
  return dense_config(&mv.nf, &mv.band_w, 1, mv.D, prec).tv > 0;
}

template <typename T, int D>
static bool prep_dense(const MeshView& mv, int prec, int method, int v0, int v1, const void* hb,
                       void* KL, unsigned long long* fb, const double* g, double* dout, double* xmove,
                       int tv_cap, int chunk, hipStream_t s) {
  if (method == 0 || !band_ok(mv, prec)) return false;
  const DenseCfg dc = dense_config(&mv.nf, &mv.band_w, 1, D, prec, tv_cap, chunk);
  if (dc.tv == 0) return false;
  CC_DISPATCH_TVCH(dc.tv, dc.ch, k_cc_prep_band<T, D, TV, CH><<<nblocks(v1 - v0, TV), CH, dc.lds, s>>>(
                                     mv, method, v0, v1, (const T*)hb, (T*)KL, g, dout));
  k_cc_dm_finish<T, D><<<nblocks(v1 - v0, WG), WG, 0, s>>>(mv, method, v0, v1, (const T*)hb, (T*)KL, fb,
                                                          g, dout, g != nullptr ? xmove : nullptr);
  return true;
}

bool launch_cc_prep(const MeshView& mv, int prec, int method, int v0, int v1, const void* hb,
                    void* KL, unsigned long long* fb, hipStream_t s, const double* g, double* dout,
                    double* xmove, int tv_cap, int chunk) {
  if (v1 <= v0) return g != nullptr;
  bool done = false;
  if (prec == 0)
    CC_DISPATCH_D(mv.D, done = prep_dense<double, D>(mv, prec, method, v0, v1, hb, KL, fb, g, dout, xmove,
                                                     tv_cap, chunk, s));
  else
    CC_DISPATCH_D(mv.D, done = prep_dense<float, D>(mv, prec, method, v0, v1, hb, KL, fb, g, dout, xmove,
                                                    tv_cap, chunk, s));
  if (done) return g != nullptr;
  const int G = support_lanes(mv);
  if (prec == 0) CC_DISPATCH_D(mv.D, prep_g<double, D>(mv, method, v0, v1, hb, KL, fb, G, s));
  else CC_DISPATCH_D(mv.D, prep_g<float, D>(mv, method, v0, v1, hb, KL, fb, G, s));
  return false;
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
  CC_DISPATCH_MAT(mat.model == MAT_FCR,
                  CC_DISPATCH_D(mv.D, k_energy<D, FCR><<<nbe + nbv, WG, 0, s>>>(mv, x, xt, mat, nbe, partials)));
}

void launch_reduce(const double* partials, int n, double* out, hipStream_t s) {
  k_reduce<<<1, WG, 0, s>>>(partials, n, out);
}

// R_j = U V^T from the rotation-variant SVD of
// M = sum_{k in N(j)} (x_k - x_j)(X_k - X_j)^T: the polar rotation (det +1).
template <int D>
__device__ __forceinline__ void rotation_body(const MeshView& mv, int j, const double* __restrict__ x,
                                              const int* __restrict__ nptr, const int* __restrict__ nidx,
                                              const double* __restrict__ Xr, double* __restrict__ rot) {
  if (j >= mv.nf) return;
  const int n = mv.n;
  double M[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) M[r][c] = 0.0;
  double xj[D], Xj[D];
#pragma unroll
  for (int c = 0; c < D; ++c) { xj[c] = x[(size_t)c * n + j]; Xj[c] = Xr[(size_t)c * n + j]; }
  for (int t = nptr[j]; t < nptr[j + 1]; ++t) {
    const int k = nidx[t];
    double dx[D], dX[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      dx[c] = x[(size_t)c * n + k] - xj[c];
      dX[c] = Xr[(size_t)c * n + k] - Xj[c];
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int c = 0; c < D; ++c) M[r][c] += dx[r] * dX[c];
  }
  double U[D][D], V[D][D], sig[D];
  svd_rv<double, D>(M, U, V, sig);
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) acc += U[r][l] * V[c][l];
      rot[(size_t)j * D * D + r * D + c] = acc;
    }
}

template <int D>
__global__ void __launch_bounds__(WG) k_rotations(MeshView mv, const double* __restrict__ x,
                                                  const int* __restrict__ nptr, const int* __restrict__ nidx,
                                                  const double* __restrict__ Xr, double* __restrict__ rot) {
  rotation_body<D>(mv, blockIdx.x * WG + threadIdx.x, x, nptr, nidx, Xr, rot);
}

void launch_rotations(const MeshView& mv, const double* x, const int* nptr, const int* nidx,
                      const double* Xr, double* rot, hipStream_t s) {
  if (mv.nf <= 0 || !x || !nptr || !nidx || !Xr || !rot) return;
  CC_DISPATCH_D(mv.D, k_rotations<D><<<nblocks(mv.nf, WG), WG, 0, s>>>(mv, x, nptr, nidx, Xr, rot));
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
                                                                 mat.mu, mat.lam, mat.model, ge, He));
  else
    CC_DISPATCH_D(mv.D, k_probe_elem<float, D><<<nb, WG, 0, s>>>(mv, xi_tmp, eperm, (const float*)est,
                                                                (float)mat.mu, (float)mat.lam, mat.model, ge,
                                                                He));
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

// ===========================================================================
// Batched stepping: every launch covers all meshes of a batch; block b of a
// launch belongs to mesh m when boff[m] <= b < boff[m+1].  Meshes whose
// control block is inactive return at once, so a captured sequence of
// launches stays valid while meshes finish at different iterations.
namespace cc {


__device__ __forceinline__ const double* pick(const BatchItem& it, int which) {
  return which ? it.xtrial : it.x;
}

__device__ __forceinline__ void vertex_range(const BatchItem& it, int colour, int& v0, int& v1) {
  if (colour < 0) { v0 = 0; v1 = it.mv.nf; }
  else if (colour < it.ncol) { v0 = it.coff[colour]; v1 = it.coff[colour + 1]; }
  else { v0 = v1 = 0; }
}

// Start of a step: control block and fallback counters of every mesh.
__global__ void kb_reset(const BatchItem* __restrict__ items, BatchCtl* ctl, int nmesh) {
  const int m = blockIdx.x * WG + threadIdx.x;
  if (m >= nmesh) return;
  BatchCtl c{};
  c.active = 1;
  c.status = -100;
  ctl[m] = c;
  unsigned long long* fb = items[m].fb;
#pragma unroll
  for (int q = 0; q < 4; ++q) fb[q] = 0ull;
}

template <int D>
__global__ void __launch_bounds__(WG) kb_predict(const BatchItem* __restrict__ items, BatchCtl* ctl,
                                                 const int* __restrict__ boff, int nmesh, double h,
                                                 int quasi) {
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const int v = (blockIdx.x - boff[mi]) * WG + threadIdx.x;
  if (v >= mv.n) return;
  const int u = mv.vperm[v], n = mv.n;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double xp = it.xu[u * D + c], vp = it.vu[u * D + c];
    ok = ok && isfinite(xp) && isfinite(vp);
    it.x0[c * n + v] = xp;
    double xh;
    if (v < mv.nf) {
      xh = quasi ? xp : xp + h * vp;
    } else {
      xh = it.xbc ? it.xbc[u * D + c] : xp;
      ok = ok && isfinite(xh);
    }
    it.xt[c * n + v] = xh;
    it.x[c * n + v] = xh;
    // both position buffers start equal, so the Dirichlet entries of the
    // trial buffer hold the targets whichever buffer the step ends in
    it.xtrial[c * n + v] = xh;
  }
  if (!ok) atomicOr(&ctl[mi].bad, 1);
}

template <int D>
__global__ void __launch_bounds__(WG) kb_finalize(const BatchItem* __restrict__ items,
                                                  const int* __restrict__ boff, int nmesh, double h,
                                                  int quasi) {
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const int v = (blockIdx.x - boff[mi]) * WG + threadIdx.x;
  if (v >= mv.n) return;
  const int u = mv.vperm[v], n = mv.n;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double xn = it.x[c * n + v];
    it.xu[u * D + c] = xn;
    it.vu[u * D + c] = quasi ? 0.0 : (xn - it.x0[c * n + v]) / h;
    if (mv.corr) mv.corr[c * n + v] = v < mv.nf ? xn - it.xt[c * n + v] : 0.0;
  }
}

template <typename T, int D, bool FCR>
__global__ void __launch_bounds__(elem_threads<T>()) kb_elem_hess(const BatchItem* __restrict__ items,
                                                   const BatchCtl* __restrict__ ctl,
                                                   const int* __restrict__ boff, int nmesh, int which,
                                                   int colour) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  // colour >= 0: only the elements that colour's moves changed
  const bool lst = colour >= 0 && colour < it.ncol;
  const int* el = lst ? mv.cel + mv.cel_ptr[colour] : nullptr;
  const int cnt = lst ? mv.cel_ptr[colour + 1] - mv.cel_ptr[colour] : mv.m;
  elem_hess_split<T, D>(mv, (bx - boff[mi]) * EWG, pick(it, which), T(it.mat.mu), T(it.mat.lam),
                        FCR ? it.mat.model : MAT_SNH, T(it.mat.s_el), (T*)it.estore, el, cnt);
}

// Corotation: vertex rotations of every mesh at positions `which`.
template <int D>
__global__ void __launch_bounds__(WG) kb_rotations(const BatchItem* __restrict__ items,
                                                   const BatchCtl* __restrict__ ctl,
                                                   const int* __restrict__ boff, int nmesh, int which) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  if (it.mv.rot == nullptr) return;
  rotation_body<D>(it.mv, (bx - boff[mi]) * WG + threadIdx.x, pick(it, which), it.nptr, it.nidx,
                   it.Xr, const_cast<double*>(it.mv.rot));
}

template <typename T, int D>
__global__ void __launch_bounds__(EWG) kb_assemble(const BatchItem* __restrict__ items,
                                                  const BatchCtl* __restrict__ ctl,
                                                  const int* __restrict__ boff, int nmesh, int colour) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const bool lst = colour >= 0 && colour < it.ncol;
  const int* sl = lst ? mv.csl + mv.csl_ptr[colour] : nullptr;
  const int cnt = lst ? mv.csl_ptr[colour + 1] - mv.csl_ptr[colour] : mv.nnzb;
  assemble_body<T, D>(mv, (bx - boff[mi]) * EWG + threadIdx.x, (const T*)it.estore,
                      T(it.mat.w_in), (T*)it.hb, sl, cnt);
}

// Every BandRec of the dense-basis meshes from their block rows and current
// rotations (after a partial assembly of corotated meshes).
template <typename T, int D>
__global__ void __launch_bounds__(EWG) kb_band_copy(const BatchItem* __restrict__ items,
                                                   const BatchCtl* __restrict__ ctl,
                                                   const int* __restrict__ boff, int nmesh) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const MeshView& mv = it.mv;
  if (mv.hq == nullptr) return;
  const int t = (bx - boff[mi]) * EWG + threadIdx.x;
  if (t < mv.nnzb) band_rec_write<T, D>(mv, t, mv.blkrow[t], (const T*)it.hb + (size_t)t * D * D);
}

template <int D, int G, bool FCR>
__global__ void __launch_bounds__(WG) kb_gradient(const BatchItem* __restrict__ items,
                                                  const BatchCtl* __restrict__ ctl,
                                                  const int* __restrict__ boff, int nmesh, int which,
                                                  int only_warm) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  __shared__ double red[WG];
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active || (only_warm && !ctl[mi].warm)) return;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const int lb = bx - boff[mi];
  const double gsq = gradient_body<D, G, FCR>(mv, grad_vertex(mv, lb * (WG / G) + threadIdx.x / G), threadIdx.x % G,
                                         pick(it, which), it.xt, it.mat, it.g);
  const double tot = block_sum<WG>(gsq, red);
  if (threadIdx.x == 0) it.partials[lb] = tot;
}

template <typename T, int D, int G>
__global__ void __launch_bounds__(WG) kb_prep(const BatchItem* __restrict__ items,
                                              const BatchCtl* __restrict__ ctl,
                                              const int* __restrict__ boff, int nmesh, int method,
                                              int colour, int cap) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  int v0, v1;
  vertex_range(it, colour, v0, v1);
  const int idx = (bx - boff[mi]) * (WG / G) + threadIdx.x / G;
  const bool act = idx < v1 - v0;
  prep_body<T, D, G>(it.mv, method, act ? sweep_vertex(it.mv, v0, v1, idx) : v0, act, threadIdx.x % G,
                     (const T*)it.hb, (T*)it.KL, it.fb,
                     cap > 0 ? reinterpret_cast<T*>(smem_raw) : nullptr, cap);
}

// Dense-basis meshes of a batch: TV vertices per workgroup (prep_band_body).
template <typename T, int D, int TV, int CH>
__global__ void __launch_bounds__(CH) kb_prep_band(const BatchItem* __restrict__ items,
                                                    const BatchCtl* __restrict__ ctl,
                                                    const int* __restrict__ boff, int nmesh,
                                                    int method, int colour, int fuse) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  int v0, v1;
  vertex_range(it, colour, v0, v1);
  const int i0 = v0 + (blockIdx.x - boff[mi]) * TV;
  prep_band_body<T, D, TV, CH>(it.mv, method, i0, min(TV, v1 - i0), (const T*)it.hb, (T*)it.KL,
                           reinterpret_cast<T*>(smem_raw), fuse ? it.g : nullptr, fuse ? it.d : nullptr);
}

template <typename T, int D>
__global__ void __launch_bounds__(WG) kb_dm_finish(const BatchItem* __restrict__ items,
                                                   const BatchCtl* __restrict__ ctl,
                                                   const int* __restrict__ boff, int nmesh,
                                                   int method, int colour, int fuse) {
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  int v0, v1;
  vertex_range(it, colour, v0, v1);
  const int i = v0 + (blockIdx.x - boff[mi]) * WG + threadIdx.x;
  // fuse 1 (Jacobi): xtrial = x + d; fuse 2 (coloured sweep): the colour's
  // vertices move in place in the sweep's running state xtrial
  if (i < v1)
    dm_finish_body<T, D>(it.mv, method, i, (const T*)it.hb, (T*)it.KL, it.fb, fuse ? it.g : nullptr,
                         fuse ? it.d : nullptr, fuse == 2 ? it.xtrial : it.x, fuse ? it.xtrial : nullptr);
}

template <typename T, int D, int G>
__global__ void __launch_bounds__(WG) kb_update(const BatchItem* __restrict__ items,
                                                const BatchCtl* __restrict__ ctl,
                                                const int* __restrict__ boff, int nmesh, int method,
                                                int colour, int into_trial) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  int v0, v1;
  vertex_range(it, colour, v0, v1);
  const int i = v0 + (bx - boff[mi]) * (WG / G) + threadIdx.x / G;
  update_body<T, D, G>(mv, method, i, i < v1, threadIdx.x % G, (const T*)it.KL, it.g,
                       into_trial ? it.xtrial : it.d, into_trial);
}

// xtrial = x + alpha d (copy_only: xtrial = x) over all D*n entries.
__global__ void __launch_bounds__(WG) kb_axpy(const BatchItem* __restrict__ items,
                                              const BatchCtl* __restrict__ ctl,
                                              const int* __restrict__ boff, int nmesh, double alpha,
                                              int copy_only) {
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const int t = (blockIdx.x - boff[mi]) * WG + threadIdx.x;
  if (t >= it.mv.D * it.mv.n) return;
  it.xtrial[t] = copy_only ? it.x[t] : it.x[t] + alpha * it.d[t];
}

// The end of a line-searched iteration in one launch: per mesh, the energy
// blocks at the trial point (as kb_energy) followed by the gradient blocks
// at the trial point (as kb_gradient), each writing its partial at its own
// block index.  The gradient is speculative: it is used only if the trial
// point is taken, and every path that leaves a mesh at its old x computes
// the gradient there again.
template <int D, bool FCR>
__global__ void __launch_bounds__(WG) kb_energy_grad(const BatchItem* __restrict__ items,
                                                     const BatchCtl* __restrict__ ctl,
                                                     const int* __restrict__ boff, int nmesh) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  __shared__ double red[WG];
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const int lb = bx - boff[mi];
  const int nbe = (mv.m + WG - 1) / WG;
  const int ne = nbe + (mv.nf + WG - 1) / WG;
  double v;
  if (lb < ne)
    v = energy_body<D, FCR>(mv, lb, nbe, it.xtrial, it.xt, it.mat);
  else
    v = gradient_body<D, GRAD_G, FCR>(mv, grad_vertex(mv, (lb - ne) * (WG / GRAD_G) + threadIdx.x / GRAD_G),
                                      threadIdx.x % GRAD_G, it.xtrial, it.xt, it.mat, it.g);
  const double tot = block_sum<WG>(v, red);
  if (threadIdx.x == 0) it.partials[lb] = tot;
}

template <int D, bool FCR>
__global__ void __launch_bounds__(WG) kb_energy(const BatchItem* __restrict__ items,
                                                const BatchCtl* __restrict__ ctl,
                                                const int* __restrict__ boff, int nmesh, int which) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  __shared__ double red[WG];
  const int mi = block_mesh(boff, nmesh, bx);
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const int lb = bx - boff[mi];
  const int nbe = (mv.m + WG - 1) / WG;
  const double v = energy_body<D, FCR>(mv, lb, nbe, pick(it, which), it.xt, it.mat);
  const double tot = block_sum<WG>(v, red);
  if (threadIdx.x == 0) it.partials[lb] = tot;
}

// Accept the iteration of an active mesh when E did not rise beyond the
// slack (or without line search); otherwise hand the mesh to the host for
// backtracking.
__device__ __forceinline__ void accept_mesh(BatchItem& item, BatchCtl& c, int line_search) {
  const double tau = 1e-12 * fmax(fabs(c.E_cur), 1.0);
  if (!line_search || c.E_trial <= c.E_cur + tau) {
    double* t = item.x;
    item.x = item.xtrial;
    item.xtrial = t;
    if (line_search) c.E_cur = c.E_trial;
    c.iters += 1;
  } else {
    c.needs_host = 1;
    c.active = 0;
  }
}

// Learned warm start: the proposal (in xtrial, its energy in E_trial)
// replaces the predictor when it has the lower step energy.
// tag: 1 the network's proposal, 2 the previous correction alone
__device__ __forceinline__ void warm_accept_mesh(BatchItem& item, BatchCtl& c, int tag) {
  if (c.E_trial < c.E_cur) {
    double* t = item.x;
    item.x = item.xtrial;
    item.xtrial = t;
    c.E_cur = c.E_trial;
    c.warm = tag;
  }
}

// Residual at an accepted proposal against the predictor's gradient norm g0.
__device__ __forceinline__ void warm_check_mesh(BatchCtl& c, double tol) {
  c.r = sqrt(c.gn2) / c.g0;
  if (c.r <= tol) { c.status = 0; c.active = 0; }
}

// Convergence test of an active mesh after its gradient norm is in gn2.
__device__ __forceinline__ void converged_mesh(BatchCtl& c, double tol, int max_iters) {
  c.r = sqrt(c.gn2) / c.g0;
  if (!isfinite(c.r)) { c.status = 2; c.active = 0; }
  else if (c.r <= tol) { c.status = 0; c.active = 0; }
  else if (c.iters >= max_iters) { c.status = 1; c.active = 0; }
}

// One workgroup per mesh: sums the partials written by the launch whose
// block offsets are boff_src; dst 0 -> E_trial, 1 -> gn2, 2 -> E_cur.  Then,
// on the same thread, post 1 applies the accept rule (dst 0) and post 2 the
// convergence test (dst 1), saving the launch of kb_accept / kb_converged.
// only_warm: meshes whose learned proposal was rejected are skipped (their
// positions, gradient and norm are those of the predictor, already known).
// Sum of a mesh's per-block partials, in a fixed order (the single-mesh
// k_reduce sums the same way).
__device__ __forceinline__ double mesh_partials_sum(const BatchItem& it, int np, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += WG) v += it.partials[i];
  return block_sum<WG>(v, red);
}

__global__ void __launch_bounds__(WG) kb_reduce(BatchItem* __restrict__ items, BatchCtl* ctl,
                                                const int* __restrict__ boff_src, int dst, int post,
                                                double tol, int max_iters, int only_warm) {
  __shared__ double red[WG];
  const int mi = blockIdx.x;
  if (!ctl[mi].active || (only_warm && !ctl[mi].warm)) return;
  const double tot = mesh_partials_sum(items[mi], boff_src[mi + 1] - boff_src[mi], red);
  if (threadIdx.x == 0) {
    BatchCtl& c = ctl[mi];
    if (dst == 0) c.E_trial = tot;
    else if (dst == 1) c.gn2 = tot;
    else c.E_cur = tot;
    if (post == 1) accept_mesh(items[mi], c, 1);
    else if (post == 2) converged_mesh(c, tol, max_iters);
    else if (post == 3) warm_accept_mesh(items[mi], c, 1);
    else if (post == 5) warm_accept_mesh(items[mi], c, 2);
    else if (post == 4) warm_check_mesh(c, tol);
  }
}

// Backtracking (Results, Subspace Quality: global line search along the
// sweep's displacement) of the active meshes, all meshes per launch.  The
// halvings alpha = 1/2, 1/4, ... are tried LS_WIDTH at a time: one launch
// evaluates E(x + alpha d) for each, and the decision takes the first that
// does not raise E, which is what trying them one after another would take.
// ctl.ls: 0 searching, 3 step found (to be written), 1 taken, 2 halvings
// exhausted.

// mode 0: d = x_trial - x for the active meshes; mode 1: x_trial = x + alpha d
// for the meshes whose step was found.
__global__ void __launch_bounds__(WG) kb_ls_vec(BatchItem* __restrict__ items,
                                                const BatchCtl* __restrict__ ctl,
                                                const int* __restrict__ boff, int nmesh, int mode) {
  const int mi = block_mesh(boff, nmesh, blockIdx.x);
  if (!ctl[mi].active || (mode == 1 && ctl[mi].ls != 3)) return;
  const BatchItem& it = items[mi];
  const int t = (blockIdx.x - boff[mi]) * WG + threadIdx.x;
  if (t >= it.mv.D * it.mv.n) return;
  if (mode == 0) it.d[t] = it.xtrial[t] + -1.0 * it.x[t];
  else it.xtrial[t] = it.x[t] + ctl[mi].alpha * it.d[t];
}

// Energy partials at x + alpha_k d, alpha_k = ctl.alpha / 2^k, k = blockIdx.y,
// laid out as kb_energy's partials, one set of `total` per k.
template <int D, bool FCR>
__global__ void __launch_bounds__(WG) kb_energy_wide(const BatchItem* __restrict__ items,
                                                     const BatchCtl* __restrict__ ctl,
                                                     const int* __restrict__ boff, int nmesh,
                                                     int total, int max_halvings,
                                                     double* __restrict__ wpart) {
  // blocks of one XCD take a contiguous range of the launch (one mesh, or
  // neighbouring ones), so each mesh's data stays in one L2
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  __shared__ double red[WG];
  const int mi = block_mesh(boff, nmesh, bx);
  const BatchCtl& c = ctl[mi];
  const int k = blockIdx.y;
  if (!c.active || c.ls != 0 || c.halvings + k > max_halvings) return;
  double alpha = c.alpha;
  for (int q = 0; q < k; ++q) alpha *= 0.5;
  const BatchItem& it = items[mi];
  const MeshView mv = it.mv;
  const int lb = bx - boff[mi];
  const int nbe = (mv.m + WG - 1) / WG;
  const double v = energy_body_along<D, FCR>(mv, lb, nbe, it.x, it.d, alpha, it.xt, it.mat);
  const double tot = block_sum<WG>(v, red);
  if (threadIdx.x == 0) wpart[(size_t)k * total + bx] = tot;
}

// Per mesh, in halving order: E at alpha_k (partials summed as kb_reduce
// sums them); the first that does not raise E beyond the slack is the step;
// at the halving limit the search stops; otherwise the next launch goes on
// from alpha / 2^width.
__global__ void __launch_bounds__(WG) kb_ls_reduce_wide(BatchCtl* ctl, const int* __restrict__ boff,
                                                        int total, int width, int max_halvings,
                                                        const double* __restrict__ wpart) {
  __shared__ double red[WG];
  const int mi = blockIdx.x;
  BatchCtl& c = ctl[mi];
  if (!c.active || c.ls != 0) return;
  const double tau = 1e-12 * fmax(fabs(c.E_cur), 1.0);
  const double Ecur = c.E_cur;
  const int np = boff[mi + 1] - boff[mi];
  double alpha = c.alpha, Et = 0.0;
  int h = c.halvings, ls = 0;
  for (int k = 0; k < width; ++k) {
    const double* part = wpart + (size_t)k * total + boff[mi];
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += WG) v += part[i];
    Et = block_sum<WG>(v, red);
    __syncthreads();                       // red is reused by the next sum
    if (Et <= Ecur + tau) { ls = 3; break; }
    if (h >= max_halvings) { ls = 2; break; }
    alpha *= 0.5;
    h += 1;
  }
  if (threadIdx.x != 0) return;
  c.E_trial = Et;
  c.alpha = alpha;
  c.halvings = h;
  c.ls = ls;
  if (ls == 2) c.active = 0;
}

// Takes the written steps: swap x and x_trial, E, one more iteration.
__global__ void kb_ls_commit(BatchItem* __restrict__ items, BatchCtl* ctl, int nmesh) {
  const int mi = blockIdx.x * WG + threadIdx.x;
  if (mi >= nmesh) return;
  BatchCtl& c = ctl[mi];
  if (!c.active || c.ls != 3) return;
  BatchItem& item = items[mi];
  double* t = item.x;
  item.x = item.xtrial;
  item.xtrial = t;
  c.E_cur = c.E_trial;
  c.iters += 1;
  c.ls = 1;
  c.active = 0;
}

// Both sums of kb_energy_grad (each in kb_reduce's order), then the accept
// rule and, for a mesh that took its trial point, the convergence test.
__global__ void __launch_bounds__(WG) kb_reduce_eg(BatchItem* __restrict__ items, BatchCtl* ctl,
                                                   double tol, int max_iters) {
  __shared__ double red[WG];
  const int mi = blockIdx.x;
  if (!ctl[mi].active) return;
  const BatchItem& it = items[mi];
  const int ne = (it.mv.m + WG - 1) / WG + (it.mv.nf + WG - 1) / WG;
  const int ng = (it.mv.nf + WG / GRAD_G - 1) / (WG / GRAD_G);
  const double E = mesh_partials_sum(it, ne, red);
  __syncthreads();                         // red is reused by the next sum
  double v = 0.0;
  for (int i = threadIdx.x; i < ng; i += WG) v += it.partials[ne + i];
  const double gn2 = block_sum<WG>(v, red);
  if (threadIdx.x != 0) return;
  BatchCtl& c = ctl[mi];
  c.E_trial = E;
  accept_mesh(items[mi], c, 1);
  if (c.active) {
    c.gn2 = gn2;
    converged_mesh(c, tol, max_iters);
  }
}

__global__ void kb_init(const BatchItem* items, BatchCtl* ctl, int nmesh, double tol, int max_iters) {
  const int m = blockIdx.x * WG + threadIdx.x;
  if (m >= nmesh) return;
  BatchCtl& c = ctl[m];
  if (c.bad) { c.status = -5; c.active = 0; return; }
  c.g0 = fmax(sqrt(c.gn2), items[m].load);   // relative to the larger of |g(x^0)| and the floor
  if (c.g0 == 0.0) { c.r = 0.0; c.status = 0; c.active = 0; return; }
  c.r = sqrt(c.gn2) / c.g0;
  if (c.r <= tol) { c.status = 0; c.active = 0; }
  else if (max_iters <= 0) { c.status = 1; c.active = 0; }
}

// Accept the iteration when E did not rise beyond the slack (or without line
// search); otherwise hand the mesh to the host for backtracking.
__global__ void kb_accept(BatchItem* items, BatchCtl* ctl, int nmesh, int line_search) {
  const int m = blockIdx.x * WG + threadIdx.x;
  if (m >= nmesh) return;
  if (!ctl[m].active) return;
  accept_mesh(items[m], ctl[m], line_search);
}

// ---- host side of a batch ---------------------------------------------------
struct Offsets {
  std::vector<int> h;
  int* d = nullptr;
  int total() const { return h.empty() ? 0 : h.back(); }
};

struct BatchPlan {
  int nmesh = 0;
  BatchConfig cfg{};
  std::vector<BatchItem> items_h;
  BatchItem* items_d = nullptr;
  BatchCtl* ctl_d = nullptr;
  Offsets pred, elem, asmb, grad, energy, axpy, axpyj, feat, rotn;   // axpyj: Jacobi trial points
  Offsets eg;       // energy then gradient blocks of each mesh (kb_energy_grad)
  std::vector<Offsets> elemc, asmbc;   // element / slot blocks of colour c's dirty lists
  std::vector<Offsets> prep, prepd, fin, upd;   // index 0: all free vertices, c+1: colour c
  int max_colours = 0;
  int tv = 0;       // vertices per workgroup of the dense condensation (0: no dense mesh)
  int ch = 0;       // its chunk of band positions (= workgroup size)
  size_t lds = 0;   // its dynamic LDS
  int scap = 0;     // staged support blocks per vertex of the sparse condensation (0: none)
  size_t slds = 0;  // its dynamic LDS
  double* wpart = nullptr;   // energy partials of LS_WIDTH backtracking steps
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_iters = 0;
  BatchHook hook = nullptr;
  void* hook_user = nullptr;
  int capturing = 0;
  int capture_failed = 0;   // graph capture failed: the iterations run uncaptured
  void mark(int kid, int begin) { if (hook) hook(hook_user, kid, begin); }
};

static void drop_graph(BatchPlan* p) {
  if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
  if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
}

void batch_set_hook(BatchPlan* p, BatchHook hook, void* user) {
  if (p->hook == hook && p->hook_user == user) return;
  drop_graph(p);
  p->hook = hook;
  p->hook_user = user;
}

int batch_capturing(BatchPlan* p) { return p->capturing; }
int batch_has_graph(BatchPlan* p) { return p->exec != nullptr; }

static void offsets_build(Offsets& o, const std::vector<int>& counts, hipStream_t s) {
  o.h.assign(counts.size() + 1, 0);
  for (size_t i = 0; i < counts.size(); ++i) o.h[i + 1] = o.h[i] + counts[i];
  if (o.d) (void)hipFree(o.d);
  (void)hipMalloc(&o.d, o.h.size() * sizeof(int));
  (void)hipMemcpyAsync(o.d, o.h.data(), o.h.size() * sizeof(int), hipMemcpyHostToDevice, s);
}

static void offsets_free(Offsets& o) {
  if (o.d) (void)hipFree(o.d);
  o.d = nullptr;
}

static void plan_vertex_offsets(BatchPlan* p, hipStream_t s) {
  const int G = p->cfg.G;
  p->prep.assign(p->max_colours + 1, Offsets{});
  p->prepd.assign(p->max_colours + 1, Offsets{});
  p->fin.assign(p->max_colours + 1, Offsets{});
  p->upd.assign(p->max_colours + 1, Offsets{});
  for (int c = -1; c < p->max_colours; ++c) {
    std::vector<int> cp(p->nmesh), cd(p->nmesh), cf(p->nmesh), cu(p->nmesh);
    for (int m = 0; m < p->nmesh; ++m) {
      const BatchItem& it = p->items_h[m];
      int v0, v1;
      if (c < 0) { v0 = 0; v1 = it.mv.nf; }
      else if (c < it.ncol) { v0 = it.coff[c]; v1 = it.coff[c + 1]; }
      else { v0 = v1 = 0; }
      const int cnt = v1 - v0;
      cp[m] = it.prep_dense ? 0 : nblocks(cnt, WG / G);
      cd[m] = it.prep_dense ? nblocks(cnt, p->tv) : 0;
      cf[m] = it.prep_dense ? nblocks(cnt, WG) : 0;
      // dense meshes get their direction from the fused condensation: in a
      // Jacobi sweep, and per colour in a coloured sweep with per-colour Hessians
      const bool fused = it.prep_dense && ((c < 0 && p->cfg.sweep == 0) ||
                                           (c >= 0 && p->cfg.sweep == 1 && p->cfg.hess_refresh == 0));
      cu[m] = fused ? 0 : nblocks(cnt, WG / G);
    }
    offsets_build(p->prep[c + 1], cp, s);
    offsets_build(p->prepd[c + 1], cd, s);
    offsets_build(p->fin[c + 1], cf, s);
    offsets_build(p->upd[c + 1], cu, s);
  }
  p->elemc.assign(p->max_colours, Offsets{});
  p->asmbc.assign(p->max_colours, Offsets{});
  for (int c = 0; c < p->max_colours; ++c) {
    std::vector<int> ce(p->nmesh), cs(p->nmesh);
    for (int m = 0; m < p->nmesh; ++m) {
      const BatchItem& it = p->items_h[m];
      ce[m] = c < it.ncol ? nblocks(it.cel_n[c], EWG) : 0;
      cs[m] = c < it.ncol ? nblocks(it.csl_n[c], EWG) : 0;
    }
    offsets_build(p->elemc[c], ce, s);
    offsets_build(p->asmbc[c], cs, s);
  }
}

BatchPlan* batch_plan_create(const BatchItem* items_host, int nmesh, const BatchConfig& cfg,
                             hipStream_t s) {
  BatchPlan* p = new BatchPlan();
  p->nmesh = nmesh;
  p->cfg = cfg;
  p->items_h.assign(items_host, items_host + nmesh);
  std::vector<int> cpred(nmesh), celem(nmesh), casm(nmesh), cgrad(nmesh), cen(nmesh), cax(nmesh),
      caxj(nmesh), cfeat(nmesh), crot(nmesh);
  {
    // one dense configuration (rows per workgroup, chunk, LDS) for every
    // dense-basis mesh; none fitting sends them to the sparse-row kernel
    std::vector<int> dense_nf, dense_bw;
    for (int m = 0; m < nmesh; ++m)
      if (p->items_h[m].prep_dense) {
        dense_nf.push_back(p->items_h[m].mv.nf);
        dense_bw.push_back(p->items_h[m].mv.band_w);
      }
    if (!dense_nf.empty()) {
      // a coloured sweep launches one colour's rows at a time; there chunks of
      // 256 measured faster than the 128 that tie with them on the full mesh
      DenseCfg dc{};
      if (cfg.sweep == 1 && cfg.chunk == 0)
        dc = dense_config(dense_nf.data(), dense_bw.data(), (int)dense_nf.size(), cfg.D, cfg.prec, cfg.tv_cap, 256);
      if (dc.tv == 0)
        dc = dense_config(dense_nf.data(), dense_bw.data(), (int)dense_nf.size(), cfg.D, cfg.prec, cfg.tv_cap,
                          cfg.chunk);
      p->tv = dc.tv;
      p->ch = dc.ch;
      p->lds = dc.lds;
      if (dc.tv == 0)
        for (int m = 0; m < nmesh; ++m) p->items_h[m].prep_dense = 0;
    }
  }
  int sparse_supp = 0;
  for (int m = 0; m < nmesh; ++m) {
    const MeshView& mv = p->items_h[m].mv;
    cpred[m] = nblocks(mv.n, WG);
    celem[m] = nblocks(mv.m, EWG);
    casm[m] = nblocks(mv.nnzb, EWG);
    cgrad[m] = nblocks(mv.nf, WG / GRAD_G);
    cen[m] = nblocks(mv.m, WG) + nblocks(mv.nf, WG);
    cax[m] = nblocks((long long)mv.D * mv.n, WG);
    // a Jacobi sweep's dense finish writes the trial point itself
    caxj[m] = (cfg.sweep == 0 && p->items_h[m].prep_dense) ? 0 : cax[m];
    cfeat[m] = nblocks(mv.nf, WG / FEAT_LANES);
    crot[m] = (cfg.corotate && mv.rot) ? nblocks(mv.nf, WG) : 0;
    p->max_colours = std::max(p->max_colours, p->items_h[m].ncol);
    if (!p->items_h[m].prep_dense && mv.smap) sparse_supp = std::max(sparse_supp, mv.smap_supp);
  }
  p->scap = sparse_stage_cap(sparse_supp, cfg.G, cfg.D, cfg.prec);
  p->slds = sparse_stage_bytes(p->scap, cfg.G, cfg.D, cfg.prec);

  offsets_build(p->pred, cpred, s);
  offsets_build(p->elem, celem, s);
  offsets_build(p->asmb, casm, s);
  offsets_build(p->grad, cgrad, s);
  offsets_build(p->energy, cen, s);
  {
    std::vector<int> ceg(nmesh);
    for (int m = 0; m < nmesh; ++m) ceg[m] = cen[m] + cgrad[m];
    offsets_build(p->eg, ceg, s);
  }
  if (p->energy.total() > 0 &&
      hipMalloc(&p->wpart, (size_t)LS_WIDTH * p->energy.total() * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    p->wpart = nullptr;
  }
  offsets_build(p->axpy, cax, s);
  offsets_build(p->axpyj, caxj, s);
  offsets_build(p->feat, cfeat, s);
  offsets_build(p->rotn, crot, s);
  plan_vertex_offsets(p, s);
  (void)hipMalloc(&p->items_d, nmesh * sizeof(BatchItem));
  (void)hipMalloc(&p->ctl_d, nmesh * sizeof(BatchCtl));
  (void)hipMemcpyAsync(p->items_d, p->items_h.data(), nmesh * sizeof(BatchItem), hipMemcpyHostToDevice, s);
  (void)hipStreamSynchronize(s);
  return p;
}

void batch_plan_destroy(BatchPlan* p) {
  if (!p) return;
  drop_graph(p);
  for (Offsets* o : {&p->pred, &p->elem, &p->asmb, &p->grad, &p->energy, &p->eg, &p->axpy, &p->axpyj, &p->feat,
                     &p->rotn})
    offsets_free(*o);
  for (auto& o : p->prep) offsets_free(o);
  for (auto& o : p->prepd) offsets_free(o);
  for (auto& o : p->fin) offsets_free(o);
  for (auto& o : p->upd) offsets_free(o);
  for (auto& o : p->elemc) offsets_free(o);
  for (auto& o : p->asmbc) offsets_free(o);
  if (p->wpart) (void)hipFree(p->wpart);
  if (p->items_d) (void)hipFree(p->items_d);
  if (p->ctl_d) (void)hipFree(p->ctl_d);
  delete p;
}

BatchItem* batch_items_dev(BatchPlan* p) { return p->items_d; }
BatchCtl* batch_ctl_dev(BatchPlan* p) { return p->ctl_d; }

static inline int gridn(const Offsets& o) { return o.total(); }

template <int D>
static void b_gradient(BatchPlan* p, int which, hipStream_t s, int post = 0, int only_warm = 0) {
  if (gridn(p->grad) == 0) return;
  p->mark(2, 1);
  CC_DISPATCH_MAT(p->cfg.any_fcr, kb_gradient<D, GRAD_G, FCR><<<gridn(p->grad), WG, 0, s>>>(
                                      p->items_d, p->ctl_d, p->grad.d, p->nmesh, which, only_warm));
  p->mark(2, 0);
  kb_reduce<<<p->nmesh, WG, 0, s>>>(p->items_d, p->ctl_d, p->grad.d, 1, post, p->cfg.tol,
                                    p->cfg.max_iters, only_warm);
}

template <int D>
static void b_energy(BatchPlan* p, int which, int dst, hipStream_t s, int post = 0) {
  if (gridn(p->energy) == 0) return;
  p->mark(5, 1);
  CC_DISPATCH_MAT(p->cfg.any_fcr, kb_energy<D, FCR><<<gridn(p->energy), WG, 0, s>>>(
                                      p->items_d, p->ctl_d, p->energy.d, p->nmesh, which));
  p->mark(5, 0);
  kb_reduce<<<p->nmesh, WG, 0, s>>>(p->items_d, p->ctl_d, p->energy.d, dst, post, p->cfg.tol,
                                    p->cfg.max_iters, 0);
}

template <typename T, int D, int G>
static void b_prep(BatchPlan* p, int colour, hipStream_t s, int fuse = 0) {
  const Offsets& o = p->prep[colour + 1];
  const Offsets& od = p->prepd[colour + 1];
  if (gridn(o) == 0 && gridn(od) == 0) return;
  p->mark(3, 1);
  if (gridn(o) > 0)
    kb_prep<T, D, G><<<gridn(o), WG, p->slds, s>>>(p->items_d, p->ctl_d, o.d, p->nmesh, p->cfg.method,
                                                  colour, p->scap);
  if (gridn(od) > 0) {
    const Offsets& of = p->fin[colour + 1];
    CC_DISPATCH_TVCH(p->tv, p->ch, kb_prep_band<T, D, TV, CH><<<gridn(od), CH, p->lds, s>>>(
                              p->items_d, p->ctl_d, od.d, p->nmesh, p->cfg.method, colour, fuse));
    kb_dm_finish<T, D><<<gridn(of), WG, 0, s>>>(p->items_d, p->ctl_d, of.d, p->nmesh, p->cfg.method,
                                               colour, fuse);
  }
  p->mark(3, 0);
}

template <typename T, int D, int G>
static void b_update(BatchPlan* p, int colour, int into_trial, hipStream_t s) {
  const Offsets& o = p->upd[colour + 1];
  if (gridn(o) == 0) return;
  p->mark(4, 1);
  kb_update<T, D, G><<<gridn(o), WG, 0, s>>>(p->items_d, p->ctl_d, o.d, p->nmesh, p->cfg.method, colour,
                                             into_trial);
  p->mark(4, 0);
}

// Element Hessians and block rows at positions `which`: of every element
// (colour < 0), or only those that colour's moves changed.
template <typename T, int D>
static void b_hessian(BatchPlan* p, int which, hipStream_t s, int colour = -1) {
  if (gridn(p->rotn) > 0)   // corotation: rotations at the positions of the Hessian
    kb_rotations<D><<<gridn(p->rotn), WG, 0, s>>>(p->items_d, p->ctl_d, p->rotn.d, p->nmesh, which);
  const Offsets& oe = colour < 0 ? p->elem : p->elemc[colour];
  const Offsets& oa = colour < 0 ? p->asmb : p->asmbc[colour];
  if (gridn(oe) > 0) {
    p->mark(0, 1);
    CC_DISPATCH_MAT(p->cfg.any_fcr, kb_elem_hess<T, D, FCR><<<gridn(oe), elem_threads<T>(), 0, s>>>(
                                        p->items_d, p->ctl_d, oe.d, p->nmesh, which, colour));
    p->mark(0, 0);
  }
  if (gridn(oa) > 0) {
    p->mark(1, 1);
    kb_assemble<T, D><<<gridn(oa), EWG, 0, s>>>(p->items_d, p->ctl_d, oa.d, p->nmesh, colour);
    // the band records of blocks the partial assembly left alone still
    // carry the previous rotations
    if (colour >= 0 && gridn(p->rotn) > 0 && p->tv > 0)
      kb_band_copy<T, D><<<gridn(p->asmb), EWG, 0, s>>>(p->items_d, p->ctl_d, p->asmb.d, p->nmesh);
    p->mark(1, 0);
  }
}

template <typename T, int D, int G>
static void b_iteration(BatchPlan* p, hipStream_t s) {
  const BatchConfig& c = p->cfg;
  const int nm = p->nmesh, gb = nblocks(nm, WG);
  if (c.sweep == 0) {
    // g holds the gradient at x (from batch_begin or the end of the previous
    // iteration), so the dense condensation forms the direction itself
    b_hessian<T, D>(p, 0, s);
    b_prep<T, D, G>(p, -1, s, 1);
    b_update<T, D, G>(p, -1, 0, s);
    if (gridn(p->axpyj) > 0)
      kb_axpy<<<gridn(p->axpyj), WG, 0, s>>>(p->items_d, p->ctl_d, p->axpyj.d, nm, 1.0, 0);
  } else {
    if (gridn(p->axpy) > 0)
      kb_axpy<<<gridn(p->axpy), WG, 0, s>>>(p->items_d, p->ctl_d, p->axpy.d, nm, 0.0, 1);
    for (int col = 0; col < p->max_colours; ++col) {
      // per-colour Hessians: all of them at the sweep's start, then only the
      // elements and block slots the previous colour's moves changed
      if (c.hess_refresh == 0) b_hessian<T, D>(p, 1, s, col == 0 ? -1 : col - 1);
      else if (col == 0) {
        b_hessian<T, D>(p, 1, s);
        b_prep<T, D, G>(p, -1, s);
      }
      if (gridn(p->grad) > 0) {
        p->mark(2, 1);
        CC_DISPATCH_MAT(c.any_fcr, kb_gradient<D, GRAD_G, FCR><<<gridn(p->grad), WG, 0, s>>>(
                                       p->items_d, p->ctl_d, p->grad.d, nm, 1, 0));
        p->mark(2, 0);
      }
      // dense meshes form b_i from the fresh gradient and move the colour's
      // vertices in the finish kernel; sparse ones take the update kernel
      if (c.hess_refresh == 0) b_prep<T, D, G>(p, col, s, 2);
      b_update<T, D, G>(p, col, 1, s);
    }
  }
  if (c.line_search) {
    // E and the gradient at the trial point, then the accept rule and the
    // convergence test
    if (gridn(p->eg) > 0) {
      p->mark(5, 1);
      CC_DISPATCH_MAT(c.any_fcr, kb_energy_grad<D, FCR><<<gridn(p->eg), WG, 0, s>>>(
                                     p->items_d, p->ctl_d, p->eg.d, nm));
      p->mark(5, 0);
      kb_reduce_eg<<<nm, WG, 0, s>>>(p->items_d, p->ctl_d, c.tol, c.max_iters);
    }
  } else {
    kb_accept<<<gb, WG, 0, s>>>(p->items_d, p->ctl_d, nm, 0);
    b_gradient<D>(p, 0, s, 2);    // gradient at the accepted point, then the convergence test
  }
}


static void one_iteration(BatchPlan* p, hipStream_t s) {
#define ITER(T, D, G) b_iteration<T, D, G>(p, s)
  const BatchConfig& c = p->cfg;
  if (c.prec == 0) {
    if (c.D == 2) { if (c.G == 64) ITER(double, 2, 64); else if (c.G == 32) ITER(double, 2, 32); else ITER(double, 2, 16); }
    else { if (c.G == 64) ITER(double, 3, 64); else if (c.G == 32) ITER(double, 3, 32); else ITER(double, 3, 16); }
  } else {
    if (c.D == 2) { if (c.G == 64) ITER(float, 2, 64); else if (c.G == 32) ITER(float, 2, 32); else ITER(float, 2, 16); }
    else { if (c.G == 64) ITER(float, 3, 64); else if (c.G == 32) ITER(float, 3, 32); else ITER(float, 3, 16); }
  }
#undef ITER
}

void batch_begin(BatchPlan* p, hipStream_t s) {
  const int nm = p->nmesh, gb = nblocks(nm, WG);
  kb_reset<<<gb, WG, 0, s>>>(p->items_d, p->ctl_d, nm);
  const int D = p->cfg.D;
  if (D == 2) kb_predict<2><<<gridn(p->pred), WG, 0, s>>>(p->items_d, p->ctl_d, p->pred.d, nm, p->cfg.h, p->cfg.quasistatic);
  else kb_predict<3><<<gridn(p->pred), WG, 0, s>>>(p->items_d, p->ctl_d, p->pred.d, nm, p->cfg.h, p->cfg.quasistatic);
  if (D == 2) b_gradient<2>(p, 0, s); else b_gradient<3>(p, 0, s);
  kb_init<<<gb, WG, 0, s>>>(p->items_d, p->ctl_d, nm, p->cfg.tol, p->cfg.max_iters);
  if (p->cfg.line_search) {
    if (D == 2) b_energy<2>(p, 0, 2, s); else b_energy<3>(p, 0, 2, s);
  }
}

hipError_t batch_iterate(BatchPlan* p, int iters, hipStream_t s) {
  const int k = p->cfg.iters_per_graph;
  // with a timing hook the launches run uncaptured: event pairs recorded as
  // graph nodes do not give per-launch durations
  if (k <= 0 || p->hook) {
    for (int i = 0; i < iters; ++i) one_iteration(p, s);
    return hipGetLastError();
  }
  if (!p->exec) {
    bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      p->capturing = 1;
      for (int i = 0; i < k; ++i) one_iteration(p, s);
      p->capturing = 0;
      ok = hipStreamEndCapture(s, &p->graph) == hipSuccess;
    }
    if (ok) ok = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {  // capture unsupported on this stream: run the launches directly (reported)
      (void)hipGetLastError();
      if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
      p->exec = nullptr;
      p->cfg.iters_per_graph = 0;
      p->capture_failed = 1;
      for (int i = 0; i < iters; ++i) one_iteration(p, s);
      return hipGetLastError();
    }
  }
  for (int done = 0; done < iters; done += k) {
    const hipError_t e = hipGraphLaunch(p->exec, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int batch_capture_failed(BatchPlan* p) { return p->capture_failed; }

// Pieces of the batched path used by the warm start (cc_mlp.hip).
void batch_energy_trial(BatchPlan* p, hipStream_t s, int post) {
  if (p->cfg.D == 3) b_energy<3>(p, 1, 0, s, post); else b_energy<2>(p, 1, 0, s, post);
}
void batch_gradient_x(BatchPlan* p, hipStream_t s, int only_warm, int post) {
  if (p->cfg.D == 3) b_gradient<3>(p, 0, s, post, only_warm);
  else b_gradient<2>(p, 0, s, post, only_warm);
}
void batch_elem_hess_x(BatchPlan* p, hipStream_t s) {
  const Offsets& oe = p->elem;
  if (gridn(oe) == 0) return;
  if (p->cfg.prec == 0)
    CC_DISPATCH_MAT(p->cfg.any_fcr, kb_elem_hess<double, 3, FCR><<<gridn(oe), elem_threads<double>(), 0, s>>>(
                                        p->items_d, p->ctl_d, oe.d, p->nmesh, 0, -1));
  else
    CC_DISPATCH_MAT(p->cfg.any_fcr, kb_elem_hess<float, 3, FCR><<<gridn(oe), elem_threads<float>(), 0, s>>>(
                                        p->items_d, p->ctl_d, oe.d, p->nmesh, 0, -1));
}
void batch_energy_x(BatchPlan* p, hipStream_t s) {
  if (p->cfg.D == 3) b_energy<3>(p, 0, 2, s); else b_energy<2>(p, 0, 2, s);
}
bool batch_ls_round(BatchPlan* p, int first, int max_halvings, hipStream_t s) {
  const int total = gridn(p->energy);
  if (gridn(p->axpy) == 0 || total == 0) return true;
  if (!p->wpart) return false;
  if (first) kb_ls_vec<<<gridn(p->axpy), WG, 0, s>>>(p->items_d, p->ctl_d, p->axpy.d, p->nmesh, 0);
  const dim3 grid(total, LS_WIDTH);
  p->mark(5, 1);
  if (p->cfg.D == 3)
    CC_DISPATCH_MAT(p->cfg.any_fcr, kb_energy_wide<3, FCR><<<grid, WG, 0, s>>>(
                                        p->items_d, p->ctl_d, p->energy.d, p->nmesh, total,
                                        max_halvings, p->wpart));
  else
    CC_DISPATCH_MAT(p->cfg.any_fcr, kb_energy_wide<2, FCR><<<grid, WG, 0, s>>>(
                                        p->items_d, p->ctl_d, p->energy.d, p->nmesh, total,
                                        max_halvings, p->wpart));
  p->mark(5, 0);
  kb_ls_reduce_wide<<<p->nmesh, WG, 0, s>>>(p->ctl_d, p->energy.d, total, LS_WIDTH, max_halvings,
                                            p->wpart);
  kb_ls_vec<<<gridn(p->axpy), WG, 0, s>>>(p->items_d, p->ctl_d, p->axpy.d, p->nmesh, 1);
  kb_ls_commit<<<(p->nmesh + WG - 1) / WG, WG, 0, s>>>(p->items_d, p->ctl_d, p->nmesh);
  return true;
}

void batch_gradient_converge(BatchPlan* p, hipStream_t s) {
  if (p->cfg.D == 3) b_gradient<3>(p, 0, s, 2); else b_gradient<2>(p, 0, s, 2);
}

BatchGrid batch_grid(BatchPlan* p) {
  BatchGrid g;
  g.nmesh = p->nmesh;
  g.pred_blocks = gridn(p->pred);
  g.pred_off = p->pred.d;
  g.feat_blocks = gridn(p->feat);
  g.feat_off = p->feat.d;
  g.tol = p->cfg.tol;
  g.max_iters = p->cfg.max_iters;
  g.any_fcr = p->cfg.any_fcr;
  g.line_search = p->cfg.line_search;
  g.prec = p->cfg.prec;
  return g;
}

void batch_finish(BatchPlan* p, hipStream_t s) {
  if (gridn(p->pred) == 0) return;
  if (p->cfg.D == 2) kb_finalize<2><<<gridn(p->pred), WG, 0, s>>>(p->items_d, p->pred.d, p->nmesh, p->cfg.h, p->cfg.quasistatic);
  else kb_finalize<3><<<gridn(p->pred), WG, 0, s>>>(p->items_d, p->pred.d, p->nmesh, p->cfg.h, p->cfg.quasistatic);
}

void batch_set_lanes(BatchPlan* p, int G) {
  if (G == p->cfg.G) return;
  p->cfg.G = G;
  drop_graph(p);
  for (auto& o : p->prep) offsets_free(o);
  for (auto& o : p->prepd) offsets_free(o);
  for (auto& o : p->fin) offsets_free(o);
  for (auto& o : p->upd) offsets_free(o);
  for (auto& o : p->elemc) offsets_free(o);
  for (auto& o : p->asmbc) offsets_free(o);
  plan_vertex_offsets(p, nullptr);
  (void)hipDeviceSynchronize();
}

// Times condensation + update (Jacobi form, writing d only) for lane count G.
float batch_time_prep_update(BatchPlan* p, int G, int reps, hipStream_t s) {
  batch_set_lanes(p, G);
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
#define PU(T, D, GG) do { b_prep<T, D, GG>(p, -1, s, p->cfg.sweep == 0); b_update<T, D, GG>(p, -1, 0, s); } while (0)
  auto run = [&]() {
    const BatchConfig& c = p->cfg;
    if (c.prec == 0) {
      if (c.D == 2) { if (G == 64) PU(double, 2, 64); else if (G == 32) PU(double, 2, 32); else PU(double, 2, 16); }
      else { if (G == 64) PU(double, 3, 64); else if (G == 32) PU(double, 3, 32); else PU(double, 3, 16); }
    } else {
      if (c.D == 2) { if (G == 64) PU(float, 2, 64); else if (G == 32) PU(float, 2, 32); else PU(float, 2, 16); }
      else { if (G == 64) PU(float, 3, 64); else if (G == 32) PU(float, 3, 32); else PU(float, 3, 16); }
    }
  };
#undef PU
  run();
  (void)hipEventRecord(a, s);
  for (int r = 0; r < reps; ++r) run();
  (void)hipEventRecord(b, s);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

}  // namespace cc
