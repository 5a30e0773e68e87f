// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cc {

// Device view of one mesh in the internal (colour-sorted) order.
// Vertices 0..nf-1 are free and sorted by colour; nf..n-1 are Dirichlet.
struct MeshView {
  int D;            // 2 or 3
  int n, nf, m;     // vertices, free vertices, elements
  const int* ev;    // [(D+1)][m] internal vertex ids
  const double* dinv_d;  // [D*D][m], row a-1 of Dm^{-1} = beta_a for a = 1..D
  const float* dinv_f;
  const double* vol_d;   // [m] rest volumes
  const float* vol_f;
  const double* mass;    // [n] lumped masses
  const int* vperm;      // [n] caller id of internal vertex
  const int* star_ptr;   // [nf+1]  incidence of free vertices
  const int* star;       // packed e*4 + local index
  const int* rowptr;     // [nf+1]  block rows over free vertices, diagonal first
  const int* colidx;     // [nnzb]
  const int* blkrow;     // [nnzb]  row of each block slot
  const int* cptr;       // [nnzb+1] element contributions of each block slot
  const int* centry;     // packed e*16 + a*4 + b
  int nnzb;
  // Band order of the free vertices (breadth-first levels from the free
  // vertices next to the Dirichlet set, neighbours appended in caller-id
  // order): bvert[p] = internal id at band position p, bpos = its inverse.
  // Every neighbour k of a vertex j lies within band_w positions after it
  // (when k comes later).  Row p's blocks (j, k) with bpos[k] >= bpos[j]
  // ("upper" blocks, the diagonal first) number bq_cnt[p] <= qmax.  When hq
  // is set (dense bases), hq[q * nf + p] is the BandRec (precision of hb) of
  // the q-th of them, written by the assembly and band-copy kernels:
  // hq_slot[t] = q * nf + p for an upper slot t of hb, -1 otherwise.
  const int* bvert;
  const int* bpos;
  const int* bq_cnt;
  const int* hq_slot;
  void* hq;
  int qmax, band_w;
  // perturbation basis, internal ids.  Sparse bases: CSR rows sorted by
  // internal id (sptr, sidx).  Dense (exact) bases: row i holds nf blocks
  // at (i * nf + p) * D*D, column p = band position, the block at the
  // vertex's own position zero; sptr and sidx are unused.
  const int64_t* sptr;   // [nf+1]
  const int* sidx;
  const double* U_d;     // [nnz][D*D]; dense bases: null when only float32 is kept
  const float* U_f;
  int dense_supp;        // 1: supp(i) = every free vertex except i (band layout)
  // support slot map of sparse bases: support entry q = (i, j) owns the
  // smap_words + 1 words at q * (smap_words + 1): the first holds
  // rowptr[j]; for the t-th block of row j, byte t of the others is SMAP_SELF
  // for column k = i, the position of k in supp(i) for k >= j, and SMAP_SKIP
  // otherwise (k < j, k outside the support, padding past the row); null when
  // the basis is dense or a support or row is too long for the byte codes
  const uint32_t* smap;
  int smap_words;
  int smap_supp;         // longest support row of the slot-mapped basis
  // corotation: per free vertex rotation R_j (row-major D*D), or null = off
  const double* rot;
  // the last finished step's correction x - x~ (free vertices, component-major
  // like x; zero on Dirichlet vertices and before the first step): the base
  // the learned warm start adds its prediction to
  double* corr;
  // free internal ids in caller order (spatially coherent on the structured
  // grids): the order in which a whole-mesh Jacobi condensation visits them
  const int* sorder;
  // block-row slots row by row in that order: the order assembly visits them
  const int* aorder;
  // coloured sweeps: the elements with a free vertex of colour c,
  // cel[cel_ptr[c] .. cel_ptr[c+1]), and the block slots those elements
  // contribute to, csl[csl_ptr[c] .. csl_ptr[c+1]) (in the assembly order);
  // after colour c moves, only these need re-evaluating
  const int* cel_ptr;
  const int* cel;
  const int* csl_ptr;
  const int* csl;
};

constexpr int SMAP_SELF = 254;
constexpr int SMAP_SKIP = 255;
constexpr int SMAP_MAX_WORDS = 16;   // rows of up to 64 blocks

// Material models (values of Material::model and of the C-ABI constants).
constexpr int MAT_SNH = 0;   // stable neo-Hookean, lam = lambda_L + mu
constexpr int MAT_FCR = 1;   // Fixed Corotational, lam = lambda_L

struct Material {
  double mu, lam;        // mu and the model's lambda (see MAT_*)
  double w_in;           // weight of the inertia term (1 dynamic, 0 quasistatic)
  double s_el;           // weight of the elastic and gravity terms (h^2 or 1)
  double grav[3];
  int model;             // MAT_SNH or MAT_FCR
};

// ---- launch wrappers (cc_kernels.hip) --------------------------------------
void launch_predict(const MeshView& mv, const int* vperm, const double* x_user,
                    const double* v_user, const double* x_bc, double h, int quasi,
                    double* x, double* xt, double* x0, int* bad, hipStream_t s);
void launch_finalize(const MeshView& mv, const int* vperm, const double* x, const double* xt, const double* x0,
                     double h, int quasi, double* x_user, double* v_user, hipStream_t s);
void launch_elem_hess(const MeshView& mv, int prec, const double* x, const Material& mat,
                      double scale, void* estore, hipStream_t s);
void launch_assemble(const MeshView& mv, int prec, const void* estore, const Material& mat,
                     void* hb, hipStream_t s);
// The same over a list of `count` elements / block slots (device ints; null:
// the first `count` of all), e.g. the ones a colour's moves change
// (MeshView::cel, csl).
void launch_elem_hess_list(const MeshView& mv, int prec, const double* x, const Material& mat,
                           double scale, void* estore, hipStream_t s, const int* elist, int count);
void launch_assemble_list(const MeshView& mv, int prec, const void* estore, const Material& mat, void* hb,
                          hipStream_t s, const int* slist, int count);
// Rewrites every BandRec of a dense-basis mesh (hq set) from the block rows
// hb and the current rotations: after a partial assembly whose rotations
// changed everywhere (a coloured sweep of a corotated mesh).
void launch_band_copy(const MeshView& mv, int prec, const void* hb, hipStream_t s);
void launch_gradient(const MeshView& mv, const double* x, const double* xt, const Material& mat,
                     double* g, double* partials, int* nparts, hipStream_t s);
// Condensation of vertices [v0, v1).  With g and dout given (g the gradient
// at the same x) the dense path also writes the directions into dout, and
// with xmove given (a coloured sweep) adds them to xmove in place; the
// return value says whether it did (else launch_cc_update).
bool launch_cc_prep(const MeshView& mv, int prec, int method, int v0, int v1, const void* hb,
                    void* KL, unsigned long long* fallbacks, hipStream_t s,
                    const double* g = nullptr, double* dout = nullptr, double* xmove = nullptr,
                    int tv_cap = 0, int chunk = 0);
void launch_cc_update(const MeshView& mv, int prec, int method, int v0, int v1, const void* KL,
                      const double* g, double* x_or_d, int accumulate, hipStream_t s);
void launch_energy(const MeshView& mv, const double* x, const double* xt, const Material& mat,
                   double* partials, int* nparts, hipStream_t s);
void launch_reduce(const double* partials, int n, double* out, hipStream_t s);
// Corotation: R_j = polar rotation of sum_{k in N(j)} (x_k - x_j)(X_k - X_j)^T for
// every free vertex j (nptr/nidx: mesh neighbours, Xr: rest positions, SoA).
void launch_rotations(const MeshView& mv, const double* x, const int* nptr, const int* nidx,
                      const double* Xr, double* rot, hipStream_t s);
void launch_axpy(int count, const double* x, const double* d, double alpha, double* out,
                 hipStream_t s);
void launch_probe_element(const MeshView& mv, int prec, const double* x_user,
                          const int* vperm_inv, const int* eperm, double* xi_tmp,
                          const Material& mat, double* ge, double* He, hipStream_t s);
void launch_gather_user(const MeshView& mv, const int* vperm_inv, const double* src_user,
                        double* dst_int, hipStream_t s);
void launch_scatter_user(const MeshView& mv, const int* vperm, const double* src_int,
                         double* dst_user, int free_only, hipStream_t s);

int reduce_partials_capacity(const MeshView& mv);

// Dense condensation: the largest chunk of band positions per pass (= its
// workgroup size) and the per-workgroup LDS limit of the device (bytes, set
// once per process).
constexpr int BWG = 512;
void set_lds_limit(size_t bytes);
// One upper block (j, k) of H in band order, as the dense condensation reads
// it: h = w R_j^T H_jk R_k (w = 1/2 on the diagonal block; R = I without
// corotation, else the vertex rotations at the Hessian's positions), pos =
// the band position of k.  Rotating H instead of the basis blocks keeps the
// condensation free of per-row rotations:
//   (R_j U_j)^T H_jk (R_k U_k) = U_j^T (R_j^T H_jk R_k) U_k.
template <typename T, int D>
struct alignas(16) BandRec {
  T h[D * D];
  int pos;
};

// Access unit (bytes) and 32-bit words of one slot of the dense
// condensation's LDS ring: tv blocks of D*D values of tsize bytes, read and
// written in 16-byte units (padded when that costs at most an eighth more),
// else in the widest unit (8 or 4 bytes) that divides them, the slot padded
// to an odd number of units, so that consecutive slots read one unit each
// from distinct banks.
__host__ __device__ constexpr int ring_slot_unit(int tv, int D, int tsize) {
  return (tv * D * D * tsize) % 16 == 0 || (16 - (tv * D * D * tsize) % 16) * 8 <= tv * D * D * tsize ? 16
         : (tv * D * D * tsize) % 8 == 0                                                              ? 8
                                                                                                        : 4;
}
__host__ __device__ constexpr int ring_slot_words(int tv, int D, int tsize) {
  const int unit = ring_slot_unit(tv, D, tsize);
  int u = (tv * D * D * tsize + unit - 1) / unit;
  if (u % 2 == 0) ++u;
  return u * unit / 4;
}

// LDS ring length of a mesh for chunks of ch positions (min(nf, ch +
// band_w): every position a chunk's rows read), and the dynamic LDS of a
// workgroup of tv rows.
int band_ring(int nf, int band_w, int ch);
size_t dense_lds_bytes(int tv, int ring, int D, int prec, int ch);
// Rows per workgroup (tv) and chunk (ch, the workgroup size) of the dense
// condensation for meshes with the given free-vertex counts and band widths:
// the most rows (4, 3, 2 or 1; at most 2 in float64) whose ring fits, at
// most cap when cap > 0 (with cap = 0, first the most rows whose ring lets
// two workgroups share a CU), then the chunk (128, 256 or 512) with more
// resident waves per CU (LDS and an estimate of the registers), ties to the
// smaller chunk, whose workgroups overlap one another's ring fill and final
// sums (chunk > 0 forces that chunk).  tv = 0: no configuration fits.
struct DenseCfg {
  int tv = 0, ch = 0;
  size_t lds = 0;
};
DenseCfg dense_config(const int* nf, const int* band_w, int count, int D, int prec, int cap = 0,
                      int chunk = 0);

// Exact basis U_i[j] = (H^{-1})_ji ((H^{-1})_ii)^{-1} from float64 block rows
// hb (cc_basis.hip), through the block-tridiagonal structure of H in band
// order: loff (host, L+1 band positions) splits the band order into levels
// such that every block (j, k) of H couples the same or adjacent levels.
// Ud (may be null) / Uf receive the dense band layout.  Returns 0, 1 when a
// pivot block is not positive definite, 2 when device memory runs out.
int exact_basis_band(const MeshView& mv, const double* hb, const int* loff_h, int L, double* Ud,
                     float* Uf, hipStream_t s);

// ---- batched stepping (many meshes per launch) -----------------------------
constexpr int MAX_COLOURS = 32;

// One mesh of a batch, resident in device memory.  The x / xtrial pointers
// are swapped in place by the control kernel when an iteration is accepted,
// so every launch reads them from here.
struct BatchItem {
  MeshView mv;
  Material mat;
  double *x, *xtrial, *xt, *x0, *d, *g;
  void *estore, *hb, *KL;
  double* partials;
  unsigned long long* fb;
  double* xu;          // caller positions (n x D), this call
  double* vu;          // caller velocities
  const double* xbc;   // caller Dirichlet targets or null
  int prep_dense;      // 1: exact-basis condensation streamed through the LDS ring
  double load;         // floor of the convergence test's denominator (the gravity
                       // load's norm, or 1e-8 of the elastic force scale)
  int ncol;
  int coff[MAX_COLOURS + 1];
  // warm start: mesh neighbours (all vertices), rest positions, scales and
  // this mesh's first row in the batch-wide feature / output buffers
  const int* nptr;
  const int* nidx;
  const double* Xr;
  double ell, youngs;
  int feat_off;
  // coloured sweeps: sizes of the per-colour dirty element / slot lists
  int cel_n[MAX_COLOURS];
  int csl_n[MAX_COLOURS];
};

// Per-mesh iteration state, device-resident.
struct BatchCtl {
  int active;          // 1 while the mesh iterates
  int iters;
  int status;          // CC_OK / CC_NOT_CONVERGED / CC_STALLED, -100 while running
  int needs_host;      // 1: energy rose at alpha = 1, backtracking left to the host
  int bad;             // non-finite input seen by the predictor
  int warm;            // 1: the learned proposal was accepted
  double E_cur, E_trial, g0, gn2, r;
  // backtracking rounds (batch_ls_round): current step fraction, halvings
  // taken, outcome (0 searching, 1 accepted, 2 halvings exhausted)
  double alpha;
  int halvings, ls;
};

struct BatchPlan;  // host-side, defined in cc_kernels.hip

struct BatchConfig {
  int D, prec, method, sweep, hess_refresh, line_search, max_iters, quasistatic;
  double tol, h;
  int G;               // lanes per vertex of the generic condensation/update kernels
  int iters_per_graph; // iterations captured per graph replay (0: no graph)
  int dense_lds;       // max dynamic LDS of the dense condensation path (bytes)
  int corotate;        // rotations re-estimated wherever the Hessian is
  int tv_cap;          // rows per workgroup of the dense condensation (0: most that fit)
  int chunk;           // its chunk of band positions (0: automatic, else 128, 256 or 512)
  int any_fcr;         // some mesh of the batch uses the Fixed Corotational model
};

BatchPlan* batch_plan_create(const BatchItem* items_host, int nmesh, const BatchConfig& cfg,
                             hipStream_t s);
void batch_plan_destroy(BatchPlan* p);
BatchItem* batch_items_dev(BatchPlan* p);
BatchCtl* batch_ctl_dev(BatchPlan* p);
// Start of a step: predictor, initial gradient norm and energy, control reset.
void batch_begin(BatchPlan* p, hipStream_t s);
// Run `iters` iterations (graph replay when captured); returns the first
// launch error.  When the capture itself fails the launches run uncaptured
// from then on and batch_capture_failed reports it.
hipError_t batch_iterate(BatchPlan* p, int iters, hipStream_t s);
int batch_capture_failed(BatchPlan* p);
// Velocities and caller positions.
void batch_finish(BatchPlan* p, hipStream_t s);
// Learned warm start after batch_begin: feat / delta hold sum(nf) rows.
struct MlpState;
constexpr int FEAT_LANES = 32;   // lanes per vertex of the feature kernels
struct BatchGrid {
  int nmesh, pred_blocks, feat_blocks;
  const int* pred_off;  // block offsets of the per-vertex launches
  const int* feat_off;  // block offsets of the feature launch
  double tol;
  int max_iters;
  int any_fcr;          // some mesh uses the Fixed Corotational model
  int line_search;      // E at the predictor is already in ctl.E_cur
  int prec;             // 0 float64, 1 float32 local arithmetic
};
BatchGrid batch_grid(BatchPlan* p);
// ctl.E_trial = E(xtrial); post 3: then the warm start's accept rule
void batch_energy_trial(BatchPlan* p, hipStream_t s, int post = 0);
void batch_energy_x(BatchPlan* p, hipStream_t s);       // ctl.E_cur = E(x)
// element Hessians of every active mesh at x into its element store
void batch_elem_hess_x(BatchPlan* p, hipStream_t s);
// g(x), ctl.gn2; only_warm: only meshes whose learned proposal was accepted
// gradient at x; post 4 (with only_warm): then the residual test of an
// accepted proposal
void batch_gradient_x(BatchPlan* p, hipStream_t s, int only_warm = 0, int post = 0);
// One backtracking round for the active meshes, whose energy rose at the
// full step (d = x_trial - x formed first when `first`): the energies at the
// next halvings of alpha, then per mesh the first that does not raise E is
// taken (x_trial = x + alpha d written, swapped in, E_cur and the iteration
// count updated), or the search stops at max_halvings (ctl.ls), or goes on
// in the next round.  False when the plan has no buffer for the energies.
bool batch_ls_round(BatchPlan* p, int first, int max_halvings, hipStream_t s);
// Gradient at x and the convergence test for the active meshes.
void batch_gradient_converge(BatchPlan* p, hipStream_t s);
void batch_warm_start(BatchPlan* p, const MlpState& net, float* feat, float* delta, int rows,
                      hipStream_t s);
// Time one condensation + update pass of every mesh with the given lane count.
float batch_time_prep_update(BatchPlan* p, int G, int reps, hipStream_t s);
void batch_set_lanes(BatchPlan* p, int G);
// Kernel timing: hook(user, kid, begin) is called around the launches of the
// element, assembly, gradient, condensation, update and energy kernels (ids as
// CC_K_* in ccgpu.h) while they are enqueued or captured.  Changing the hook
// drops a captured graph.
typedef void (*BatchHook)(void* user, int kid, int begin);
void batch_set_hook(BatchPlan* p, BatchHook hook, void* user);
// 1 while a graph is being captured (hooks may record events into it).
int batch_capturing(BatchPlan* p);
int batch_has_graph(BatchPlan* p);

}  // namespace cc
