// Host side of libccgpu: context, mesh and basis uploads, colouring and
// layouts, the library's basis builder and the implicit-step driver.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ccgpu.h"
#include "cc_kernels.h"
#include "cc_mlp.h"

using cc::Material;
using cc::MeshView;

namespace {

struct Mesh {
  int D = 0, K = 0, n = 0, nf = 0, m = 0, ncol = 0;
  double E = 0, nu = 0, rho = 0, mu = 0, lam = 0, volume = 0;
  int model = cc::MAT_SNH;         // material model; lam is that model's lambda
  std::vector<double> X;           // caller order, n x D
  std::vector<int> elems;          // caller order, m x K
  std::vector<uint8_t> fixed;
  std::vector<int> colour;         // caller order
  std::vector<int> vperm, vinv, eperm, coff;
  std::vector<int> rowptr, colidx; // host copy of the block-row pattern (internal ids)
  std::vector<double> mass_int;    // internal order
  double mass_free_norm = 0;       // |m| over free vertices (the gravity load's scale)
  int nnzb = 0;
  // device: static mesh data
  int *ev = nullptr, *star_ptr = nullptr, *star = nullptr, *d_rowptr = nullptr, *d_colidx = nullptr,
      *blkrow = nullptr, *cptr = nullptr, *centry = nullptr, *d_vperm = nullptr, *d_vinv = nullptr,
      *d_eperm = nullptr, *d_sorder = nullptr, *d_aorder = nullptr, *d_cel_ptr = nullptr, *d_cel = nullptr,
      *d_csl_ptr = nullptr, *d_csl = nullptr;
  // band order of the free vertices and the upper-block structure of the
  // dense condensation (MeshView::bvert ...); lev_off: breadth-first levels
  // in band positions (every block couples the same or adjacent levels)
  std::vector<int> bvert_h, bpos_h, lev_off;
  std::vector<int> cel_ptr_h, csl_ptr_h;   // per-colour dirty element / slot list offsets
  int *d_bvert = nullptr, *d_bpos = nullptr, *d_bqcnt = nullptr, *d_hqslot = nullptr;
  void* hq = nullptr;
  int qmax = 0, band_w = 0;

  double *dinv_d = nullptr, *vol_d = nullptr, *mass = nullptr;
  float *dinv_f = nullptr, *vol_f = nullptr;
  // basis
  bool has_basis = false;
  int dense = 0;
  int64_t snnz = 0;
  int64_t* sptr = nullptr;
  int* sidx = nullptr;
  double* U_d = nullptr;
  float* U_f = nullptr;
  uint32_t* smap = nullptr;  // support slot map (sparse bases)
  int smap_words = 0, smap_supp = 0;
  // work buffers
  double *x = nullptr, *xt = nullptr, *x0 = nullptr, *xtrial = nullptr, *dvec = nullptr,
         *g = nullptr, *partials = nullptr, *scal = nullptr;
  double* rot = nullptr;  // corotation: rotation of every free vertex (D*D each)
  double* corr = nullptr; // last step's correction x - x~ (MeshView::corr)
  void *estore = nullptr, *hb = nullptr, *KL = nullptr;
  unsigned long long* fb = nullptr;
  int* bad = nullptr;
  // last-step info
  double last_E = 0, last_paper = 0;
  long long last_fb[3] = {0, 0, 0}, last_halvings = 0, last_sweep_fb = 0;
  int last_warm = 0;
  // warm start: all mesh neighbours of free vertices (internal ids), rest
  // positions (SoA), mean rest edge length, feature and output scratch
  int *nptr = nullptr, *nidx = nullptr;
  int* frank = nullptr;  // rank of each internal free vertex among free caller ids
  double* Xr = nullptr;
  double ell = 0;
  float *feat = nullptr, *delta = nullptr;

  MeshView view() const {
    MeshView v{};
    v.D = D; v.n = n; v.nf = nf; v.m = m;
    v.ev = ev; v.dinv_d = dinv_d; v.dinv_f = dinv_f; v.vol_d = vol_d; v.vol_f = vol_f;
    v.mass = mass; v.vperm = d_vperm; v.star_ptr = star_ptr; v.star = star; v.rowptr = d_rowptr;
    v.colidx = d_colidx; v.blkrow = blkrow; v.cptr = cptr; v.centry = centry; v.nnzb = nnzb;
    v.bvert = d_bvert; v.bpos = d_bpos; v.bq_cnt = d_bqcnt; v.hq_slot = d_hqslot;
    v.hq = dense ? hq : nullptr;   // the assembly writes the band copy only for dense bases
    v.qmax = qmax; v.band_w = band_w;
    v.sptr = sptr; v.sidx = sidx; v.U_d = U_d; v.U_f = U_f; v.dense_supp = dense;
    v.smap = smap; v.smap_words = smap_words; v.smap_supp = smap_supp;
    v.sorder = d_sorder;
    v.aorder = d_aorder;
    v.cel_ptr = d_cel_ptr; v.cel = d_cel; v.csl_ptr = d_csl_ptr; v.csl = d_csl;
    v.corr = corr;
    return v;
  }
};

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPC(call)                                    \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) throw HipError{_e, #call};  \
  } while (0)

struct ApiError {
  cc_status code;
  std::string msg;
};

// Exact bases keep a float64 copy (for CC_FP64 steps) while it takes at most
// this many bytes; larger ones are stored in float32 only.
constexpr size_t DENSE_F64_MAX_BYTES = size_t(4) << 30;
// Unknowns per level of the block-tridiagonal exact-basis build.
constexpr int LEVEL_DOFS = 768;

template <typename T>
T* dalloc(size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  HIPC(hipMalloc(&p, count * sizeof(T)));
  return static_cast<T*>(p);
}

template <typename T>
T* dupload(const std::vector<T>& h, hipStream_t s) {
  T* p = dalloc<T>(h.size());
  if (!h.empty()) HIPC(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return p;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

void free_basis(Mesh& M) {
  dfree(M.sptr); dfree(M.sidx); dfree(M.U_d); dfree(M.U_f); dfree(M.smap);
  M.smap_words = 0;
  M.smap_supp = 0;
  M.has_basis = false;
  M.dense = 0;
  M.snnz = 0;
}

void free_mesh(Mesh& M) {
  dfree(M.ev); dfree(M.star_ptr); dfree(M.star); dfree(M.d_rowptr); dfree(M.d_colidx);
  dfree(M.blkrow); dfree(M.cptr); dfree(M.centry); dfree(M.d_vperm); dfree(M.d_vinv);
  dfree(M.d_bvert); dfree(M.d_bpos); dfree(M.d_bqcnt); dfree(M.d_hqslot); dfree(M.hq);
  dfree(M.d_eperm); dfree(M.d_sorder); dfree(M.d_aorder);
  dfree(M.d_cel_ptr); dfree(M.d_cel); dfree(M.d_csl_ptr); dfree(M.d_csl); dfree(M.dinv_d); dfree(M.vol_d); dfree(M.mass); dfree(M.dinv_f); dfree(M.vol_f);
  free_basis(M);
  dfree(M.x); dfree(M.xt); dfree(M.x0); dfree(M.xtrial); dfree(M.dvec); dfree(M.g);
  dfree(M.partials); dfree(M.scal); dfree(M.estore); dfree(M.hb); dfree(M.KL); dfree(M.fb);
  dfree(M.bad); dfree(M.rot); dfree(M.corr);
  dfree(M.nptr); dfree(M.nidx); dfree(M.frank); dfree(M.Xr); dfree(M.feat); dfree(M.delta);
}

}  // namespace

// Scratch of cc_mlp_gradient_noalloc: the per-wave partial gradients and
// losses and the loss scalar of one gradient evaluation, in a file-scope
// device array, so that the entry point allocates nothing.  Each device holds
// its own copy for the life of the process; host code uses only the device
// address resolved once per device (scratch_of), never the array's name.
constexpr size_t NOALLOC_FLOATS = cc::MLP_PART_FLOATS + cc::MLP_LPART_FLOATS + 64;
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

namespace {
std::mutex g_scratch_mu;
std::vector<float*> g_scratch;   // device address of `scratch`, by device id

// Resolve (once per device, with that device current) the address of the
// scratch array; false when the runtime cannot name it.
bool resolve_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch.size() <= device) g_scratch.resize(device + 1, nullptr);
  if (g_scratch[device]) return true;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    return false;
  }
  g_scratch[device] = static_cast<float*>(p);
  return true;
}

float* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device < (int)g_scratch.size() ? g_scratch[device] : nullptr;
}
}  // namespace

struct cc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<Mesh*> meshes;
  double* pinned = nullptr;  // host pinned scalars
  cc::MlpState mlp;          // learned warm start
  float *bfeat = nullptr, *bdelta = nullptr;  // batch-wide feature / output rows
  size_t bcap = 0;
  // kernel timing (cc_profile_*)
  int prof_mask = 0;
  double prof_ms[CC_K_COUNT] = {0};
  long long prof_n[CC_K_COUNT] = {0};
  struct Pending { int kid; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  // batched stepping: tuning and the cached plan of the last batch
  int batch_lanes = 16;
  int batch_iters_per_graph = 4;
  int dense_rows = 0;        // rows per workgroup of the dense condensation (0: most that fit)
  int dense_chunk = 0;       // its chunk of band positions (0: automatic)
  // kernel timing inside the batched path: event pairs of uncaptured launches
  // go to `pending`; pairs captured into the graph stay registered and are
  // read after every replay
  std::vector<Pending> graph_pairs;
  hipEvent_t hook_open[CC_K_COUNT] = {nullptr};
  bool hook_on = false;

  void harvest_graph() {
    for (auto& p : graph_pairs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        prof_ms[p.kid] += ms;
        prof_n[p.kid] += 1;
      }
    }
  }
  void drop_graph_pairs() {
    for (auto& p : graph_pairs) { event_pool.push_back(p.a); event_pool.push_back(p.b); }
    graph_pairs.clear();
  }
  cc::BatchPlan* plan = nullptr;
  std::vector<int> plan_ids;
  // iterations the previous step of this plan needed (most iterating mesh):
  // the next step starts with that many iterations queued before the first
  // host check (finished meshes are masked on the device, so extra queued
  // iterations cost only their launches)
  int plan_prev_iters = 0;
  // most iterations of the previous step of this plan backtracked: they end
  // at the host, so queueing more than one replay ahead only runs masked
  // launches
  bool plan_prev_ls = false;
  std::vector<double> plan_key;

  hipEvent_t take_event() {
    if (!event_pool.empty()) { hipEvent_t e = event_pool.back(); event_pool.pop_back(); return e; }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // Call only after the stream has been synchronised.
  void harvest() {
    for (auto& p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        prof_ms[p.kid] += ms;
        prof_n[p.kid] += 1;
      }
      event_pool.push_back(p.a);
      event_pool.push_back(p.b);
    }
    pending.clear();
  }
  template <typename F>
  void timed(int kid, F&& launch) {
    if (!(prof_mask & (1 << kid))) { launch(); return; }
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) { launch(); return; }
    (void)hipEventRecord(a, stream);
    launch();
    (void)hipEventRecord(b, stream);
    pending.push_back({kid, a, b});
  }
};

namespace {

cc_status fail(cc_ctx* ctx, cc_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

template <typename F>
cc_status guarded(cc_ctx* ctx, F&& f) {
  if (!ctx) return CC_E_INVALID_ARG;
  try {
    HIPC(hipSetDevice(ctx->device));
    return f();
  } catch (const HipError& e) {
    return fail(ctx, CC_E_HIP, std::string("HIP error in ") + e.what + ": " + hipGetErrorString(e.e));
  } catch (const ApiError& e) {
    return fail(ctx, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(ctx, CC_E_INVALID_ARG, "host allocation failed");
  }
}

Mesh& get_mesh(cc_ctx* ctx, int32_t id) {
  if (id < 0 || id >= (int32_t)ctx->meshes.size() || !ctx->meshes[id])
    throw ApiError{CC_E_INVALID_ARG, "unknown mesh id"};
  return *ctx->meshes[id];
}

// ---- rest data ---------------------------------------------------------
bool invert(int D, const double* A, double* Ainv, double& det) {
  if (D == 2) {
    det = A[0] * A[3] - A[1] * A[2];
    if (!(det > 0)) return false;
    Ainv[0] = A[3] / det; Ainv[1] = -A[1] / det; Ainv[2] = -A[2] / det; Ainv[3] = A[0] / det;
    return true;
  }
  const double a = A[0], b = A[1], c = A[2], d = A[3], e = A[4], f = A[5], g = A[6], h = A[7], i = A[8];
  det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  if (!(det > 0)) return false;
  Ainv[0] = (e * i - f * h) / det; Ainv[1] = (c * h - b * i) / det; Ainv[2] = (b * f - c * e) / det;
  Ainv[3] = (f * g - d * i) / det; Ainv[4] = (a * i - c * g) / det; Ainv[5] = (c * d - a * f) / det;
  Ainv[6] = (d * h - e * g) / det; Ainv[7] = (b * g - a * h) / det; Ainv[8] = (a * e - b * d) / det;
  return true;
}

// Band order of the free vertices: breadth-first search over the free-vertex
// graph (edge iff two free vertices share an element) from the free vertices
// that share an element with one connected piece of the Dirichlet set (the
// piece holding its smallest caller id; several pieces, such as the two held
// ends of a beam, would start the search from both ends and double the
// level width), in caller-id order; the unvisited neighbours of each visited
// vertex are appended in caller-id order (a Cuthill-McKee order without the
// degree key, which keeps the structured grids' slabs in lexicographic
// order).  A component reached from no start begins at its smallest caller
// id.  Levels are the breadth-first distances, so every edge joins the same
// or adjacent levels.
// Band order of the free vertices: breadth-first levels from a start set,
// restarted at the smallest caller id left over when the free vertices fall
// apart; within a level, vertices in caller-id order.  Three start sets are
// tried and the order with the smallest band width kept (the ring of the
// dense condensation holds chunk + band width positions): the free vertices
// next to the connected piece of the Dirichlet set holding its smallest id,
// and the free vertices at either end of the rest shape's longest bounding-box
// axis (whose levels, on a bar clamped along a long side, are its short cross
// sections instead of its long ones).
void build_band(Mesh& M) {
  const int nf = M.nf, n = M.n, K = M.K, D = M.D;
  // vertex -> elements
  std::vector<int> vptr(n + 1, 0), vel((size_t)M.m * K);
  for (int e = 0; e < M.m; ++e)
    for (int a = 0; a < K; ++a) vptr[M.elems[e * K + a] + 1]++;
  for (int v = 0; v < n; ++v) vptr[v + 1] += vptr[v];
  {
    std::vector<int> fill(vptr.begin(), vptr.end() - 1);
    for (int e = 0; e < M.m; ++e)
      for (int a = 0; a < K; ++a) vel[fill[M.elems[e * K + a]]++] = e;
  }
  std::vector<std::vector<int>> start_sets;
  {
    std::vector<char> piece(n, 0);      // the chosen connected piece of the Dirichlet set
    int f0 = -1;
    for (int v = 0; v < n && f0 < 0; ++v)
      if (M.fixed[v]) f0 = v;
    if (f0 >= 0) {
      std::vector<int> stack{f0};
      piece[f0] = 1;
      while (!stack.empty()) {
        const int u = stack.back();
        stack.pop_back();
        for (int t = vptr[u]; t < vptr[u + 1]; ++t)
          for (int a = 0; a < K; ++a) {
            const int w = M.elems[vel[t] * K + a];
            if (M.fixed[w] && !piece[w]) { piece[w] = 1; stack.push_back(w); }
          }
      }
    }
    std::vector<char> adj_fixed(nf, 0);
    for (int e = 0; e < M.m; ++e) {
      bool touch = false;
      for (int a = 0; a < K; ++a) touch |= piece[M.elems[e * K + a]] != 0;
      if (!touch) continue;
      for (int a = 0; a < K; ++a) {
        const int v = M.elems[e * K + a];
        if (!M.fixed[v]) adj_fixed[M.vinv[v]] = 1;
      }
    }
    std::vector<int> st;
    for (int j = 0; j < nf; ++j)
      if (adj_fixed[j]) st.push_back(j);
    start_sets.push_back(st);
  }
  if (nf > 0) {
    std::vector<double> lo(D, 1e300), hi(D, -1e300);
    for (int v = 0; v < n; ++v)
      for (int c = 0; c < D; ++c) {
        lo[c] = std::min(lo[c], M.X[(size_t)v * D + c]);
        hi[c] = std::max(hi[c], M.X[(size_t)v * D + c]);
      }
    int ax = 0;
    for (int c = 1; c < D; ++c)
      if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
    double cmin = 1e300, cmax = -1e300;
    for (int j = 0; j < nf; ++j) {
      const double c = M.X[(size_t)M.vperm[j] * D + ax];
      cmin = std::min(cmin, c);
      cmax = std::max(cmax, c);
    }
    const double tol = 1e-6 * (hi[ax] - lo[ax]);
    std::vector<int> s0, s1;
    for (int j = 0; j < nf; ++j) {
      const double c = M.X[(size_t)M.vperm[j] * D + ax];
      if (c <= cmin + tol) s0.push_back(j);
      if (c >= cmax - tol) s1.push_back(j);
    }
    start_sets.push_back(s0);
    start_sets.push_back(s1);
  }
  auto by_caller = [&](int a, int b) { return M.vperm[a] < M.vperm[b]; };
  struct Band { std::vector<int> order, lev; int bw = 0; };
  auto run = [&](std::vector<int> starts) {
    Band B;
    B.lev.assign(nf, -1);
    B.order.reserve(nf);
    int level_base = 0;
    std::vector<int> nb;
    auto bfs = [&](std::vector<int> st) {
      std::sort(st.begin(), st.end(), by_caller);
      size_t head = B.order.size();
      for (int v : st) { B.lev[v] = level_base; B.order.push_back(v); }
      int top = level_base;
      while (head < B.order.size()) {
        const int u = B.order[head++];
        nb.clear();
        for (int t = M.rowptr[u] + 1; t < M.rowptr[u + 1]; ++t)
          if (B.lev[M.colidx[t]] < 0) nb.push_back(M.colidx[t]);
        std::sort(nb.begin(), nb.end(), by_caller);
        for (int w : nb) { B.lev[w] = B.lev[u] + 1; top = std::max(top, B.lev[w]); B.order.push_back(w); }
      }
      level_base = top + 1;
    };
    if (!starts.empty()) bfs(starts);
    while ((int)B.order.size() < nf) {
      int best = -1;
      for (int j = 0; j < nf; ++j)
        if (B.lev[j] < 0 && (best < 0 || M.vperm[j] < M.vperm[best])) best = j;
      bfs({best});
    }
    std::vector<int> pos(nf);
    for (int p = 0; p < nf; ++p) pos[B.order[p]] = p;
    for (int p = 0; p < nf; ++p) {
      const int j = B.order[p];
      for (int t = M.rowptr[j] + 1; t < M.rowptr[j + 1]; ++t) B.bw = std::max(B.bw, pos[M.colidx[t]] - p);
    }
    return B;
  };
  Band best;
  bool have = false;
  for (const auto& st : start_sets) {
    Band B = run(st);
    if (!have || B.bw < best.bw) { best = std::move(B); have = true; }
  }
  if (!have) best = run({});
  M.bvert_h = best.order;
  M.bpos_h.assign(nf, 0);
  for (int p = 0; p < nf; ++p) M.bpos_h[best.order[p]] = p;
  M.lev_off.assign(1, 0);
  for (int p = 1; p <= nf; ++p)
    if (p == nf || best.lev[best.order[p]] != best.lev[best.order[p - 1]]) M.lev_off.push_back(p);
}

void build_mesh(cc_ctx* ctx, Mesh& M) {
  const int D = M.D, K = M.K, n = M.n, m = M.m;
  hipStream_t s = ctx->stream;
  // rest data in caller element order
  std::vector<double> dinv_u((size_t)m * D * D), vol_u(m);
  for (int e = 0; e < m; ++e) {
    double Dm[9], Di[9], det;
    for (int a = 1; a <= D; ++a)
      for (int c = 0; c < D; ++c)
        Dm[c * D + (a - 1)] = M.X[(size_t)M.elems[e * K + a] * D + c] - M.X[(size_t)M.elems[e * K] * D + c];
    if (!invert(D, Dm, Di, det))
      throw ApiError{CC_E_MESH, "element " + std::to_string(e) + " has non-positive rest volume"};
    for (int r = 0; r < D * D; ++r) dinv_u[(size_t)e * D * D + r] = Di[r];
    vol_u[e] = det / (D == 2 ? 2.0 : 6.0);
  }
  std::vector<double> mass_u(n, 0.0);
  M.volume = 0;
  for (int e = 0; e < m; ++e) {
    M.volume += vol_u[e];
    for (int a = 0; a < K; ++a) mass_u[M.elems[e * K + a]] += M.rho * vol_u[e] / K;
  }
  // free-vertex graph and greedy colouring (increasing id, smallest free colour)
  std::vector<std::vector<int>> nbr(n);
  for (int e = 0; e < m; ++e)
    for (int a = 0; a < K; ++a) {
      const int va = M.elems[e * K + a];
      if (M.fixed[va]) continue;
      for (int b = 0; b < K; ++b) {
        const int vb = M.elems[e * K + b];
        if (b != a && !M.fixed[vb]) nbr[va].push_back(vb);
      }
    }
  for (auto& l : nbr) {
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  }
  M.colour.assign(n, -1);
  M.ncol = 0;
  std::vector<int> mark;
  for (int i = 0; i < n; ++i) {
    if (M.fixed[i]) continue;
    mark.assign(nbr[i].size() + 2, 0);
    for (int j : nbr[i]) {
      const int c = M.colour[j];
      if (c >= 0 && c < (int)mark.size()) mark[c] = 1;
    }
    int c = 0;
    while (mark[c]) ++c;
    M.colour[i] = c;
    M.ncol = std::max(M.ncol, c + 1);
  }
  // layouts: vertices by (colour, id), Dirichlet last; elements by (smallest
  // caller id among free vertices, id), all-Dirichlet elements last, so that
  // the elements of neighbouring vertices (in caller order) sit together
  M.vperm.resize(n);
  for (int i = 0; i < n; ++i) M.vperm[i] = i;
  std::stable_sort(M.vperm.begin(), M.vperm.end(), [&](int a, int b) {
    const long long ka = M.colour[a] >= 0 ? M.colour[a] : (1LL << 40);
    const long long kb = M.colour[b] >= 0 ? M.colour[b] : (1LL << 40);
    return ka < kb;
  });
  M.vinv.resize(n);
  for (int v = 0; v < n; ++v) M.vinv[M.vperm[v]] = v;
  M.nf = 0;
  for (int i = 0; i < n; ++i) M.nf += M.fixed[i] ? 0 : 1;
  M.coff.assign(M.ncol + 1, 0);
  for (int i = 0; i < n; ++i)
    if (M.colour[i] >= 0) M.coff[M.colour[i] + 1]++;
  for (int c = 0; c < M.ncol; ++c) M.coff[c + 1] += M.coff[c];
  std::vector<long long> ekey(m);
  for (int e = 0; e < m; ++e) {
    long long k = 1LL << 40;
    for (int a = 0; a < K; ++a) {
      const int v = M.elems[e * K + a];
      if (!M.fixed[v]) k = std::min<long long>(k, v);
    }
    ekey[e] = k;
  }
  M.eperm.resize(m);
  for (int e = 0; e < m; ++e) M.eperm[e] = e;
  std::stable_sort(M.eperm.begin(), M.eperm.end(), [&](int a, int b) { return ekey[a] < ekey[b]; });
  // internal element arrays (SoA)
  std::vector<int> ev((size_t)K * m);
  std::vector<double> dinv_i((size_t)D * D * m), vol_i(m);
  for (int e = 0; e < m; ++e) {
    const int eu = M.eperm[e];
    for (int a = 0; a < K; ++a) ev[(size_t)a * m + e] = M.vinv[M.elems[eu * K + a]];
    for (int r = 0; r < D * D; ++r) dinv_i[(size_t)r * m + e] = dinv_u[(size_t)eu * D * D + r];
    vol_i[e] = vol_u[eu];
  }
  M.mass_int.resize(n);
  for (int v = 0; v < n; ++v) M.mass_int[v] = mass_u[M.vperm[v]];
  {
    double m2 = 0;
    for (int v = 0; v < n; ++v)
      if (!M.fixed[M.vperm[v]]) m2 += M.mass_int[v] * M.mass_int[v];
    M.mass_free_norm = std::sqrt(m2);
  }
  // star of every free vertex (internal), in element order
  const int nf = M.nf;
  std::vector<int> star_ptr(nf + 1, 0);
  for (int e = 0; e < m; ++e)
    for (int a = 0; a < K; ++a)
      if (ev[(size_t)a * m + e] < nf) star_ptr[ev[(size_t)a * m + e] + 1]++;
  for (int j = 0; j < nf; ++j) star_ptr[j + 1] += star_ptr[j];
  std::vector<int> star(star_ptr[nf]), fill(star_ptr.begin(), star_ptr.end() - 1);
  for (int e = 0; e < m; ++e)
    for (int a = 0; a < K; ++a) {
      const int v = ev[(size_t)a * m + e];
      if (v < nf) star[fill[v]++] = e * 4 + a;
    }
  // block rows (diagonal first, then neighbours by internal id)
  M.rowptr.assign(nf + 1, 0);
  M.colidx.clear();
  for (int j = 0; j < nf; ++j) {
    std::vector<int> row;
    for (int u : nbr[M.vperm[j]]) row.push_back(M.vinv[u]);
    std::sort(row.begin(), row.end());
    M.colidx.push_back(j);
    for (int k : row) M.colidx.push_back(k);
    M.rowptr[j + 1] = (int)M.colidx.size();
  }
  M.nnzb = (int)M.colidx.size();
  std::vector<int> blkrow(M.nnzb);
  for (int j = 0; j < nf; ++j)
    for (int t = M.rowptr[j]; t < M.rowptr[j + 1]; ++t) blkrow[t] = j;
  // element contributions of every block slot
  std::vector<std::vector<int>> contrib(M.nnzb);
  for (int j = 0; j < nf; ++j)
    for (int t = star_ptr[j]; t < star_ptr[j + 1]; ++t) {
      const int e = star[t] >> 2, a = star[t] & 3;
      for (int b = 0; b < K; ++b) {
        const int k = ev[(size_t)b * m + e];
        if (k >= nf) continue;
        int slot;
        if (k == j) {
          slot = M.rowptr[j];
        } else {
          auto it = std::lower_bound(M.colidx.begin() + M.rowptr[j] + 1, M.colidx.begin() + M.rowptr[j + 1], k);
          slot = (int)(it - M.colidx.begin());
        }
        contrib[slot].push_back(e * 16 + a * 4 + b);
      }
    }
  std::vector<int> cptr(M.nnzb + 1, 0), centry;
  for (int t = 0; t < M.nnzb; ++t) {
    cptr[t + 1] = cptr[t] + (int)contrib[t].size();
    centry.insert(centry.end(), contrib[t].begin(), contrib[t].end());
  }
  std::vector<float> dinv_f(dinv_i.begin(), dinv_i.end()), vol_f(vol_i.begin(), vol_i.end());
  // device uploads
  M.ev = dupload(ev, s);
  M.dinv_d = dupload(dinv_i, s);
  M.dinv_f = dupload(dinv_f, s);
  M.vol_d = dupload(vol_i, s);
  M.vol_f = dupload(vol_f, s);
  M.mass = dupload(M.mass_int, s);
  M.star_ptr = dupload(star_ptr, s);
  M.star = dupload(star, s);
  M.d_rowptr = dupload(M.rowptr, s);
  M.d_colidx = dupload(M.colidx, s);
  M.blkrow = dupload(blkrow, s);
  build_band(M);
  M.d_bvert = dupload(M.bvert_h, s);
  M.d_bpos = dupload(M.bpos_h, s);
  {
    // upper blocks of every band row: the diagonal first, then by band position
    std::vector<int> cnt(nf, 0), hslot(M.nnzb, -1);
    std::vector<std::vector<std::pair<int, int>>> up(nf);
    M.qmax = 0;
    M.band_w = 0;
    for (int p = 0; p < nf; ++p) {
      const int j = M.bvert_h[p];
      for (int t = M.rowptr[j]; t < M.rowptr[j + 1]; ++t) {
        const int pk = M.bpos_h[M.colidx[t]];
        if (pk >= p) up[p].push_back({pk, t});
      }
      std::sort(up[p].begin(), up[p].end());
      cnt[p] = (int)up[p].size();
      M.qmax = std::max(M.qmax, cnt[p]);
      if (!up[p].empty()) M.band_w = std::max(M.band_w, up[p].back().first - p);
    }
    for (int p = 0; p < nf; ++p)
      for (int q = 0; q < cnt[p]; ++q) hslot[up[p][q].second] = q * nf + p;
    M.d_bqcnt = dupload(cnt, s);
    M.d_hqslot = dupload(hslot, s);
    // one BandRec per (q, p), sized for float64 (float32 records are smaller);
    // records past a row's count are never read
    const size_t rec = D == 2 ? sizeof(cc::BandRec<double, 2>) : sizeof(cc::BandRec<double, 3>);
    const size_t hqb = (size_t)std::max(M.qmax, 1) * std::max(nf, 1) * rec;
    M.hq = dalloc<double>(hqb / sizeof(double));
    HIPC(hipMemsetAsync(M.hq, 0, hqb, s));
  }
  M.cptr = dupload(cptr, s);
  M.centry = dupload(centry, s);
  M.d_vperm = dupload(M.vperm, s);
  M.d_vinv = dupload(M.vinv, s);
  {  // free internal ids by caller id
    std::vector<int> so;
    so.reserve(nf);
    for (int u = 0; u < n; ++u)
      if (M.vinv[u] < nf) so.push_back(M.vinv[u]);
    M.d_sorder = dupload(so, s);
    std::vector<int> ao;
    ao.reserve(M.nnzb);
    for (int j : so)
      for (int t = M.rowptr[j]; t < M.rowptr[j + 1]; ++t) ao.push_back(t);
    M.d_aorder = dupload(ao, s);
    // per colour: elements with a free vertex of the colour (element order),
    // and the block slots they contribute to (assembly order)
    std::vector<int> slot_rank(M.nnzb);
    for (size_t r = 0; r < ao.size(); ++r) slot_rank[ao[r]] = (int)r;
    std::vector<int> cel_ptr(M.ncol + 1, 0), cel, csl_ptr(M.ncol + 1, 0), csl;
    std::vector<int> emark(m, -1), smark(M.nnzb, -1);
    for (int c = 0; c < M.ncol; ++c) {
      for (int e = 0; e < m; ++e)
        for (int a = 0; a < K; ++a) {
          const int v = ev[(size_t)a * m + e];
          if (v < nf && M.colour[M.vperm[v]] == c) { emark[e] = c; break; }
        }
      for (int e = 0; e < m; ++e)
        if (emark[e] == c) cel.push_back(e);
      cel_ptr[c + 1] = (int)cel.size();
      std::vector<int> sl;
      for (int t = 0; t < M.nnzb; ++t)
        for (int q = cptr[t]; q < cptr[t + 1]; ++q)
          if (emark[centry[q] >> 4] == c) { sl.push_back(t); break; }
      std::sort(sl.begin(), sl.end(), [&](int a, int b) { return slot_rank[a] < slot_rank[b]; });
      csl.insert(csl.end(), sl.begin(), sl.end());
      csl_ptr[c + 1] = (int)csl.size();
    }
    (void)smark;
    M.d_cel_ptr = dupload(cel_ptr, s);
    M.d_cel = dupload(cel, s);
    M.d_csl_ptr = dupload(csl_ptr, s);
    M.d_csl = dupload(csl, s);
    M.cel_ptr_h = cel_ptr;
    M.csl_ptr_h = csl_ptr;
  }
  M.d_eperm = dupload(M.eperm, s);
  {  // warm-start data: all neighbours, rest positions, mean rest edge length
    std::vector<std::vector<int>> alln(nf);
    double esum = 0;
    long long ecnt = 0;
    for (int e = 0; e < m; ++e)
      for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
          const int va = M.elems[e * K + a], vb = M.elems[e * K + b];
          if (a < b) {
            double l2 = 0;
            for (int c = 0; c < D; ++c) {
              const double dd = M.X[(size_t)va * D + c] - M.X[(size_t)vb * D + c];
              l2 += dd * dd;
            }
            esum += std::sqrt(l2);
            ++ecnt;
          }
          if (a != b && !M.fixed[va]) alln[M.vinv[va]].push_back(M.vinv[vb]);
        }
    M.ell = ecnt ? esum / ecnt : 1.0;
    std::vector<int> nptr(nf + 1, 0), nidx;
    for (int j = 0; j < nf; ++j) {
      auto& l = alln[j];
      std::sort(l.begin(), l.end());
      l.erase(std::unique(l.begin(), l.end()), l.end());
      nidx.insert(nidx.end(), l.begin(), l.end());
      nptr[j + 1] = (int)nidx.size();
    }
    M.nptr = dupload(nptr, s);
    M.nidx = dupload(nidx, s);
    std::vector<double> Xr((size_t)D * n);
    for (int v = 0; v < n; ++v)
      for (int c = 0; c < D; ++c) Xr[(size_t)c * n + v] = M.X[(size_t)M.vperm[v] * D + c];
    M.Xr = dupload(Xr, s);
    std::vector<int> frank(nf);
    {
      int r = 0;
      for (int u = 0; u < n; ++u)
        if (!M.fixed[u]) frank[M.vinv[u]] = r++;
    }
    M.frank = dupload(frank, s);
    M.feat = dalloc<float>((size_t)std::max(nf, 1) * 16);
    M.delta = dalloc<float>((size_t)std::max(nf, 1) * 3);
  }
  // work buffers
  const size_t nd = (size_t)D * n;
  M.x = dalloc<double>(nd); M.xt = dalloc<double>(nd); M.x0 = dalloc<double>(nd);
  M.xtrial = dalloc<double>(nd); M.dvec = dalloc<double>(nd); M.g = dalloc<double>(nd);
  HIPC(hipMemsetAsync(M.g, 0, nd * sizeof(double), s));
  HIPC(hipMemsetAsync(M.dvec, 0, nd * sizeof(double), s));
  const int cap = cc::reduce_partials_capacity(M.view());
  M.partials = dalloc<double>(cap);
  M.scal = dalloc<double>(8);
  const int NB = K * (K + 1) / 2;
  M.estore = dalloc<double>((size_t)NB * m * D * D);
  M.hb = dalloc<double>((size_t)M.nnzb * D * D);
  M.KL = dalloc<double>((size_t)nf * 2 * D * D);
  M.rot = dalloc<double>((size_t)std::max(nf, 1) * D * D);
  M.corr = dalloc<double>((size_t)D * n);
  HIPC(hipMemsetAsync(M.corr, 0, (size_t)D * n * sizeof(double), s));
  M.fb = dalloc<unsigned long long>(4);
  M.bad = dalloc<int>(1);
  HIPC(hipStreamSynchronize(s));
}

// ---- basis upload ------------------------------------------------------
// Slot map of a sparse basis (MeshView::smap): one byte per support entry
// (i, j) and block of row j, so the condensation kernel finds U_i[k] for each
// block (j, k), k >= j, without searching supp(i).  Left null, and the kernel searches,
// when a support holds more than SMAP_SELF entries or a row more than
// 4 * SMAP_MAX_WORDS blocks.
void build_slot_map(Mesh& M, const std::vector<int64_t>& sptr, const std::vector<int>& sidx,
                    hipStream_t s) {
  const int nf = M.nf;
  int maxrow = 0;
  int64_t maxsupp = 0;
  for (int j = 0; j < nf; ++j) maxrow = std::max(maxrow, M.rowptr[j + 1] - M.rowptr[j]);
  for (int i = 0; i < nf; ++i) maxsupp = std::max(maxsupp, sptr[i + 1] - sptr[i]);
  const int words = (maxrow + 3) / 4;
  if (sptr[nf] == 0 || maxsupp > cc::SMAP_SELF || words > cc::SMAP_MAX_WORDS) return;
  const int stride = words + 1;   // row start of j, then the codes
  std::vector<uint32_t> map((size_t)sptr[nf] * stride, 0xffffffffu);
  for (int i = 0; i < nf; ++i) {
    const int* s0 = sidx.data() + sptr[i];
    const int* s1 = sidx.data() + sptr[i + 1];
    for (int64_t q = sptr[i]; q < sptr[i + 1]; ++q) {
      const int j = sidx[q];
      map[(size_t)q * stride] = (uint32_t)M.rowptr[j];
      uint8_t* b = reinterpret_cast<uint8_t*>(&map[(size_t)q * stride + 1]);
      for (int t = M.rowptr[j]; t < M.rowptr[j + 1]; ++t) {
        const int k = M.colidx[t];
        uint8_t code = (uint8_t)cc::SMAP_SKIP;
        if (k == i) {
          code = (uint8_t)cc::SMAP_SELF;
        } else if (k >= j) {   // blocks below the diagonal enter through symmetry
          const int* it = std::lower_bound(s0, s1, k);
          if (it != s1 && *it == k) code = (uint8_t)(it - s0);
        }
        b[t - M.rowptr[j]] = code;
      }
    }
  }
  M.smap = dupload(map, s);
  M.smap_words = words;
  M.smap_supp = (int)maxsupp;
}

void upload_basis(cc_ctx* ctx, Mesh& M, const int64_t* ptr, const int32_t* idx, const double* U) {
  const int D = M.D, DD = D * D, n = M.n, nf = M.nf;
  if (!ptr || (ptr[n] > 0 && (!idx || !U))) throw ApiError{CC_E_INVALID_ARG, "null basis array"};
  if (ptr[0] != 0) throw ApiError{CC_E_SUBSPACE, "ptr[0] must be 0"};
  for (int i = 0; i < n; ++i) {
    if (ptr[i + 1] < ptr[i]) throw ApiError{CC_E_SUBSPACE, "ptr must be non-decreasing"};
    if (M.fixed[i] && ptr[i + 1] != ptr[i])
      throw ApiError{CC_E_SUBSPACE, "row of Dirichlet vertex " + std::to_string(i) + " is not empty"};
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
      const int j = idx[k];
      if (j < 0 || j >= n) throw ApiError{CC_E_SUBSPACE, "basis index out of range"};
      if (j == i) throw ApiError{CC_E_SUBSPACE, "basis row contains its own vertex"};
      if (M.fixed[j]) throw ApiError{CC_E_SUBSPACE, "basis index names a Dirichlet vertex"};
      if (k > ptr[i] && idx[k - 1] >= j) throw ApiError{CC_E_SUBSPACE, "basis row not strictly ascending"};
    }
  }
  const int64_t nnz = ptr[n];
  for (int64_t k = 0; k < nnz * DD; ++k)
    if (!std::isfinite(U[k])) throw ApiError{CC_E_NONFINITE, "non-finite basis entry"};
  // internal rows: internal vertex i <- caller vertex vperm[i], entries sorted by internal id
  std::vector<int64_t> sptr(nf + 1, 0);
  for (int i = 0; i < nf; ++i) {
    const int u = M.vperm[i];
    sptr[i + 1] = sptr[i] + (ptr[u + 1] - ptr[u]);
  }
  std::vector<int> sidx(nnz);
  std::vector<double> Ud((size_t)nnz * DD);
  bool dense = true;
  std::vector<std::pair<int, int64_t>> row;
  for (int i = 0; i < nf; ++i) {
    const int u = M.vperm[i];
    row.clear();
    for (int64_t k = ptr[u]; k < ptr[u + 1]; ++k) row.push_back({M.vinv[idx[k]], k});
    std::sort(row.begin(), row.end());
    for (size_t t = 0; t < row.size(); ++t) {
      sidx[sptr[i] + t] = row[t].first;
      std::memcpy(&Ud[(size_t)(sptr[i] + t) * DD], &U[(size_t)row[t].second * DD], DD * sizeof(double));
    }
    if ((int)row.size() != nf - 1) dense = false;
  }
  free_basis(M);
  hipStream_t s = ctx->stream;
  if (dense && nf > 1) {
    // every row holds every other free vertex: the band layout of the exact
    // basis (nf blocks per row, columns by band position, own block zero)
    const size_t blocks = (size_t)nf * nf;
    std::vector<double> band(blocks * DD, 0.0);
    for (int i = 0; i < nf; ++i)
      for (int64_t q = sptr[i]; q < sptr[i + 1]; ++q)
        std::memcpy(&band[((size_t)i * nf + M.bpos_h[sidx[q]]) * DD], &Ud[(size_t)q * DD], DD * sizeof(double));
    if (blocks * DD * sizeof(double) <= DENSE_F64_MAX_BYTES) M.U_d = dupload(band, s);
    std::vector<float> Uf(band.begin(), band.end());
    M.U_f = dupload(Uf, s);
    M.dense = 1;
  } else {
    M.sptr = dupload(sptr, s);
    M.sidx = dupload(sidx, s);
    M.U_d = dupload(Ud, s);
    std::vector<float> Uf(Ud.begin(), Ud.end());
    M.U_f = dupload(Uf, s);
    M.dense = 0;
    build_slot_map(M, sptr, sidx, s);
  }
  M.snnz = nnz;

  HIPC(hipStreamSynchronize(s));
  M.has_basis = true;
}

// dense Cholesky A = L L^T (row-major, in place lower); false if not SPD
bool dense_chol(std::vector<double>& A, int N) {
  for (int j = 0; j < N; ++j) {
    double s = A[(size_t)j * N + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * N + k] * A[(size_t)j * N + k];
    if (!(s > 0)) return false;
    const double l = std::sqrt(s);
    A[(size_t)j * N + j] = l;
    for (int i = j + 1; i < N; ++i) {
      double t = A[(size_t)i * N + j];
      const double* ri = &A[(size_t)i * N];
      const double* rj = &A[(size_t)j * N];
      for (int k = 0; k < j; ++k) t -= ri[k] * rj[k];
      A[(size_t)i * N + j] = t / l;
    }
  }
  return true;
}

// solve L L^T X = B for R right-hand sides stored row-major N x R
void dense_chol_solve(const std::vector<double>& L, int N, std::vector<double>& B, int R) {
  for (int i = 0; i < N; ++i)
    for (int r = 0; r < R; ++r) {
      double s = B[(size_t)i * R + r];
      for (int k = 0; k < i; ++k) s -= L[(size_t)i * N + k] * B[(size_t)k * R + r];
      B[(size_t)i * R + r] = s / L[(size_t)i * N + i];
    }
  for (int i = N - 1; i >= 0; --i)
    for (int r = 0; r < R; ++r) {
      double s = B[(size_t)i * R + r];
      for (int k = i + 1; k < N; ++k) s -= L[(size_t)k * N + i] * B[(size_t)k * R + r];
      B[(size_t)i * R + r] = s / L[(size_t)i * N + i];
    }
}

// x_user: null for the rest state, else caller-order device positions (n x D)
void build_basis(cc_ctx* ctx, Mesh& M, int radius, double dt, int quasi, const double* x_user = nullptr) {
  const int D = M.D, DD = D * D, nf = M.nf, n = M.n;
  hipStream_t s = ctx->stream;
  // Hessian block rows in float64 from the library's kernels, at rest or at x_user
  if (x_user == nullptr) {
    std::vector<double> Xi((size_t)D * n);
    for (int v = 0; v < n; ++v)
      for (int c = 0; c < D; ++c) Xi[(size_t)c * n + v] = M.X[(size_t)M.vperm[v] * D + c];
    HIPC(hipMemcpyAsync(M.x, Xi.data(), Xi.size() * sizeof(double), hipMemcpyHostToDevice, s));
  } else {
    cc::launch_gather_user(M.view(), M.d_vinv, x_user, M.x, s);
  }
  Material mat{};
  mat.mu = M.mu; mat.lam = M.lam; mat.model = M.model;
  mat.w_in = quasi ? 0.0 : 1.0;
  mat.s_el = quasi ? 1.0 : dt * dt;
  MeshView mv = M.view();
  cc::launch_elem_hess(mv, 0, M.x, mat, mat.s_el, M.estore, s);
  cc::launch_assemble(mv, 0, M.estore, mat, M.hb, s);
  if (radius == 0) {  // exact basis from the block-tridiagonal factorisation of H (band order)
    const size_t blocks = (size_t)nf * nf;
    // breadth-first levels merged until each holds at least LEVEL_DOFS unknowns
    // (fewer, larger products; merged levels still couple only neighbours)
    std::vector<int> loff{0};
    for (size_t t = 1; t < M.lev_off.size(); ++t) {
      const int b = M.lev_off[t];
      if ((b - loff.back()) * D >= LEVEL_DOFS || b == nf) loff.push_back(b);
    }
    double* Ud = nullptr;
    float* Uf = nullptr;
    try {
      Uf = dalloc<float>(blocks * DD);
      if (blocks * DD * sizeof(double) <= DENSE_F64_MAX_BYTES) Ud = dalloc<double>(blocks * DD);
    } catch (...) {
      dfree(Ud); dfree(Uf);
      throw;
    }
    const int rc = cc::exact_basis_band(mv, (const double*)M.hb, loff.data(), (int)loff.size() - 1, Ud, Uf, s);
    if (rc != 0) {
      dfree(Ud); dfree(Uf);
      if (rc == 1) throw ApiError{CC_E_SUBSPACE, "step Hessian not positive definite"};
      throw ApiError{CC_E_HIP, "exact basis: out of device memory or a failed launch"};
    }
    free_basis(M);
    M.U_d = Ud;
    M.U_f = Uf;
    M.dense = 1;
    M.snnz = (int64_t)nf * (nf > 0 ? nf - 1 : 0);
    HIPC(hipStreamSynchronize(s));
    M.has_basis = true;
    return;
  }
  std::vector<double> hb((size_t)M.nnzb * DD);
  HIPC(hipMemcpyAsync(hb.data(), M.hb, hb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  auto block = [&](int j, int k, double* out) -> bool {  // H_jk, false if structurally zero
    if (j == k) {
      std::memcpy(out, &hb[(size_t)M.rowptr[j] * DD], DD * sizeof(double));
      return true;
    }
    auto b = M.colidx.begin() + M.rowptr[j] + 1, e = M.colidx.begin() + M.rowptr[j + 1];
    auto it = std::lower_bound(b, e, k);
    if (it == e || *it != k) return false;
    std::memcpy(out, &hb[(size_t)(it - M.colidx.begin()) * DD], DD * sizeof(double));
    return true;
  };
  // supports (internal ids), then U rows in internal order
  std::vector<std::vector<int>> supp(nf);
  if (radius > 0) {
    std::vector<int> seen(nf, -1);
    for (int i = 0; i < nf; ++i) {
      std::vector<int> frontier{i}, all;
      seen[i] = i;
      for (int r = 0; r < radius; ++r) {
        std::vector<int> nxt;
        for (int v : frontier)
          for (int t = M.rowptr[v] + 1; t < M.rowptr[v + 1]; ++t) {
            const int w = M.colidx[t];
            if (seen[w] != i) { seen[w] = i; nxt.push_back(w); all.push_back(w); }
          }
        frontier.swap(nxt);
      }
      std::sort(all.begin(), all.end());
      supp[i] = all;
    }
  }
  std::vector<std::vector<double>> Urows(nf);
  if (radius > 0) {
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    std::vector<int> failed(nth, 0);
    for (unsigned w = 0; w < nth; ++w)
      pool.emplace_back([&, w]() {
        std::vector<double> A, B;
        std::vector<int> pos(nf, -1);
        for (int i = (int)w; i < nf; i += (int)nth) {
          const auto& C = supp[i];
          const int nc = (int)C.size(), N = nc * D;
          if (nc == 0) continue;
          for (int a = 0; a < nc; ++a) pos[C[a]] = a;
          A.assign((size_t)N * N, 0.0);
          B.assign((size_t)N * D, 0.0);
          double blk[9];
          for (int a = 0; a < nc; ++a) {
            const int j = C[a];
            for (int t = M.rowptr[j]; t < M.rowptr[j + 1]; ++t) {
              const int k = M.colidx[t];
              if (k == i) {
                for (int r = 0; r < D; ++r)
                  for (int c2 = 0; c2 < D; ++c2) B[(size_t)(a * D + r) * D + c2] = -hb[(size_t)t * DD + r * D + c2];
              } else if (pos[k] >= 0 && (k == j || std::binary_search(C.begin(), C.end(), k))) {
                const int bcol = pos[k];
                for (int r = 0; r < D; ++r)
                  for (int c2 = 0; c2 < D; ++c2)
                    A[(size_t)(a * D + r) * N + bcol * D + c2] = hb[(size_t)t * DD + r * D + c2];
              }
            }
          }
          (void)blk;
          if (!dense_chol(A, N)) { failed[w] = 1; }
          else dense_chol_solve(A, N, B, D);
          Urows[i] = B;
          for (int a = 0; a < nc; ++a) pos[C[a]] = -1;
        }
      });
    for (auto& t : pool) t.join();
    for (int f : failed)
      if (f) throw ApiError{CC_E_SUBSPACE, "patch Hessian not positive definite"};
  }
  // convert to the caller format (caller ids, ascending) and upload
  std::vector<int64_t> ptr(n + 1, 0);
  for (int i = 0; i < nf; ++i) ptr[M.vperm[i] + 1] = (int64_t)supp[i].size();
  for (int u = 0; u < n; ++u) ptr[u + 1] += ptr[u];
  std::vector<int> idx(ptr[n]);
  std::vector<double> U((size_t)ptr[n] * DD);
  for (int i = 0; i < nf; ++i) {
    const int u = M.vperm[i];
    std::vector<std::pair<int, int>> ord;
    for (int a = 0; a < (int)supp[i].size(); ++a) ord.push_back({M.vperm[supp[i][a]], a});
    std::sort(ord.begin(), ord.end());
    for (size_t t = 0; t < ord.size(); ++t) {
      idx[ptr[u] + t] = ord[t].first;
      const int a = ord[t].second;
      for (int r = 0; r < D; ++r)
        for (int c2 = 0; c2 < D; ++c2)
          U[(size_t)(ptr[u] + t) * DD + r * D + c2] = Urows[i][(size_t)(a * D + r) * D + c2];
    }
  }
  upload_basis(ctx, M, ptr.data(), idx.data(), U.data());
}

// The floor of the convergence test's denominator: the larger of
// |s_el m_i grav| over the free degrees of freedom (the gravity load's part of
// the step gradient, which keeps the test reachable for a loaded body that has
// settled) and 1e-8 s_el E V^((D-1)/D) (V the rest volume: 1e-8 of the elastic
// force scale, which does the same for an unloaded body at rest, whose start
// gradient is only the rounding of its element forces).
double load_norm(const Mesh& M, const Material& mat) {
  double g2 = 0;
  for (int c = 0; c < M.D; ++c) g2 += mat.grav[c] * mat.grav[c];
  const double floor = 1e-8 * mat.s_el * M.E * std::pow(M.volume, (M.D - 1.0) / M.D);
  return std::max(mat.s_el * M.mass_free_norm * std::sqrt(g2), floor);
}

// ---- step driver ---------------------------------------------------------
struct Stepper {
  cc_ctx* ctx;
  Mesh& M;
  MeshView mv;
  Material mat;
  const cc_params& p;
  hipStream_t s;

  double read_scalar(const double* dptr) {
    HIPC(hipMemcpyAsync(ctx->pinned, dptr, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    ctx->harvest();
    return ctx->pinned[0];
  }
  double energy(const double* x) {
    int np = 0;
    ctx->timed(CC_K_ENERGY, [&] { cc::launch_energy(mv, x, M.xt, mat, M.partials, &np, s); });
    cc::launch_reduce(M.partials, np, M.scal, s);
    return read_scalar(M.scal);
  }
  double grad_norm2(const double* x) {
    int np = 0;
    ctx->timed(CC_K_GRADIENT, [&] { cc::launch_gradient(mv, x, M.xt, mat, M.g, M.partials, &np, s); });
    if (np == 0) return 0.0;
    cc::launch_reduce(M.partials, np, M.scal + 1, s);
    return read_scalar(M.scal + 1);
  }
  void gradient_only(const double* x) {
    int np = 0;
    ctx->timed(CC_K_GRADIENT, [&] { cc::launch_gradient(mv, x, M.xt, mat, M.g, M.partials, &np, s); });
  }
  // Element Hessians and block rows at x: of every element (colour < 0), or
  // only of those that the moves of colour `colour`'s vertices changed.
  void hessian(const double* x, int colour = -1) {
    mv.rot = p.corotate ? M.rot : nullptr;   // corotation: rotations at the Hessian's positions
    if (p.corotate) {
      if (!M.rot || !M.nptr || !M.nidx || !M.Xr)
        throw ApiError{CC_E_STATE, "corotation buffers missing"};
      cc::launch_rotations(mv, x, M.nptr, M.nidx, M.Xr, M.rot, s);
    }
    const int* el = colour < 0 ? nullptr : mv.cel + M.cel_ptr_h[colour];
    const int ne = colour < 0 ? M.m : M.cel_ptr_h[colour + 1] - M.cel_ptr_h[colour];
    const int* sl = colour < 0 ? nullptr : mv.csl + M.csl_ptr_h[colour];
    const int ns = colour < 0 ? M.nnzb : M.csl_ptr_h[colour + 1] - M.csl_ptr_h[colour];
    ctx->timed(CC_K_ELEM_HESS, [&] {
      cc::launch_elem_hess_list(mv, p.precision, x, mat, mat.s_el, M.estore, s, el, ne);
    });
    ctx->timed(CC_K_ASSEMBLE, [&] {
      cc::launch_assemble_list(mv, p.precision, M.estore, mat, M.hb, s, sl, ns);
      // a partial assembly leaves band records of unchanged blocks whose
      // rotations did change
      if (colour >= 0 && mv.rot != nullptr) cc::launch_band_copy(mv, p.precision, M.hb, s);
    });
  }
  void prep(int method, int v0, int v1) {
    ctx->timed(CC_K_CC_PREP, [&] {
      cc::launch_cc_prep(mv, p.precision, method, v0, v1, M.hb, M.KL, M.fb, s, nullptr, nullptr, nullptr,
                         ctx->dense_rows, ctx->dense_chunk);
    });
  }
  // Condensation that also writes the Jacobi directions into out when the
  // dense path can (g must hold the gradient at the same x); false: call update.
  bool prep_direction(int method, double* out) {
    bool done = false;
    ctx->timed(CC_K_CC_PREP, [&] {
      done = cc::launch_cc_prep(mv, p.precision, method, 0, M.nf, M.hb, M.KL, M.fb, s, M.g, out, nullptr,
                                ctx->dense_rows, ctx->dense_chunk);
    });
    return done;
  }
  void update(int method, int v0, int v1, double* out, int acc) {
    ctx->timed(CC_K_CC_UPDATE, [&] { cc::launch_cc_update(mv, p.precision, method, v0, v1, M.KL, M.g, out, acc, s); });
  }
  // One sweep from x into out (x unchanged).  method as requested.
  // sweep_kind: CC_SWEEP_* to override p.sweep (the line search's Jacobi
  // fallback of a coloured sweep), -1 for p.sweep
  void sweep(const double* x, double* out, int method, int sweep_kind = -1) {
    const int nd = M.D * M.n;
    if ((sweep_kind < 0 ? p.sweep : sweep_kind) == CC_SWEEP_JACOBI) {
      hessian(x);
      gradient_only(x);
      if (!prep_direction(method, M.dvec)) update(method, 0, M.nf, M.dvec, 0);
      cc::launch_axpy(nd, x, M.dvec, 1.0, out, s);
      return;
    }
    HIPC(hipMemcpyAsync(out, x, (size_t)nd * sizeof(double), hipMemcpyDeviceToDevice, s));
    int moved = -1;   // the last colour that moved in this sweep
    for (int c = 0; c < M.ncol; ++c) {
      const int v0 = M.coff[c], v1 = M.coff[c + 1];
      if (v1 <= v0) continue;
      if (p.hess_refresh == CC_HESS_PER_COLOR) {
        // every Hessian at the sweep's start, then only what the previous
        // colour's moves changed
        hessian(out, moved);
        moved = c;
        gradient_only(out);
        // a dense basis forms b_i from this gradient and moves the colour's
        // vertices in the finish kernel; other bases take the update kernel
        bool done = false;
        ctx->timed(CC_K_CC_PREP, [&] {
          done = cc::launch_cc_prep(mv, p.precision, method, v0, v1, M.hb, M.KL, M.fb, s, M.g, M.dvec, out,
                                    ctx->dense_rows, ctx->dense_chunk);
        });
        if (!done) update(method, v0, v1, out, 1);
        continue;
      }
      if (c == 0) {
        hessian(out);
        prep(method, 0, M.nf);
      }
      gradient_only(out);
      update(method, v0, v1, out, 1);
    }
  }
};

}  // namespace

// Empty kernel: the boundary of a timed region in a kernel trace
// (cc_profile_enable).
__global__ void k_profile_mark() {}

extern "C" {

void cc_params_default(cc_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->method = CC_METHOD_CC;
  p->sweep = CC_SWEEP_JACOBI;
  p->hess_refresh = CC_HESS_PER_COLOR;
  p->precision = CC_FP64;
  p->line_search = 1;
  p->max_iters = 10000;
  p->max_halvings = 20;
}

cc_status cc_create(int32_t device, void* hip_stream, cc_ctx** out) {
  if (!out) return CC_E_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return CC_E_NO_DEVICE;
  if (device < 0 || device >= count) return CC_E_INVALID_ARG;
  cc_ctx* ctx = new (std::nothrow) cc_ctx();
  if (!ctx) return CC_E_INVALID_ARG;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void**)&ctx->pinned, 64 * 1024, hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return CC_E_HIP;
  }
  if (!resolve_scratch(device)) {   // address of this device's scratch array
    (void)hipHostFree(ctx->pinned);
    delete ctx;
    return CC_E_HIP;
  }
  int lds = 0;  // per-workgroup LDS budget of the dense condensation
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
      lds > 0)
    cc::set_lds_limit((size_t)lds);
  *out = ctx;
  return CC_OK;
}

void cc_destroy(cc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (Mesh* M : ctx->meshes)
    if (M) { free_mesh(*M); delete M; }
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->plan) cc::batch_plan_destroy(ctx->plan);
  ctx->harvest();
  ctx->drop_graph_pairs();
  {
    cc::MlpState& q = ctx->mlp;
    dfree(q.W); dfree(q.m); dfree(q.v); dfree(q.grad); dfree(q.part); dfree(q.lpart); dfree(q.loss);
    dfree(q.W1b); dfree(q.W2b); dfree(q.W3b); dfree(q.mean); dfree(q.istd);
  }
  dfree(ctx->bfeat);
  dfree(ctx->bdelta);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  delete ctx;
}

const char* cc_last_error(const cc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

cc_status cc_profile_enable(cc_ctx* ctx, int32_t mask) {
  return guarded(ctx, [&]() -> cc_status {
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->harvest();
    // an empty kernel marks where a timed region starts and ends in a
    // kernel trace
    if (mask != 0 || ctx->prof_mask != 0) {
      k_profile_mark<<<1, 64, 0, ctx->stream>>>();
      HIPC(hipGetLastError());
    }
    ctx->prof_mask = mask;
    for (int k = 0; k < CC_K_COUNT; ++k) { ctx->prof_ms[k] = 0; ctx->prof_n[k] = 0; }
    return CC_OK;
  });
}

cc_status cc_profile_read(cc_ctx* ctx, int32_t kernel_id, double* total_ms, int64_t* launches) {
  return guarded(ctx, [&]() -> cc_status {
    if (kernel_id < 0 || kernel_id >= CC_K_COUNT) return fail(ctx, CC_E_INVALID_ARG, "bad kernel id");
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->harvest();
    if (total_ms) *total_ms = ctx->prof_ms[kernel_id];
    if (launches) *launches = ctx->prof_n[kernel_id];
    return CC_OK;
  });
}

cc_status cc_mesh_upload(cc_ctx* ctx, int32_t dim, int32_t n_verts, const double* X, int32_t n_elems,
                         const int32_t* elems, const uint8_t* is_fixed, double youngs, double poisson,
                         double density, int32_t* mesh_id) {
  return guarded(ctx, [&]() -> cc_status {
    if ((dim != 2 && dim != 3) || n_verts <= 0 || n_elems < 0 || !X || !is_fixed || !mesh_id ||
        (n_elems > 0 && !elems))
      return fail(ctx, CC_E_INVALID_ARG, "bad mesh arguments");
    if (!(youngs > 0) || !(poisson > -1.0 && poisson < 0.5) || !(density > 0))
      return fail(ctx, CC_E_INVALID_ARG, "bad material constants");
    if (n_elems >= (1 << 27)) return fail(ctx, CC_E_INVALID_ARG, "too many elements");
    const int K = dim + 1;
    for (long long k = 0; k < (long long)n_verts * dim; ++k)
      if (!std::isfinite(X[k])) return fail(ctx, CC_E_NONFINITE, "non-finite rest position");
    for (long long k = 0; k < (long long)n_elems * K; ++k)
      if (elems[k] < 0 || elems[k] >= n_verts) return fail(ctx, CC_E_MESH, "element index out of range");
    Mesh* M = new Mesh();
    M->D = dim; M->K = K; M->n = n_verts; M->m = n_elems;
    M->E = youngs; M->nu = poisson; M->rho = density;
    M->mu = youngs / (2.0 * (1.0 + poisson));
    M->lam = youngs * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson)) + M->mu;
    M->X.assign(X, X + (size_t)n_verts * dim);
    M->elems.assign(elems, elems + (size_t)n_elems * K);
    M->fixed.resize(n_verts);
    for (int i = 0; i < n_verts; ++i) M->fixed[i] = is_fixed[i] ? 1 : 0;
    try {
      build_mesh(ctx, *M);
    } catch (...) {
      free_mesh(*M);
      delete M;
      throw;
    }
    ctx->meshes.push_back(M);
    *mesh_id = (int32_t)ctx->meshes.size() - 1;
    return CC_OK;
  });
}

static_assert(CC_MATERIAL_SNH == cc::MAT_SNH && CC_MATERIAL_FCR == cc::MAT_FCR, "material ids");

cc_status cc_mesh_set_material(cc_ctx* ctx, int32_t mesh_id, int32_t model) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (model != CC_MATERIAL_SNH && model != CC_MATERIAL_FCR)
      return fail(ctx, CC_E_INVALID_ARG, "unknown material model");
    const double lam_l = M.E * M.nu / ((1.0 + M.nu) * (1.0 - 2.0 * M.nu));
    M.model = model == CC_MATERIAL_FCR ? cc::MAT_FCR : cc::MAT_SNH;
    M.lam = model == CC_MATERIAL_FCR ? lam_l : lam_l + M.mu;
    return CC_OK;
  });
}

cc_status cc_color(cc_ctx* ctx, int32_t mesh_id, int32_t* colors, int32_t* n_colors) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (colors) std::memcpy(colors, M.colour.data(), M.n * sizeof(int32_t));
    if (n_colors) *n_colors = M.ncol;
    return CC_OK;
  });
}

cc_status cc_layout(cc_ctx* ctx, int32_t mesh_id, int32_t* vperm, int32_t* eperm) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (vperm) std::memcpy(vperm, M.vperm.data(), M.n * sizeof(int32_t));
    if (eperm) std::memcpy(eperm, M.eperm.data(), M.m * sizeof(int32_t));
    return CC_OK;
  });
}

cc_status cc_subspace_upload(cc_ctx* ctx, int32_t mesh_id, const int64_t* ptr, const int32_t* idx,
                             const double* U, double dt_used) {
  (void)dt_used;
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    upload_basis(ctx, M, ptr, idx, U);
    return CC_OK;
  });
}

cc_status cc_subspace_build(cc_ctx* ctx, int32_t mesh_id, int32_t radius, double dt, int32_t quasistatic) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (radius < 0 || (!quasistatic && !(dt > 0))) return fail(ctx, CC_E_INVALID_ARG, "bad basis arguments");
    build_basis(ctx, M, radius, dt, quasistatic);
    return CC_OK;
  });
}

cc_status cc_subspace_build_at(cc_ctx* ctx, int32_t mesh_id, const double* x, int32_t radius, double dt,
                               int32_t quasistatic) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (!x) return fail(ctx, CC_E_INVALID_ARG, "null state buffer");
    if (radius < 0 || (!quasistatic && !(dt > 0))) return fail(ctx, CC_E_INVALID_ARG, "bad basis arguments");
    build_basis(ctx, M, radius, dt, quasistatic, x);
    return CC_OK;
  });
}

cc_status cc_subspace_nnz(cc_ctx* ctx, int32_t mesh_id, int64_t* nnz) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (!M.has_basis) return fail(ctx, CC_E_STATE, "no basis uploaded");
    if (nnz) *nnz = M.snnz;
    return CC_OK;
  });
}

}  // extern "C"

namespace {
// Basis row of internal vertex i in the caller format: caller ids ascending
// and their blocks (float64; a dense basis kept in float32 only is widened).
void basis_row(cc_ctx* ctx, Mesh& M, int i, std::vector<std::pair<int, int64_t>>& row,
               std::vector<double>& blocks) {
  const int DD = M.D * M.D, nf = M.nf;
  hipStream_t s = ctx->stream;
  row.clear();
  if (M.dense) {
    blocks.assign((size_t)nf * DD, 0.0);
    if (M.U_d) {
      HIPC(hipMemcpyAsync(blocks.data(), M.U_d + (size_t)i * nf * DD, blocks.size() * sizeof(double),
                          hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
    } else {
      std::vector<float> bf((size_t)nf * DD);
      HIPC(hipMemcpyAsync(bf.data(), M.U_f + (size_t)i * nf * DD, bf.size() * sizeof(float),
                          hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      for (size_t e = 0; e < bf.size(); ++e) blocks[e] = bf[e];
    }
    for (int p = 0; p < nf; ++p)
      if (M.bvert_h[p] != i) row.push_back({M.vperm[M.bvert_h[p]], p});
  } else {
    int64_t sp[2];
    HIPC(hipMemcpyAsync(sp, M.sptr + i, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    const int64_t len = sp[1] - sp[0];
    std::vector<int> si(len);
    blocks.assign((size_t)len * DD, 0.0);
    if (len > 0) {
      HIPC(hipMemcpyAsync(si.data(), M.sidx + sp[0], len * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(blocks.data(), M.U_d + sp[0] * DD, blocks.size() * sizeof(double),
                          hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
    }
    for (int64_t q = 0; q < len; ++q) row.push_back({M.vperm[si[q]], q});
  }
  std::sort(row.begin(), row.end());
}
}  // namespace

extern "C" {

cc_status cc_subspace_download(cc_ctx* ctx, int32_t mesh_id, int64_t* ptr, int32_t* idx, double* U) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (!M.has_basis) return fail(ctx, CC_E_STATE, "no basis uploaded");
    const int DD = M.D * M.D, nf = M.nf, n = M.n;
    std::vector<std::vector<std::pair<int, int64_t>>> rows(nf);
    std::vector<int64_t> cp(n + 1, 0);
    std::vector<std::pair<int, int64_t>> row;
    std::vector<double> blocks;
    for (int i = 0; i < nf; ++i) {
      basis_row(ctx, M, i, row, blocks);
      cp[M.vperm[i] + 1] = (int64_t)row.size();
    }
    for (int u = 0; u < n; ++u) cp[u + 1] += cp[u];
    if (ptr) std::memcpy(ptr, cp.data(), cp.size() * sizeof(int64_t));
    if (!idx && !U) return CC_OK;
    for (int i = 0; i < nf; ++i) {
      basis_row(ctx, M, i, row, blocks);
      const int u = M.vperm[i];
      for (size_t t = 0; t < row.size(); ++t) {
        if (idx) idx[cp[u] + t] = row[t].first;
        if (U) std::memcpy(&U[(size_t)(cp[u] + t) * DD], &blocks[(size_t)row[t].second * DD], DD * sizeof(double));
      }
    }
    return CC_OK;
  });
}

cc_status cc_subspace_row(cc_ctx* ctx, int32_t mesh_id, int32_t vertex, int64_t* len, int32_t* idx, double* U) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (!M.has_basis) return fail(ctx, CC_E_STATE, "no basis uploaded");
    if (vertex < 0 || vertex >= M.n) return fail(ctx, CC_E_INVALID_ARG, "vertex out of range");
    const int DD = M.D * M.D;
    const int i = M.vinv[vertex];
    if (i >= M.nf) {
      if (len) *len = 0;
      return CC_OK;
    }
    std::vector<std::pair<int, int64_t>> row;
    std::vector<double> blocks;
    basis_row(ctx, M, i, row, blocks);
    if (len) *len = (int64_t)row.size();
    for (size_t t = 0; t < row.size(); ++t) {
      if (idx) idx[t] = row[t].first;
      if (U) std::memcpy(&U[t * DD], &blocks[(size_t)row[t].second * DD], DD * sizeof(double));
    }
    return CC_OK;
  });
}

static cc_status check_params(cc_ctx* ctx, const cc_params* p, const Mesh& M, double dt) {
  if (!p) return fail(ctx, CC_E_INVALID_ARG, "null params");
  if (p->method < 0 || p->method > 2 || p->sweep < 0 || p->sweep > 1 || p->hess_refresh < 0 ||
      p->hess_refresh > 1 || p->precision < 0 || p->precision > 1 || p->max_iters < 0 ||
      p->max_halvings < 0)
    return fail(ctx, CC_E_INVALID_ARG, "bad solver parameters");
  if (!p->quasistatic && !(dt > 0)) return fail(ctx, CC_E_INVALID_ARG, "dt must be positive");
  if (p->method != CC_METHOD_CD && !M.has_basis)
    return fail(ctx, CC_E_STATE, "method needs a basis: call cc_subspace_upload or cc_subspace_build");
  if (p->method != CC_METHOD_CD && p->precision == CC_FP64 && M.has_basis && M.U_d == nullptr)
    return fail(ctx, CC_E_STATE, "the exact basis of this mesh is kept in float32 only: use CC_FP32_MIXED");
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(p->gravity[c])) return fail(ctx, CC_E_NONFINITE, "non-finite gravity");
  if (p->warm_start != 0 && p->warm_start != 1) return fail(ctx, CC_E_INVALID_ARG, "bad warm_start");
  if (p->corotate != 0 && p->corotate != 1) return fail(ctx, CC_E_INVALID_ARG, "bad corotate");
  if (p->warm_start && (!ctx->mlp.set || M.D != 3 || p->quasistatic))
    return fail(ctx, CC_E_STATE, "warm start needs cc_mlp_set and a dynamic 3D mesh");
  return CC_OK;
}

cc_status cc_step(cc_ctx* ctx, int32_t mesh_id, double* x, double* v, const double* x_bc, double dt,
                  const cc_params* params, double tol, int32_t* iters, double* rel_grad) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (!x || !v) return fail(ctx, CC_E_INVALID_ARG, "null state buffer");
    cc_status st = check_params(ctx, params, M, dt);
    if (st != CC_OK) return st;
    if (!(tol >= 0)) return fail(ctx, CC_E_INVALID_ARG, "tol must be >= 0");
    const cc_params& p = *params;
    hipStream_t s = ctx->stream;
    Material mat{};
    mat.mu = M.mu; mat.lam = M.lam; mat.model = M.model;
    mat.w_in = p.quasistatic ? 0.0 : 1.0;
    mat.s_el = p.quasistatic ? 1.0 : dt * dt;
    for (int c = 0; c < 3; ++c) mat.grav[c] = p.gravity[c];
    const double h = p.quasistatic ? 1.0 : dt;
    Stepper S{ctx, M, M.view(), mat, p, s};
    HIPC(hipMemsetAsync(M.bad, 0, sizeof(int), s));
    HIPC(hipMemsetAsync(M.fb, 0, 4 * sizeof(unsigned long long), s));
    cc::launch_predict(S.mv, M.d_vperm, x, v, x_bc, h, p.quasistatic, M.x, M.xt, M.x0, M.bad, s);
    int bad = 0;
    HIPC(hipMemcpyAsync(&bad, M.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (bad) return fail(ctx, CC_E_NONFINITE, "non-finite x, v or x_bc");
    // the convergence test is relative to the larger of the predictor's
    // gradient and the floor (the gravity load's part of it, s_el |m_i g| over
    // free DOFs, or 1e-8 of the elastic force scale)
    const double gstart = std::sqrt(S.grad_norm2(M.x));
    const double g0 = std::max(gstart, load_norm(M, mat));
    const int nd = M.D * M.n;
    double r = 0.0, Ecur = 0.0;
    int k = 0;
    long long halvings = 0, sweep_fb = 0;
    cc_status result = CC_OK;
    int warm = 0;
    // a coloured sweep of CC or JGS2 is taken at its full step only; when
    // that raises E the iteration falls back to a Jacobi sweep
    const bool coloured = p.sweep != CC_SWEEP_JACOBI && p.method != CC_METHOD_CD;
    const int lim0 = coloured ? 0 : p.max_halvings;
    if (g0 > 0) {
      r = gstart / g0;
      if (p.warm_start) {
        // learned proposal at the predictor, kept only if it lowers E
        cc::launch_elem_hess_list(S.mv, p.precision, M.x, mat, mat.s_el, M.estore, s, nullptr, M.m);
        cc::launch_features(S.mv, M.x, M.x0, h, M.E, p.precision, M.estore, mat.s_el, M.ell, M.nptr, M.nidx, M.Xr,
                            M.feat, nullptr,
                            s);
        cc::mlp_forward(ctx->mlp, M.feat, M.nf, M.delta, s);
        // x~ + c + l Delta, then x~ + c alone (c: the last step's
        // correction), each kept only below the start's energy so far
        double Ebest = S.energy(M.x);
        for (int cand = 1; cand <= 2; ++cand) {
          cc::launch_proposal(M.n, M.nf, M.xt, M.corr, M.delta, M.ell, cand == 1 ? 1.0 : 0.0, M.xtrial, s);
          const double Ep = S.energy(M.xtrial);
          if (Ep < Ebest) {
            std::swap(M.x, M.xtrial);
            Ebest = Ep;
            warm = cand;
          }
        }
        if (warm) r = std::sqrt(S.grad_norm2(M.x)) / g0;
        else (void)S.grad_norm2(M.x);  // g at the predictor for the first iteration
      }
      if (p.line_search) Ecur = S.energy(M.x);
      while (r > tol && k < p.max_iters) {
        S.sweep(M.x, M.xtrial, p.method);
        if (p.line_search) {
          const double tau = 1e-12 * std::max(std::fabs(Ecur), 1.0);
          // displacement of this iteration
          cc::launch_axpy(nd, M.xtrial, M.x, -1.0, M.dvec, s);
          double alpha = 1.0, Et = S.energy(M.xtrial);
          int hv = 0;
          while (!(Et <= Ecur + tau) && hv < lim0) {
            alpha *= 0.5;
            ++hv;
            cc::launch_axpy(nd, M.x, M.dvec, alpha, M.xtrial, s);
            Et = S.energy(M.xtrial);
          }
          if (!(Et <= Ecur + tau)) {
            // fallbacks: a Jacobi sweep of the same method (coloured sweeps
            // of CC or JGS2), then coordinate descent, each with the search
            const int nfb = coloured ? 2 : 1;
            for (int f = 0; f < nfb && !(Et <= Ecur + tau); ++f) {
              const bool jac = nfb == 2 && f == 0;
              S.sweep(M.x, M.xtrial, jac ? p.method : CC_METHOD_CD, jac ? CC_SWEEP_JACOBI : -1);
              cc::launch_axpy(nd, M.xtrial, M.x, -1.0, M.dvec, s);
              alpha = 1.0;
              Et = S.energy(M.xtrial);
              hv = 0;
              while (!(Et <= Ecur + tau) && hv < p.max_halvings) {
                alpha *= 0.5;
                ++hv;
                cc::launch_axpy(nd, M.x, M.dvec, alpha, M.xtrial, s);
                Et = S.energy(M.xtrial);
              }
            }
            if (!(Et <= Ecur + tau)) {
              result = CC_STALLED;
              break;
            }
            ++sweep_fb;
          }
          halvings += hv;
          Ecur = Et;
        }
        std::swap(M.x, M.xtrial);
        ++k;
        const double gn = std::sqrt(S.grad_norm2(M.x));
        r = gn / g0;
        if (!std::isfinite(r)) {
          std::swap(M.x, M.xtrial);
          result = CC_STALLED;
          break;
        }
      }
      if (result == CC_OK && r > tol) result = CC_NOT_CONVERGED;
    }
    M.last_E = S.energy(M.x);
    M.last_halvings = halvings;
    M.last_sweep_fb = sweep_fb;
    {
      const double gn = r * g0;
      const double pm = gn / (M.volume * M.n * M.E);
      M.last_paper = p.quasistatic ? pm : pm / dt;
    }
    unsigned long long fbh[4];
    HIPC(hipMemcpyAsync(fbh, M.fb, sizeof(fbh), hipMemcpyDeviceToHost, s));
    cc::launch_finalize(S.mv, M.d_vperm, M.x, M.xt, M.x0, h, p.quasistatic, x, v, s);
    HIPC(hipStreamSynchronize(s));
    ctx->harvest();
    for (int c = 0; c < 3; ++c) M.last_fb[c] = (long long)fbh[c];
    M.last_warm = warm;
    if (iters) *iters = k;
    if (rel_grad) *rel_grad = r;
    return result;
  });
}

cc_status cc_step_info(cc_ctx* ctx, int32_t mesh_id, double* energy, double* paper_residual,
                       int64_t* fallbacks3, int64_t* halvings, int32_t* warm_accepted,
                       int64_t* sweep_fallbacks) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (energy) *energy = M.last_E;
    if (paper_residual) *paper_residual = M.last_paper;
    if (fallbacks3) for (int c = 0; c < 3; ++c) fallbacks3[c] = M.last_fb[c];
    if (halvings) *halvings = M.last_halvings;
    if (warm_accepted) *warm_accepted = M.last_warm;
    if (sweep_fallbacks) *sweep_fallbacks = M.last_sweep_fb;
    return CC_OK;
  });
}

cc_status cc_probe_element(cc_ctx* ctx, int32_t mesh_id, const double* x, int32_t precision, double* ge,
                           double* He) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (!x || !ge || !He || (precision != 0 && precision != 1))
      return fail(ctx, CC_E_INVALID_ARG, "bad probe arguments");
    hipStream_t s = ctx->stream;
    const int K = M.K, NB = K * (K + 1) / 2;
    double* tmp = dalloc<double>((size_t)M.D * M.n + (size_t)NB * M.m * M.D * M.D);
    MeshView mv = M.view();
    Material mat{};
    mat.mu = M.mu; mat.lam = M.lam; mat.model = M.model;
    cc::launch_gather_user(mv, M.d_vinv, x, tmp, s);
    cc::launch_probe_element(mv, precision, x, M.d_vinv, M.d_eperm, tmp, mat, ge, He, s);
    HIPC(hipStreamSynchronize(s));
    dfree(tmp);
    return CC_OK;
  });
}

cc_status cc_probe_sweep(cc_ctx* ctx, int32_t mesh_id, const double* x, const double* x_tilde, double dt,
                         const cc_params* params, double* energy, double* g, double* dx) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (!x || !x_tilde) return fail(ctx, CC_E_INVALID_ARG, "null probe input");
    cc_status st = check_params(ctx, params, M, dt);
    if (st != CC_OK) return st;
    const cc_params& p = *params;
    hipStream_t s = ctx->stream;
    Material mat{};
    mat.mu = M.mu; mat.lam = M.lam; mat.model = M.model;
    mat.w_in = p.quasistatic ? 0.0 : 1.0;
    mat.s_el = p.quasistatic ? 1.0 : dt * dt;
    for (int c = 0; c < 3; ++c) mat.grav[c] = p.gravity[c];
    Stepper S{ctx, M, M.view(), mat, p, s};
    cc::launch_gather_user(S.mv, M.d_vinv, x, M.x, s);
    cc::launch_gather_user(S.mv, M.d_vinv, x_tilde, M.xt, s);
    if (energy) *energy = S.energy(M.x);
    S.gradient_only(M.x);
    if (g) cc::launch_scatter_user(S.mv, M.d_vperm, M.g, g, 1, s);
    if (dx) {
      S.hessian(M.x);
      HIPC(hipMemsetAsync(M.fb, 0, 4 * sizeof(unsigned long long), s));
      if (!cc::launch_cc_prep(S.mv, p.precision, p.method, 0, M.nf, M.hb, M.KL, M.fb, s, M.g, M.dvec))
        cc::launch_cc_update(S.mv, p.precision, p.method, 0, M.nf, M.KL, M.g, M.dvec, 0, s);
      cc::launch_scatter_user(S.mv, M.d_vperm, M.dvec, dx, 1, s);
    }
    HIPC(hipStreamSynchronize(s));
    return CC_OK;
  });
}


// ---- batched stepping ----------------------------------------------------------
static cc::BatchItem make_item(Mesh& M, const Material& mat) {
  cc::BatchItem it{};
  it.mv = M.view();
  it.mat = mat;
  it.x = M.x; it.xtrial = M.xtrial; it.xt = M.xt; it.x0 = M.x0; it.d = M.dvec; it.g = M.g;
  it.estore = M.estore; it.hb = M.hb; it.KL = M.KL;
  it.partials = M.partials;
  it.fb = M.fb;
  it.nptr = M.nptr; it.nidx = M.nidx; it.Xr = M.Xr; it.ell = M.ell; it.youngs = M.E;
  it.ncol = M.ncol;
  for (int c = 0; c <= M.ncol && c <= cc::MAX_COLOURS; ++c) it.coff[c] = M.coff[c];
  for (int c = 0; c < M.ncol && c < cc::MAX_COLOURS; ++c) {
    it.cel_n[c] = M.cel_ptr_h[c + 1] - M.cel_ptr_h[c];
    it.csl_n[c] = M.csl_ptr_h[c + 1] - M.csl_ptr_h[c];
  }
  return it;
}

static cc_status batch_validate(cc_ctx* ctx, int32_t n, const int32_t* mesh_ids, const cc_params* params,
                                double dt, std::vector<Mesh*>& ms) {
  if (n <= 0 || !mesh_ids) return fail(ctx, CC_E_INVALID_ARG, "empty batch");
  ms.clear();
  for (int i = 0; i < n; ++i) {
    Mesh& M = get_mesh(ctx, mesh_ids[i]);
    for (Mesh* o : ms)
      if (o == &M) return fail(ctx, CC_E_INVALID_ARG, "mesh listed twice in a batch");
    if (!ms.empty() && ms[0]->D != M.D) return fail(ctx, CC_E_INVALID_ARG, "batch mixes dimensions");
    if (M.ncol > cc::MAX_COLOURS) return fail(ctx, CC_E_INVALID_ARG, "too many colours for a batch");
    cc_status st = check_params(ctx, params, M, dt);
    if (st != CC_OK) return st;
    ms.push_back(&M);
  }
  return CC_OK;
}

static bool use_dense_band(const cc_ctx* ctx, const Mesh& M, int prec) {
  return M.dense && M.nf > 1 &&
         cc::dense_config(&M.nf, &M.band_w, 1, M.D, prec, ctx->dense_rows, ctx->dense_chunk).tv > 0 &&
         (prec != CC_FP64 || M.U_d != nullptr);
}

static void ctx_batch_hook(void* user, int kid, int begin) {
  cc_ctx* ctx = static_cast<cc_ctx*>(user);
  if (!(ctx->prof_mask & (1 << kid))) return;
  if (begin) {
    ctx->hook_open[kid] = ctx->take_event();
    if (ctx->hook_open[kid]) (void)hipEventRecord(ctx->hook_open[kid], ctx->stream);
    return;
  }
  hipEvent_t a = ctx->hook_open[kid];
  ctx->hook_open[kid] = nullptr;
  if (!a) return;
  hipEvent_t b = ctx->take_event();
  if (!b) return;
  (void)hipEventRecord(b, ctx->stream);
  ctx->pending.push_back({kid, a, b});
}

static cc::BatchPlan* batch_plan_for(cc_ctx* ctx, const std::vector<Mesh*>& ms, const int32_t* ids,
                                     const cc_params& p, double dt, double tol) {
  const int n = (int)ms.size();
  std::vector<double> key = {(double)p.method, (double)p.sweep, (double)p.hess_refresh,
                             (double)p.precision, (double)p.line_search, (double)p.max_iters,
                             (double)p.quasistatic, dt, tol, (double)ctx->batch_lanes,
                             (double)ctx->batch_iters_per_graph, (double)p.corotate,
                             (double)ctx->dense_rows, (double)ctx->dense_chunk};
  int any_fcr = 0;
  for (int i = 0; i < n; ++i) {
    key.push_back((double)(ms[i]->has_basis ? ms[i]->dense : -1));
    any_fcr |= ms[i]->model == cc::MAT_FCR ? 1 : 0;
  }
  key.push_back((double)any_fcr);
  std::vector<int> idv(ids, ids + n);
  if (ctx->plan && ctx->plan_ids == idv && ctx->plan_key == key) return ctx->plan;
  if (ctx->plan) { cc::batch_plan_destroy(ctx->plan); ctx->plan = nullptr; }
  ctx->drop_graph_pairs();
  ctx->hook_on = false;
  std::vector<cc::BatchItem> items(n);
  for (int i = 0; i < n; ++i) {
    Material mat{};
    items[i] = make_item(*ms[i], mat);
    items[i].prep_dense = (p.method != CC_METHOD_CD && use_dense_band(ctx, *ms[i], p.precision)) ? 1 : 0;
    items[i].mv.rot = p.corotate ? ms[i]->rot : nullptr;
  }
  cc::BatchConfig cfg{};
  cfg.D = ms[0]->D; cfg.prec = p.precision; cfg.method = p.method; cfg.sweep = p.sweep;
  cfg.hess_refresh = p.hess_refresh; cfg.line_search = p.line_search; cfg.max_iters = p.max_iters;
  cfg.quasistatic = p.quasistatic; cfg.tol = tol; cfg.h = p.quasistatic ? 1.0 : dt;
  // the legacy null stream cannot be captured: its launches run uncaptured
  // (documented behaviour, not a fallback)
  cfg.G = ctx->batch_lanes;
  cfg.iters_per_graph = ctx->stream != nullptr ? ctx->batch_iters_per_graph : 0;
  cfg.corotate = p.corotate;
  cfg.any_fcr = any_fcr;
  cfg.tv_cap = ctx->dense_rows;
  cfg.chunk = ctx->dense_chunk;
  ctx->plan = cc::batch_plan_create(items.data(), n, cfg, ctx->stream);
  ctx->plan_ids = idv;
  ctx->plan_prev_iters = 0;
  ctx->plan_prev_ls = false;
  ctx->plan_key = key;
  return ctx->plan;
}

// Fallback sweeps of mesh m of the plan after the batched backtracking
// rounds exhausted their halvings along the sweep's displacement (a coloured
// sweep of CC or JGS2 gets none): a Jacobi sweep of the same method for a
// coloured sweep, then a CD sweep, each from x with a host line search along
// it, as in the single-mesh path.
static void batch_host_fallback(cc_ctx* ctx, Mesh& M, cc::BatchItem& it, cc::BatchCtl& c,
                                   const cc_params& p, double tol) {
  hipStream_t s = ctx->stream;
  M.x = it.x;
  M.xtrial = it.xtrial;
  Stepper S{ctx, M, M.view(), it.mat, p, s};
  const int nd = M.D * M.n;
  const double tau = 1e-12 * std::max(std::fabs(c.E_cur), 1.0);
  // a Jacobi sweep of the same method (coloured sweeps of CC or JGS2), then
  // coordinate descent, each with the search
  const int nfb = (p.sweep != CC_SWEEP_JACOBI && p.method != CC_METHOD_CD) ? 2 : 1;
  double alpha = 1.0, Et = 0.0;
  int hv = 0;
  for (int f = 0; f < nfb; ++f) {
    const bool jac = nfb == 2 && f == 0;
    S.sweep(M.x, M.xtrial, jac ? p.method : CC_METHOD_CD, jac ? CC_SWEEP_JACOBI : -1);
    cc::launch_axpy(nd, M.xtrial, M.x, -1.0, M.dvec, s);
    alpha = 1.0;
    Et = S.energy(M.xtrial);
    hv = 0;
    while (!(Et <= c.E_cur + tau) && hv < p.max_halvings) {
      alpha *= 0.5;
      ++hv;
      cc::launch_axpy(nd, M.x, M.dvec, alpha, M.xtrial, s);
      Et = S.energy(M.xtrial);
    }
    if (Et <= c.E_cur + tau) break;
  }
  if (!(Et <= c.E_cur + tau)) {
    c.status = CC_STALLED;
    c.active = 0;
    // g at x must stay valid for a later Jacobi iteration of this mesh
    (void)S.grad_norm2(M.x);
    return;
  }
  M.last_halvings += hv;
  ++M.last_sweep_fb;
  std::swap(M.x, M.xtrial);
  c.E_cur = Et;
  c.iters += 1;
  c.gn2 = S.grad_norm2(M.x);
  c.r = std::sqrt(c.gn2) / c.g0;
  if (!std::isfinite(c.r)) { c.status = CC_STALLED; c.active = 0; }
  else if (c.r <= tol) { c.status = CC_OK; c.active = 0; }
  else if (c.iters >= p.max_iters) { c.status = CC_NOT_CONVERGED; c.active = 0; }
  else c.active = 1;
  it.x = M.x;
  it.xtrial = M.xtrial;
}

cc_status cc_step_batch(cc_ctx* ctx, int32_t n, const int32_t* mesh_ids, double* const* x,
                        double* const* v, const double* const* x_bc, const double* gravity, double dt,
                        const cc_params* params, double tol, int32_t* iters, double* rel_grad,
                        int32_t* status) {
  return guarded(ctx, [&]() -> cc_status {
    std::vector<Mesh*> ms;
    cc_status st = batch_validate(ctx, n, mesh_ids, params, dt, ms);
    if (st != CC_OK) return st;
    if (!x || !v) return fail(ctx, CC_E_INVALID_ARG, "null state arrays");
    for (int i = 0; i < n; ++i)
      if (!x[i] || !v[i]) return fail(ctx, CC_E_INVALID_ARG, "null state buffer");
    if (!(tol >= 0)) return fail(ctx, CC_E_INVALID_ARG, "tol must be >= 0");
    if (gravity)
      for (int k = 0; k < 3 * n; ++k)
        if (!std::isfinite(gravity[k])) return fail(ctx, CC_E_NONFINITE, "non-finite gravity");
    const cc_params& p = *params;
    hipStream_t s = ctx->stream;
    cc::BatchPlan* plan = batch_plan_for(ctx, ms, mesh_ids, p, dt, tol);
    // refresh the per-call fields of every item (buffers, material, caller pointers)
    std::vector<cc::BatchItem> items(n);
    for (int i = 0; i < n; ++i) {
      Mesh& M = *ms[i];
      Material mat{};
      mat.mu = M.mu; mat.lam = M.lam; mat.model = M.model;
      mat.w_in = p.quasistatic ? 0.0 : 1.0;
      mat.s_el = p.quasistatic ? 1.0 : dt * dt;
      for (int c = 0; c < 3; ++c) mat.grav[c] = gravity ? gravity[3 * i + c] : p.gravity[c];
      items[i] = make_item(M, mat);
      items[i].prep_dense = (p.method != CC_METHOD_CD && use_dense_band(ctx, M, p.precision)) ? 1 : 0;
      items[i].mv.rot = p.corotate ? M.rot : nullptr;
      items[i].feat_off = 0;
      for (int q = 0; q < i; ++q) items[i].feat_off += ms[q]->nf;
      items[i].xu = x[i];
      items[i].vu = v[i];
      items[i].xbc = x_bc ? x_bc[i] : nullptr;
      items[i].load = load_norm(M, mat);
      M.last_halvings = 0;          // fallback counters are cleared by batch_begin
      M.last_sweep_fb = 0;
    }
    cc::BatchItem* items_d = cc::batch_items_dev(plan);
    cc::BatchCtl* ctl_d = cc::batch_ctl_dev(plan);
    HIPC(hipMemcpyAsync(items_d, items.data(), n * sizeof(cc::BatchItem), hipMemcpyHostToDevice, s));
    const bool want_hook = ctx->prof_mask != 0;
    if (want_hook != ctx->hook_on) {
      cc::batch_set_hook(plan, want_hook ? ctx_batch_hook : nullptr, ctx);  // drops the graph
      ctx->drop_graph_pairs();
      ctx->hook_on = want_hook;
    }
    cc::batch_begin(plan, s);
    if (p.warm_start) {
      size_t rows = 0;
      for (int i = 0; i < n; ++i) rows += ms[i]->nf;
      if (rows > ctx->bcap) {
        dfree(ctx->bfeat);
        dfree(ctx->bdelta);
        ctx->bfeat = dalloc<float>(rows * 16);
        ctx->bdelta = dalloc<float>(rows * 3);
        ctx->bcap = rows;
      }
      cc::batch_warm_start(plan, ctx->mlp, ctx->bfeat, ctx->bdelta, (int)rows, s);
    }
    std::vector<cc::BatchCtl> ctl(n);
    const int k = std::max(1, ctx->batch_iters_per_graph);
    auto pull_ctl = [&]() {
      HIPC(hipMemcpyAsync(ctx->pinned, ctl_d, n * sizeof(cc::BatchCtl), hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      std::memcpy(ctl.data(), ctx->pinned, n * sizeof(cc::BatchCtl));
    };
    // the pinned buffer may be read by a copy still in flight: wait first
    auto push_ctl = [&]() {
      HIPC(hipStreamSynchronize(s));
      std::memcpy(ctx->pinned, ctl.data(), n * sizeof(cc::BatchCtl));
      HIPC(hipMemcpyAsync(ctl_d, ctx->pinned, n * sizeof(cc::BatchCtl), hipMemcpyHostToDevice, s));
    };
    if ((size_t)n * sizeof(cc::BatchCtl) > 64 * 1024)
      return fail(ctx, CC_E_INVALID_ARG, "batch too large");
    // The first round is queued without reading the control blocks back:
    // meshes that converged at the predictor, or whose input is not finite,
    // are already inactive on the device and skip it; the read after the
    // round reports them.
    for (auto& c : ctl) c.active = 1;
    long long guard = 0;
    int queue = ctx->plan_prev_ls ? k : std::min(std::max(ctx->plan_prev_iters, k), 16);   // first round
    int backtracks = 0;
    bool first = true;
    while (true) {
      bool any = false;
      for (auto& c : ctl) any = any || c.active;
      if (!any) break;
      HIPC(cc::batch_iterate(plan, (queue + k - 1) / k * k, s));
      queue = k;
      if (!cc::batch_has_graph(plan) && !ctx->graph_pairs.empty()) ctx->drop_graph_pairs();
      pull_ctl();
      if (first) {
        first = false;
        bool bad = false;
        for (int i = 0; i < n; ++i) bad = bad || ctl[i].bad;
        if (bad) {
          // the other meshes may have run the round: keep the host's view of
          // their position buffers in step with the device before failing
          HIPC(hipMemcpyAsync(items.data(), items_d, n * sizeof(cc::BatchItem), hipMemcpyDeviceToHost, s));
          HIPC(hipStreamSynchronize(s));
          for (int i = 0; i < n; ++i) {
            ms[i]->x = items[i].x;
            ms[i]->xtrial = items[i].xtrial;
          }
          return fail(ctx, CC_E_NONFINITE, "non-finite x, v or x_bc in batch");
        }
      }
      ctx->harvest();
      if (cc::batch_has_graph(plan)) ctx->harvest_graph();
      bool host = false;
      for (auto& c : ctl) host = host || c.needs_host;
      if (host) {
        ++backtracks;
        // Meshes whose energy rose at the full step backtrack together: a
        // round evaluates the next eight halvings of every searching mesh at
        // once and takes the first that does not raise E.  Two rounds are
        // queued per read-back; a mesh that has decided skips the second.
        // A coloured sweep of CC or JGS2 takes no halvings: its meshes go
        // straight to the host fallback, which starts with a Jacobi sweep.
        const bool coloured = p.sweep != CC_SWEEP_JACOBI && p.method != CC_METHOD_CD;
        const int lim0 = coloured ? 0 : p.max_halvings;
        std::vector<int> was_active(n);
        for (int i = 0; i < n; ++i) {
          was_active[i] = ctl[i].active;
          ctl[i].active = ctl[i].needs_host;
          ctl[i].alpha = 0.5;
          ctl[i].halvings = 1;
          ctl[i].ls = ctl[i].needs_host && lim0 < 1 ? 2 : 0;
          if (ctl[i].ls == 2) ctl[i].active = 0;
        }
        push_ctl();
        for (int r = 0;; ++r) {
          bool searching = false;
          for (auto& c : ctl) searching = searching || c.active;
          if (!searching) break;
          // every round decides a mesh or takes it eight halvings further
          if (r > lim0 + 1)
            throw ApiError{CC_E_HIP, "batched line search did not finish"};
          for (int q = 0; q < 2; ++q)
            if (!cc::batch_ls_round(plan, r == 0 && q == 0, lim0, s))
              throw ApiError{CC_E_HIP, "no device memory for the batched line search"};
          pull_ctl();
        }
        // accepted steps: gradient at the new x and the convergence test
        bool any_acc = false;
        for (int i = 0; i < n; ++i) {
          ctl[i].active = ctl[i].needs_host && ctl[i].ls == 1;
          any_acc = any_acc || ctl[i].active;
          if (ctl[i].active) ms[i]->last_halvings += ctl[i].halvings;
        }
        if (any_acc) {
          push_ctl();
          cc::batch_gradient_converge(plan, s);
          pull_ctl();
        }
        // exhausted halvings: the fallback sweeps on the host,
        // which needs the meshes' current buffer roles from the device
        bool any_cd = false;
        for (int i = 0; i < n; ++i) any_cd = any_cd || (ctl[i].needs_host && ctl[i].ls == 2);
        if (any_cd) {
          HIPC(hipMemcpyAsync(items.data(), items_d, n * sizeof(cc::BatchItem), hipMemcpyDeviceToHost, s));
          HIPC(hipStreamSynchronize(s));
        }
        for (int i = 0; i < n; ++i) {
          if (ctl[i].needs_host && ctl[i].ls == 2) {
            batch_host_fallback(ctx, *ms[i], items[i], ctl[i], p, tol);
            HIPC(hipMemcpyAsync(items_d + i, &items[i], sizeof(cc::BatchItem), hipMemcpyHostToDevice, s));
            HIPC(hipStreamSynchronize(s));   // items[i] is pageable host memory
          }
          if (!ctl[i].needs_host) ctl[i].active = was_active[i];
          ctl[i].needs_host = 0;
        }
        push_ctl();   // stream-ordered before the next replay and read-back
      }
      if (++guard > (long long)p.max_iters + 16) break;  // every replay advances every active mesh
    }
    cc::batch_finish(plan, s);
    ctx->plan_prev_iters = 0;
    for (auto& c : ctl) ctx->plan_prev_iters = std::max(ctx->plan_prev_iters, c.iters);
    ctx->plan_prev_ls = 2 * backtracks >= std::max(ctx->plan_prev_iters, 1);
    HIPC(hipMemcpyAsync(items.data(), items_d, n * sizeof(cc::BatchItem), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    ctx->harvest();
    cc_status worst = CC_OK;
    for (int i = 0; i < n; ++i) {
      Mesh& M = *ms[i];
      M.x = items[i].x;          // keep the mesh's own buffer roles in step with the device
      M.xtrial = items[i].xtrial;
      int stt = ctl[i].status == -100 ? CC_NOT_CONVERGED : ctl[i].status;
      if (iters) iters[i] = ctl[i].iters;
      if (rel_grad) rel_grad[i] = ctl[i].r;
      if (status) status[i] = stt;
      M.last_E = ctl[i].E_cur;
      {  // the paper's normalised residual |g| / (V n E), divided by h when dynamic
        const double pm = ctl[i].r * ctl[i].g0 / (M.volume * M.n * M.E);
        M.last_paper = p.quasistatic ? pm : pm / dt;
      }
      M.last_warm = ctl[i].warm;
      if (stt < 0 ? (worst >= 0 || stt < worst) : (worst >= 0 && stt > worst)) worst = stt;
    }
    if (worst >= 0 && worst < CC_GRAPH_FALLBACK && cc::batch_capture_failed(plan)) {
      ctx->err = "graph capture failed on this stream: the iterations ran as direct launches";
      worst = CC_GRAPH_FALLBACK;
    }
    return worst;
  });
}

cc_status cc_batch_tuning(cc_ctx* ctx, int32_t lanes, int32_t iters_per_graph) {
  return guarded(ctx, [&]() -> cc_status {
    if ((lanes != 16 && lanes != 32 && lanes != 64) || iters_per_graph < 0 || iters_per_graph > 64)
      return fail(ctx, CC_E_INVALID_ARG, "lanes must be 16, 32 or 64; iters_per_graph 0..64");
    ctx->batch_lanes = lanes;
    ctx->batch_iters_per_graph = iters_per_graph;
    return CC_OK;
  });
}

cc_status cc_dense_tuning(cc_ctx* ctx, int32_t rows_per_workgroup, int32_t chunk) {
  return guarded(ctx, [&]() -> cc_status {
    if (rows_per_workgroup < 0 || rows_per_workgroup > 4)
      return fail(ctx, CC_E_INVALID_ARG, "rows per workgroup must be 0 (automatic), 1, 2, 3 or 4");
    if (chunk != 0 && chunk != 128 && chunk != 256 && chunk != 512)
      return fail(ctx, CC_E_INVALID_ARG, "chunk must be 0 (automatic), 128, 256 or 512");
    ctx->dense_rows = rows_per_workgroup;
    ctx->dense_chunk = chunk;
    return CC_OK;
  });
}

cc_status cc_autotune_batch(cc_ctx* ctx, int32_t n, const int32_t* mesh_ids, const cc_params* params,
                            int32_t* lanes_out, double* ms_out) {
  return guarded(ctx, [&]() -> cc_status {
    std::vector<Mesh*> ms;
    const double dt = 1.0 / 60.0;
    cc_status st = batch_validate(ctx, n, mesh_ids, params, dt, ms);
    if (st != CC_OK) return st;
    cc::BatchPlan* plan = batch_plan_for(ctx, ms, mesh_ids, *params, dt, 0.0);
    std::vector<cc::BatchItem> items(n);
    for (int i = 0; i < n; ++i) {
      Material mat{};
      mat.mu = ms[i]->mu; mat.lam = ms[i]->lam; mat.model = ms[i]->model;
      items[i] = make_item(*ms[i], mat);
      items[i].prep_dense = (params->method != CC_METHOD_CD && use_dense_band(ctx, *ms[i], params->precision)) ? 1 : 0;
      items[i].mv.rot = params->corotate ? ms[i]->rot : nullptr;
    }
    HIPC(hipMemcpyAsync(cc::batch_items_dev(plan), items.data(), n * sizeof(cc::BatchItem),
                        hipMemcpyHostToDevice, ctx->stream));
    // every mesh active, timing only (K, L and d are scratch)
    std::vector<cc::BatchCtl> ctl(n);
    for (auto& c : ctl) { c = cc::BatchCtl{}; c.active = 1; }
    HIPC(hipMemcpyAsync(cc::batch_ctl_dev(plan), ctl.data(), n * sizeof(cc::BatchCtl),
                        hipMemcpyHostToDevice, ctx->stream));
    const int choices[3] = {16, 32, 64};
    double best = 1e300;
    int bestG = 16;
    for (int c = 0; c < 3; ++c) {
      const float t = cc::batch_time_prep_update(plan, choices[c], 5, ctx->stream);
      if (ms_out) ms_out[c] = t;
      if (t < best) { best = t; bestG = choices[c]; }
    }
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->batch_lanes = bestG;
    cc::batch_plan_destroy(ctx->plan);
    ctx->plan = nullptr;
    ctx->plan_ids.clear();
    if (lanes_out) *lanes_out = bestG;
    return CC_OK;
  });
}


// ---- learned warm start -------------------------------------------------------
static void mlp_alloc(cc_ctx* ctx) {
  cc::MlpState& q = ctx->mlp;
  if (q.W) return;
  q.W = dalloc<float>(cc::MLP_NPARAM);
  q.m = dalloc<float>(cc::MLP_NPARAM);
  q.v = dalloc<float>(cc::MLP_NPARAM);
  q.grad = dalloc<float>(cc::MLP_NPARAM);
  q.part = dalloc<float>(cc::MLP_PART_FLOATS);
  q.lpart = dalloc<float>(cc::MLP_LPART_FLOATS);
  q.loss = dalloc<float>(1);
  q.W1b = dalloc<uint16_t>(cc::MLP_IN_PAD * cc::MLP_HID);
  q.W2b = dalloc<uint16_t>(cc::MLP_HID * cc::MLP_HID);
  q.W3b = dalloc<uint16_t>(cc::MLP_HID * cc::MLP_OUT);
  q.mean = dalloc<float>(cc::MLP_IN);
  q.istd = dalloc<float>(cc::MLP_IN);
}

static cc_status mlp_ready(cc_ctx* ctx) {
  if (!ctx->mlp.set) return fail(ctx, CC_E_STATE, "no network: call cc_mlp_set first");
  return CC_OK;
}

cc_status cc_mlp_set(cc_ctx* ctx, const float* params, const float* mean, const float* istd) {
  return guarded(ctx, [&]() -> cc_status {
    if (!params) return fail(ctx, CC_E_INVALID_ARG, "null parameters");
    for (int k = 0; k < cc::MLP_NPARAM; ++k)
      if (!std::isfinite(params[k])) return fail(ctx, CC_E_NONFINITE, "non-finite parameter");
    mlp_alloc(ctx);
    cc::MlpState& q = ctx->mlp;
    hipStream_t s = ctx->stream;
    HIPC(hipMemcpyAsync(q.W, params, cc::MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    HIPC(hipMemsetAsync(q.m, 0, cc::MLP_NPARAM * sizeof(float), s));
    HIPC(hipMemsetAsync(q.v, 0, cc::MLP_NPARAM * sizeof(float), s));
    std::vector<float> mu(cc::MLP_IN, 0.f), is(cc::MLP_IN, 1.f);
    if (mean) mu.assign(mean, mean + cc::MLP_IN);
    if (istd) is.assign(istd, istd + cc::MLP_IN);
    HIPC(hipMemcpyAsync(q.mean, mu.data(), cc::MLP_IN * sizeof(float), hipMemcpyHostToDevice, s));
    HIPC(hipMemcpyAsync(q.istd, is.data(), cc::MLP_IN * sizeof(float), hipMemcpyHostToDevice, s));
    cc::mlp_refresh_bf16(q, s);
    HIPC(hipStreamSynchronize(s));
    q.t = 0;
    q.set = true;
    return CC_OK;
  });
}

cc_status cc_mlp_get(cc_ctx* ctx, float* params, float* mean, float* istd) {
  return guarded(ctx, [&]() -> cc_status {
    cc_status st = mlp_ready(ctx);
    if (st != CC_OK) return st;
    cc::MlpState& q = ctx->mlp;
    hipStream_t s = ctx->stream;
    if (params) HIPC(hipMemcpyAsync(params, q.W, cc::MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
    if (mean) HIPC(hipMemcpyAsync(mean, q.mean, cc::MLP_IN * sizeof(float), hipMemcpyDeviceToHost, s));
    if (istd) HIPC(hipMemcpyAsync(istd, q.istd, cc::MLP_IN * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return CC_OK;
  });
}

cc_status cc_mlp_norm_from_data(cc_ctx* ctx, const float* X, int32_t N) {
  return guarded(ctx, [&]() -> cc_status {
    cc_status st = mlp_ready(ctx);
    if (st != CC_OK) return st;
    if (!X || N <= 0) return fail(ctx, CC_E_INVALID_ARG, "empty feature set");
    cc::mlp_stats(ctx->mlp, X, N, ctx->stream);
    HIPC(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

cc_status cc_mlp_features(cc_ctx* ctx, int32_t mesh_id, const double* x, const double* v, const double* x_bc,
                          double dt, float* feat, double* x_base, double* ell) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (M.D != 3) return fail(ctx, CC_E_INVALID_ARG, "features are defined for 3D meshes");
    if (!x || !v || !feat || !(dt > 0)) return fail(ctx, CC_E_INVALID_ARG, "bad feature arguments");
    hipStream_t s = ctx->stream;
    MeshView mv = M.view();
    HIPC(hipMemsetAsync(M.bad, 0, sizeof(int), s));
    cc::launch_predict(mv, M.d_vperm, x, v, x_bc, dt, 0, M.x, M.xt, M.x0, M.bad, s);
    cc::Material mat{};
    mat.mu = M.mu; mat.lam = M.lam; mat.model = M.model;
    mat.w_in = 1.0;
    mat.s_el = dt * dt;
    cc::launch_elem_hess_list(mv, 0, M.x, mat, mat.s_el, M.estore, s, nullptr, M.m);
    cc::launch_features(mv, M.x, M.x0, dt, M.E, 0, M.estore, mat.s_el, M.ell, M.nptr, M.nidx, M.Xr, feat, M.frank,
                        s);
    if (x_base) cc::launch_base_user(mv, M.d_vperm, M.x, x_base, s);
    if (ell) *ell = M.ell;
    int bad = 0;
    HIPC(hipMemcpyAsync(&bad, M.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (bad) return fail(ctx, CC_E_NONFINITE, "non-finite x, v or x_bc");
    return CC_OK;
  });
}

cc_status cc_mlp_forward(cc_ctx* ctx, const float* X, int32_t B, float* Y) {
  return guarded(ctx, [&]() -> cc_status {
    cc_status st = mlp_ready(ctx);
    if (st != CC_OK) return st;
    if (B < 0 || (B > 0 && (!X || !Y))) return fail(ctx, CC_E_INVALID_ARG, "bad forward arguments");
    cc::mlp_forward(ctx->mlp, X, B, Y, ctx->stream);
    HIPC(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

cc_status cc_mlp_gradient(cc_ctx* ctx, const float* X, const float* T, const int32_t* idx, int32_t B,
                          float* grad, float* loss) {
  return guarded(ctx, [&]() -> cc_status {
    cc_status st = mlp_ready(ctx);
    if (st != CC_OK) return st;
    if (B <= 0 || !X || !T || !idx) return fail(ctx, CC_E_INVALID_ARG, "bad gradient arguments");
    cc::MlpState& q = ctx->mlp;
    cc::mlp_gradient(q, X, T, idx, B, grad ? grad : q.grad, q.loss, ctx->stream);
    float l = 0.f;
    HIPC(hipMemcpyAsync(&l, q.loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    if (loss) *loss = l;
    return CC_OK;
  });
}

cc_status cc_mlp_gradient_noalloc(cc_ctx* ctx, const float* X, const float* T, const int32_t* idx,
                                  int32_t B, float* grad, float* loss) {
  return guarded(ctx, [&]() -> cc_status {
    cc_status st = mlp_ready(ctx);
    if (st != CC_OK) return st;
    if (!X || !T || !idx || !grad) return fail(ctx, CC_E_INVALID_ARG, "null gradient argument");
    if (B < 1 || B > CC_MLP_NOALLOC_MAX_ROWS)
      return fail(ctx, CC_E_INVALID_ARG, "cc_mlp_gradient_noalloc: B must be in 1.." +
                                             std::to_string(CC_MLP_NOALLOC_MAX_ROWS));
    float* base = scratch_of(ctx->device);
    if (!base) return fail(ctx, CC_E_STATE, "scratch address of this device not resolved");
    float* part = base;
    float* lpart = base + cc::MLP_PART_FLOATS;
    float* lslot = lpart + cc::MLP_LPART_FLOATS;
    cc::mlp_gradient_into(ctx->mlp, X, T, idx, B, grad, loss ? loss : lslot, part, lpart, ctx->stream);
    HIPC(hipGetLastError());
    return CC_OK;
  });
}

cc_status cc_mlp_adam(cc_ctx* ctx, const float* grad, float lr) {
  return guarded(ctx, [&]() -> cc_status {
    cc_status st = mlp_ready(ctx);
    if (st != CC_OK) return st;
    if (!grad || !(lr > 0)) return fail(ctx, CC_E_INVALID_ARG, "bad Adam arguments");
    cc::mlp_adam(ctx->mlp, grad, lr, ctx->stream);
    HIPC(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

cc_status cc_mlp_train_step(cc_ctx* ctx, const float* X, const float* T, const int32_t* idx, int32_t B,
                            float lr, float* loss) {
  return guarded(ctx, [&]() -> cc_status {
    cc_status st = mlp_ready(ctx);
    if (st != CC_OK) return st;
    if (B <= 0 || !X || !T || !idx || !(lr > 0)) return fail(ctx, CC_E_INVALID_ARG, "bad training arguments");
    cc::MlpState& q = ctx->mlp;
    cc::mlp_gradient(q, X, T, idx, B, q.grad, q.loss, ctx->stream);
    cc::mlp_adam(q, q.grad, lr, ctx->stream);
    if (loss) {
      HIPC(hipMemcpyAsync(loss, q.loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
      HIPC(hipStreamSynchronize(ctx->stream));
    }
    return CC_OK;
  });
}


cc_status cc_mlp_targets(cc_ctx* ctx, int32_t mesh_id, const double* x_new, const double* x_base, float* T) {
  return guarded(ctx, [&]() -> cc_status {
    Mesh& M = get_mesh(ctx, mesh_id);
    if (M.D != 3 || !x_new || !x_base || !T) return fail(ctx, CC_E_INVALID_ARG, "bad target arguments");
    cc::launch_targets(M.view(), x_new, x_base, M.ell, M.frank, T, ctx->stream);
    HIPC(hipStreamSynchronize(ctx->stream));
    return CC_OK;
  });
}

}  // extern "C"
