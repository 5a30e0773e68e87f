/*
 * ccgpu -- Coordinate Condensation on AMD MI355X (gfx950), C ABI.
 *
 * The library advances implicit-Euler elastodynamics by minimising the step
 * energy E(x) = 1/2 (x - x~)^T M (x - x~) + h^2 Psi(x)  (paper: Background,
 * "Optimization-Based Integration") with Coordinate Condensation: per-vertex
 * local solves augmented by a precomputed perturbation subspace and condensed
 * by a Schur complement (paper: Method, Eqs. displacement, block, update and
 * schur; Algorithm 1).  Psi is the stable neo-Hookean energy
 * mu/2(|F|^2 - d) - mu(J-1) + lambda/2 (J-1)^2 with lambda = lambda_L + mu,
 * integrated over linear simplices (triangles in 2D, tetrahedra in 3D) with
 * element-wise PSD projection of d2Psi/dF2.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - Every entry point returns a cc_status.  0 is success, positive values are
 *   warnings whose outputs are valid, negative values are errors.  No C++
 *   exception crosses the ABI.  cc_last_error() describes the last failure.
 * - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *   memory on the context's device.  The caller owns every pointer it passes;
 *   uploads are deep-copied into library-owned device memory, released by
 *   cc_destroy.  No pointer passed in is retained after the call returns.
 * - Positions and velocities are float64, row-major (n x dim), in the
 *   caller's vertex order.  Element arrays are int32, row-major
 *   (n_elems x (dim+1)), in the caller's element order.
 * - All device work is ordered on the stream given to cc_create.  Calls that
 *   return host results synchronise that stream before returning.
 * - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef CCGPU_H
#define CCGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cc_status;

#define CC_OK                0
#define CC_NOT_CONVERGED     1   /* iteration cap reached; outputs = last iterate   */
#define CC_STALLED           2   /* line search and its CD fallback both failed    */
#define CC_GRAPH_FALLBACK    3   /* cc_step_batch: graph capture failed on the stream,
                                    the iterations ran as direct launches (outputs valid) */
#define CC_E_INVALID_ARG    -1
#define CC_E_MESH           -2   /* bad index or non-positive rest volume           */
#define CC_E_SUBSPACE       -3   /* unsorted / out-of-range / Dirichlet basis index */
#define CC_E_HIP            -4   /* a HIP runtime call failed                       */
#define CC_E_NONFINITE      -5   /* NaN/Inf in inputs                               */
#define CC_E_STATE          -6   /* wrong call order (e.g. step before subspace)    */
#define CC_E_NO_DEVICE      -7

/* method */
#define CC_METHOD_CD    0   /* plain block coordinate descent: dx_i = -H_ii^{-1} g_i   */
#define CC_METHOD_CC    1   /* Coordinate Condensation (Method, Eq. update/schur)       */
#define CC_METHOD_JGS2  2   /* printed JGS2 form (Background, JGS2 subsection)          */
/* sweep */
#define CC_SWEEP_JACOBI     0   /* Algorithm 1: all vertices from one snapshot          */
#define CC_SWEEP_COLORED_GS 1   /* one graph colour at a time, latest positions         */
/* hess_refresh (coloured sweep only) */
#define CC_HESS_PER_COLOR 0     /* g and H re-evaluated before every colour             */
#define CC_HESS_PER_SWEEP 1     /* H evaluated once per sweep, g before every colour    */
/* precision */
#define CC_FP64        0
#define CC_FP32_MIXED  1        /* FP32 element Hessians, assembly and local solves;
                                   FP64 positions, gradient, energy and norms           */

typedef struct cc_ctx cc_ctx;

typedef struct {
  int32_t method;         /* CC_METHOD_*                                               */
  int32_t sweep;          /* CC_SWEEP_*                                                */
  int32_t hess_refresh;   /* CC_HESS_*                                                 */
  int32_t precision;      /* CC_FP64 / CC_FP32_MIXED                                   */
  int32_t line_search;    /* 0 off (Algorithm 1), 1 global backtracking along the
                             iteration's displacement (Results, basis-quality study):
                             alpha halved while E rises above E + 1e-12 max(|E|, 1);
                             when max_halvings do not find a step, a coordinate-
                             descent sweep with the same search; none found:
                             CC_STALLED.  A coloured sweep of CC or JGS2 is taken at
                             its full step only: if that raises E, the iteration
                             takes a Jacobi sweep of the same method with the
                             search, then the coordinate-descent fallback            */
  int32_t max_iters;      /* iteration cap (>= 0)                                      */
  int32_t max_halvings;   /* line-search halvings (>= 0)                               */
  int32_t quasistatic;    /* 1: E = Psi - m g.x (no inertia, no h^2)                   */
  int32_t warm_start;     /* 0 none, 1 learned proposal set by cc_mlp_set              */
  double  gravity[3];     /* gravitational acceleration; dim 2 uses the first two      */
  int32_t corotate;       /* 1: rotate every basis block by its vertex's rotation,
                             U_i[j] -> R_j U_i[j], with R_j the polar rotation of the
                             displacement of j's mesh neighbourhood, re-estimated
                             wherever g and H are (Method, Accounting for Large
                             Deformations, Eq. rotation); 0 off                         */
} cc_params;

/* Fill *p with defaults: CC, Jacobi, per-colour Hessians, FP64, line search on,
   10000 iterations, 20 halvings, dynamic, no warm start, gravity 0, no
   corotation. */
void cc_params_default(cc_params* p);

/* Create a context on HIP device `device`, ordering work on `hip_stream`
   (a hipStream_t, or NULL for the null stream).  *out receives the context. */
cc_status cc_create(int32_t device, void* hip_stream, cc_ctx** out);
void      cc_destroy(cc_ctx* ctx);
/* Message of the last failure; owned by the context, valid until the next call. */
const char* cc_last_error(const cc_ctx* ctx);

/* Upload a mesh (host arrays).  Rest data (shape gradients, volumes, lumped
   masses rho*sum V_e/(d+1)), the greedy colouring and the colour-sorted
   layouts are built here.  Elements must be positively oriented
   (det [X1-X0 ... Xd-X0] > 0), otherwise CC_E_MESH.  Repeated uploads create
   further meshes (for batched stepping); *mesh_id receives the new id. */
cc_status cc_mesh_upload(cc_ctx* ctx, int32_t dim, int32_t n_verts, const double* X,
                         int32_t n_elems, const int32_t* elems, const uint8_t* is_fixed,
                         double youngs, double poisson, double density, int32_t* mesh_id);

/* Material models (Results, Implementation Details names Fixed Corotational;
   stable neo-Hookean is the default).  mu = E/(2(1+nu)), lambda_L =
   E nu/((1+nu)(1-2nu)):
     CC_MATERIAL_SNH  Psi = mu/2(|F|^2 - d) - mu(J-1) + lambda/2 (J-1)^2,
                      lambda = lambda_L + mu;
     CC_MATERIAL_FCR  Psi = mu |F - R|^2 + lambda/2 (J-1)^2, lambda = lambda_L,
                      R the rotation nearest to F.
   Both have the same rest linearisation, so a basis built for one serves the
   other.  Hessians are projected to the PSD cone element by element. */
#define CC_MATERIAL_SNH 0
#define CC_MATERIAL_FCR 1

/* Select the material model of a mesh (default CC_MATERIAL_SNH); E and nu are
   those given at upload.  Takes effect from the next step or probe.  An
   unknown model gives CC_E_INVALID_ARG and leaves the mesh unchanged. */
cc_status cc_mesh_set_material(cc_ctx* ctx, int32_t mesh_id, int32_t model);

/* Greedy colouring of the free-vertex graph (edge iff two free vertices share
   an element), visiting vertices in increasing id and taking the smallest
   colour unused by coloured neighbours.  colors (host, n_verts) receives the
   colour of each vertex, -1 for Dirichlet vertices. */
cc_status cc_color(cc_ctx* ctx, int32_t mesh_id, int32_t* colors, int32_t* n_colors);

/* Internal orderings (host outputs): vperm[new] = caller vertex id, sorted by
   (colour, id) with Dirichlet vertices last; eperm[new] = caller element id,
   sorted by (smallest caller id among the element's free vertices, id) with
   all-Dirichlet elements last. */
cc_status cc_layout(cc_ctx* ctx, int32_t mesh_id, int32_t* vperm, int32_t* eperm);

/* Upload the per-vertex perturbation basis U_i = -H_CC^{-1} H_Ci (Background,
   JGS2 subsection; Method, Coordinate Condensation), host CSR in caller vertex
   ids: ptr (n_verts+1, int64), idx (ptr[n], int32, strictly ascending per
   row, free vertices other than the row's vertex), U (ptr[n] x dim x dim,
   float64, row-major; block k maps a displacement of vertex i to that of
   vertex idx[k]).  Rows of Dirichlet vertices must be empty.  Violations give
   CC_E_SUBSPACE.  dt_used records the step size the basis was built for. */
cc_status cc_subspace_upload(cc_ctx* ctx, int32_t mesh_id, const int64_t* ptr,
                             const int32_t* idx, const double* U, double dt_used);

/* Build the basis in the library from the rest Hessian of the step energy
   (M + h^2 K(X), or K(X) when quasistatic):
   radius > 0: patch basis, support = free vertices within `radius` hops,
               everything outside the patch held, U_i = -H[C,C]^{-1} H[C,i];
   radius = 0: exact basis over every other free vertex, U_i[j] =
               Z_ji Z_ii^{-1} with Z = H^{-1}, formed on the GPU in float64
               column block by column block from the block-tridiagonal
               factorisation of H in breadth-first level order (levels of
               n unknowns: O(N^2 n) work and O(N n) temporary memory for N
               free unknowns).  Stores n_free^2 blocks in float32, plus a
               float64 copy when that takes at most 4 GiB (larger bases
               then step in CC_FP32_MIXED only; CC_FP64 gives CC_E_STATE).
   The rest Hessian is evaluated by the library's own GPU kernels in FP64;
   the patch solves run on the host. */
cc_status cc_subspace_build(cc_ctx* ctx, int32_t mesh_id, int32_t radius, double dt,
                            int32_t quasistatic);

/* The same bases built from the projected step Hessian at the state x instead
   of at rest: x is a device float64 buffer, n_verts x dim, caller vertex
   order (Dirichlet rows are the positions their elements see).  This is the
   reconstruction of the paper's restarted variant (Results, Subspace
   Quality).  The Hessian must be positive definite on the free degrees of
   freedom (CC_E_SUBSPACE otherwise; the previous basis is then kept). */
cc_status cc_subspace_build_at(cc_ctx* ctx, int32_t mesh_id, const double* x, int32_t radius,
                               double dt, int32_t quasistatic);

/* Number of basis blocks of a mesh (*nnz), and a copy of the basis in the
   upload format (host outputs sized n_verts+1, nnz, nnz*dim*dim). */
cc_status cc_subspace_nnz(cc_ctx* ctx, int32_t mesh_id, int64_t* nnz);
cc_status cc_subspace_download(cc_ctx* ctx, int32_t mesh_id, int64_t* ptr, int32_t* idx,
                               double* U);
/* One basis row in the upload format: the row of caller vertex `vertex`
   (*len entries, caller ids ascending in idx, blocks in U as float64; a basis
   kept in float32 only is widened).  idx and U must hold n_free - 1 entries
   for an exact basis; any output may be NULL.  Dirichlet rows are empty. */
cc_status cc_subspace_row(cc_ctx* ctx, int32_t mesh_id, int32_t vertex, int64_t* len, int32_t* idx,
                          double* U);

/* One implicit time step of mesh `mesh_id`.
   x, v: device (n_verts x dim) float64, read as x^t, v^t and overwritten with
         x^{t+1} and v^{t+1} = (x^{t+1} - x^t)/h (all vertices).
   x_bc: device (n_verts x dim) targets for the Dirichlet vertices, or NULL to
         keep their current positions.
   The predictor is x~ = x^t + h v^t with Dirichlet targets imposed; the
   iteration stops when |g(x_k)|_2 <= tol max(|g(x^_0)|_2, |f_g|_2, f_min)
   over free DOFs, with x^_0 the predictor (quasistatic: the start state with
   targets), f_g = h^2 m_i g (quasistatic: m_i g) the gravity load's part of
   the gradient, which keeps the test reachable for a loaded body at rest, and
   f_min = 1e-8 h^2 E V^((dim-1)/dim) (quasistatic: without h^2; V the rest
   volume), which does the same for an unloaded body at rest.
   *iters receives the iteration count, *rel_grad the final ratio.
   Returns CC_OK, CC_NOT_CONVERGED, CC_STALLED or an error. */
cc_status cc_step(cc_ctx* ctx, int32_t mesh_id, double* x, double* v, const double* x_bc,
                  double dt, const cc_params* params, double tol, int32_t* iters,
                  double* rel_grad);

/* One implicit time step of n meshes stepped together (same dim, each with
   its own material, basis and optional gravity).  Every launch of the
   iteration covers all meshes; a mesh that reaches its tolerance or its
   iteration cap is masked out while the others continue.  The launches of
   `iters_per_graph` iterations (cc_batch_tuning) are captured once in a HIP
   graph and replayed, with one host synchronisation per replay; meshes whose
   energy rises at alpha = 1 backtrack together on the device, eight halvings
   per launch, taking the first that does not raise E (the rule of cc_step),
   and only a mesh whose halvings run out goes to the host for the
   coordinate-descent fallback.  Arrays (host): mesh_ids[n]; x[n], v[n] and x_bc[n] hold device
   pointers as in cc_step (x_bc may be NULL or contain NULLs); gravity is
   n x 3 (host) or NULL to use params->gravity for every mesh.  Outputs
   (host, n each): iters, rel_grad, status (per-mesh cc_status).  The return
   value is the worst per-mesh status (errors before warnings), or
   CC_GRAPH_FALLBACK when the graph capture failed and the iterations ran
   as direct launches (every output valid).  On the legacy null stream no
   capture is attempted (see below) and nothing is reported.  The stream
   given to cc_create must not be the legacy null stream for graph capture;
   with it the launches run uncaptured. */
cc_status cc_step_batch(cc_ctx* ctx, int32_t n, const int32_t* mesh_ids, double* const* x,
                        double* const* v, const double* const* x_bc, const double* gravity,
                        double dt, const cc_params* params, double tol, int32_t* iters,
                        double* rel_grad, int32_t* status);

/* Tuning of the batched path.  lanes: lanes per vertex of the condensation
   and update kernels for bases stored as sparse rows (16, 32 or 64);
   iters_per_graph: iterations per graph replay (0 disables graphs).
   cc_batch_tuning sets them for later cc_step_batch calls; cc_autotune_batch
   times the condensation and update kernels of the given batch for every
   lane count on the current device state (no simulation state changes),
   keeps the fastest and returns it with the per-choice milliseconds
   (ms_out: 3 values for 16, 32, 64; may be NULL). */
cc_status cc_batch_tuning(cc_ctx* ctx, int32_t lanes, int32_t iters_per_graph);
/* Rows per workgroup of the exact-basis condensation (every basis row it
   stages serves that many vertices per H block it loads): 0 = the most whose
   LDS ring fits (4 in float32, 2 in float64 on MI355X), or a cap of 1 to
   4; and its chunk of band positions per pass, which is also its workgroup
   size: 0 = the one that leaves more waves resident per CU, or 128 / 256 /
   512.
   A forced chunk whose ring does not fit sends the mesh to the sparse-row
   kernel.  Applies to later cc_step, cc_probe_sweep and cc_step_batch calls;
   invalid values return CC_E_INVALID_ARG. */
cc_status cc_dense_tuning(cc_ctx* ctx, int32_t rows_per_workgroup, int32_t chunk);
cc_status cc_autotune_batch(cc_ctx* ctx, int32_t n, const int32_t* mesh_ids, const cc_params* params,
                            int32_t* lanes_out, double* ms_out);

/* Extra results of the last cc_step on a mesh (host outputs, any may be NULL):
   final step energy, the paper's normalised residual |g|/(V n E) (divided by
   h when dynamic), fallback counters (Ht or empty support, Schur, H_ii),
   line-search halvings taken, which warm-start proposal was accepted
   (0 none, 1 the network's x~ + c + l Delta, 2 the correction alone x~ + c),
   and the iterations whose displacement came from a fallback sweep (Jacobi
   or coordinate descent, see line_search).  Filled by cc_step and by
   cc_step_batch for each of its meshes. */
cc_status cc_step_info(cc_ctx* ctx, int32_t mesh_id, double* energy, double* paper_residual,
                       int64_t* fallbacks3, int64_t* halvings, int32_t* warm_accepted,
                       int64_t* sweep_fallbacks);

/* ---- parity probes: single kernels on caller device buffers ------------- */

/* Element gradient and projected Hessian at positions x (device, n x dim),
   without the h^2 factor: ge (device, n_elems x (dim+1) x dim) and
   He (device, n_elems x (dim+1) x (dim+1) x dim x dim, block [a][b] row-major),
   in caller element order, computed in `precision`. */
cc_status cc_probe_element(cc_ctx* ctx, int32_t mesh_id, const double* x, int32_t precision,
                           double* ge, double* He);

/* Step energy, free-vertex gradient (device g: n x dim, Dirichlet rows zero)
   and one Jacobi sweep's per-vertex directions dx (device n x dim, Dirichlet
   rows zero) at x, for inertial target x_tilde (device n x dim).  Any output
   pointer may be NULL. */
cc_status cc_probe_sweep(cc_ctx* ctx, int32_t mesh_id, const double* x, const double* x_tilde,
                         double dt, const cc_params* params, double* energy, double* g,
                         double* dx);

/* ---- learned warm start ----------------------------------------------------
   A per-vertex network proposes the start state of a step: features f_i (16
   values) of every free vertex at the inertial predictor x~ (relative
   predictor displacement, h v, the step-Hessian diagonal block and strain
   statistics of the incident elements), z-scored with stored statistics,
   pass through a 32-64-64-16 SiLU network (BF16 MFMA products, FP32
   accumulation) whose first three outputs Delta_i give
   x_i = x~_i + c_i + l Delta_i (l: mean rest edge length; c_i: the vertex's
   correction x_end - x~ of the mesh's last step, zero before the first, so
   the network learns how the correction changes from step to step).  With
   cc_params.warm_start = 1 cc_step and cc_step_batch use the proposal only
   when E(proposal) < E(x~) (float64); the convergence denominator stays
   |g(x~)|.  Not part of the paper: an extension evaluated against plain
   CC. */
#define CC_MLP_NPARAM 7312  /* packed float32 W1 32x64, b1 64, W2 64x64, b2 64,
                               W3 64x16, b3 16, row-major ([in][out])             */
#define CC_MLP_NFEAT  16

/* Load parameters (host, CC_MLP_NPARAM floats) and normalisation (host,
   16 means and 16 reciprocal standard deviations; NULL = 0 and 1); resets
   the Adam state. */
cc_status cc_mlp_set(cc_ctx* ctx, const float* params, const float* mean, const float* istd);
/* Copy the current parameters and normalisation to host arrays (any NULL). */
cc_status cc_mlp_get(cc_ctx* ctx, float* params, float* mean, float* istd);
/* Set the normalisation from N feature rows X (device, N x 16). */
cc_status cc_mlp_norm_from_data(cc_ctx* ctx, const float* X, int32_t N);
/* Features of a 3D mesh for the step that starts at x, v (device n x 3) with
   targets x_bc (device or NULL): feat (device, n_free x 16, one row per free
   vertex in ascending caller id), x_base (device n x 3, or NULL): the base
   the warm start adds l * Delta to, the predictor with targets plus, on free
   vertices, the mesh's last step correction x_end - x~ (zero before the
   mesh's first step; every cc_step / cc_step_batch on the mesh updates it),
   *ell (host, or NULL). */
cc_status cc_mlp_features(cc_ctx* ctx, int32_t mesh_id, const double* x, const double* v,
                          const double* x_bc, double dt, float* feat, double* x_base, double* ell);
/* Training targets T (device, n_free x 3, rows as in cc_mlp_features):
   (x_new - x_base) / l for the free vertices (x_new, x_base: device n x 3). */
cc_status cc_mlp_targets(cc_ctx* ctx, int32_t mesh_id, const double* x_new, const double* x_base,
                         float* T);
/* Network outputs Y (device, B x 3) for raw feature rows X (device, B x 16). */
cc_status cc_mlp_forward(cc_ctx* ctx, const float* X, int32_t B, float* Y);
/* Mean-squared-error gradient over the rows idx[0..B) (device int32) of X
   (device N x 16) against targets T (device N x 3): grad (device,
   CC_MLP_NPARAM floats, or NULL to keep it internal), *loss (host, or NULL). */
cc_status cc_mlp_gradient(cc_ctx* ctx, const float* X, const float* T, const int32_t* idx, int32_t B,
                          float* grad, float* loss);
/* cc_mlp_gradient without any device allocation, for callers that cannot
   allocate: code under HIP graph capture, training loops that forbid it.
   The per-wave partial gradients live in a static device array of the
   library (about 30 MB per device, held until the process ends) instead of
   context memory; the result equals cc_mlp_gradient's (same kernels, same
   summation order).  grad: device, CC_MLP_NPARAM floats (required); loss:
   device, one float (or NULL).  Nothing is copied to the host and the stream
   is not synchronised.  B must be in 1..CC_MLP_NOALLOC_MAX_ROWS, else
   CC_E_INVALID_ARG.  Calls that overlap on one device (other streams or
   threads) share the array and race; calls ordered on one stream do not. */
#define CC_MLP_NOALLOC_MAX_ROWS (1 << 26)
cc_status cc_mlp_gradient_noalloc(cc_ctx* ctx, const float* X, const float* T, const int32_t* idx,
                                  int32_t B, float* grad, float* loss);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) with gradient grad (device). */
cc_status cc_mlp_adam(cc_ctx* ctx, const float* grad, float lr);
/* cc_mlp_gradient followed by cc_mlp_adam on the same rows. */
cc_status cc_mlp_train_step(cc_ctx* ctx, const float* X, const float* T, const int32_t* idx, int32_t B,
                            float lr, float* loss);

/* ---- measurement --------------------------------------------------------- */

/* Kernel identifiers for cc_profile_*. */
#define CC_K_ELEM_HESS  0   /* element Hessians                          */
#define CC_K_ASSEMBLE   1   /* block-row assembly                        */
#define CC_K_GRADIENT   2   /* float64 free-vertex gradient + norm parts  */
#define CC_K_CC_PREP    3   /* per-vertex condensation (A, Ht, K, L)      */
#define CC_K_CC_UPDATE  4   /* per-vertex update dx = -K (g - L U^T g)    */
#define CC_K_ENERGY     5   /* float64 step energy partials               */
#define CC_K_COUNT      6

/* Record the duration of every launch of the kernels whose bit is set in
   `mask` (bit k = kernel id k) with HIP events on the context's stream;
   mask = 0 stops recording.  Enabling clears the accumulators.  Timing adds
   two event records per timed launch.  Enabling, and stopping a recording,
   also launch an empty kernel `k_profile_mark` on the context's stream, the
   region's boundary in a kernel trace. */
cc_status cc_profile_enable(cc_ctx* ctx, int32_t mask);
/* Accumulated device milliseconds and launch count of kernel `kernel_id`
   since the last cc_profile_enable (host outputs). */
cc_status cc_profile_read(cc_ctx* ctx, int32_t kernel_id, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* CCGPU_H */
