"""Coordinate Condensation, coordinate descent and Newton (FP64).

Per-vertex update (Method section, Eqs. displacement -> schur):
the displacement of the local problem of vertex i is B_i q_i with
B_i = diag(I, U_i) and q_i = (dx_i, da_i).  Minimising the quadratic model of
E at the current x over q_i gives the coupled system

    [ H_ii      H_iC U_i      ] [dx_i]     [ g_i        ]
    [ U_i^T H_Ci  U_i^T H_CC U_i ] [da_i] = - [ U_i^T g_C ]

and block elimination gives

    A_i   = H_iC U_i                    (d x d)
    Ht_i  = U_i^T H_CC U_i              (reduced complementary stiffness)
    S_i   = A_i Ht_i^{-1} A_i^T         (Schur correction)
    gt_i  = g_i - A_i Ht_i^{-1} U_i^T g_C
    dx_i  = -(H_ii - S_i)^{-1} gt_i      ; da_i is discarded (Maintaining Locality)

Plain coordinate descent (Background, Coordinate Descent) is the case S = 0,
gt = g_i: one block-Newton step per vertex (reading of its exact argmin).  The
JGS2 update printed in the Background section, dx_i = -(H_ii + Ht_i)^{-1}
(g_i + U_i^T g_C), is also provided.

Sweeps:
* Jacobi (Algorithm 1): every dx_i from one snapshot of g and H, then
  x <- x + d.
* Coloured Gauss-Seidel ("most recent values", Background): colours in
  increasing order; before each colour g is re-evaluated at the current x;
  H is re-evaluated before each colour (HESS_COLOUR, the default reading) or
  once at the start of the sweep (HESS_SWEEP, an explicit lagged-Hessian
  mode).  The colour's vertices then move simultaneously.

Corotated basis (Method, Accounting for Large Deformations, Eq. rotation),
with params.corotate: wherever g and H are evaluated, every basis block is
rotated, U_i^rot[j] = R_j U_i[j], with R_j the rotation factor of the polar
decomposition of sum_{k in N(j)} (x_k - x_j)(X_k - X_j)^T over the mesh
neighbours of j (this package's reading of "the displacement of the
neighbourhood").  Pins: tests/test_oracle_corotation.py -- the polar factor
against M (M^T M)^(-1/2), rigid motions give R_j = Q, identity at rest,
rotation equivariance of the directions (which the unrotated basis lacks),
convergence to Newton's minimiser under a 60 degree twist.

Readings taken where the paper is silent:
* small solves are Cholesky factorisations that fail when a pivot falls below
  1e-12 times the trace of the matrix; if Ht_i fails or the support is empty,
  or H_ii - S_i fails, vertex i takes the coordinate-descent step; if H_ii
  fails too, dx_i = 0;
* global backtracking line search along the sweep's displacement d (Results,
  Sensitivity to basis quality): alpha = 1, halved while
  E(x + alpha d) > E(x) + tau with tau = 1e-12 max(|E(x)|, 1), at most
  max_halvings (20: alpha >= 2^-20, below which a step moves x by less than
  the rounding of its coordinates' changes) times; on failure, one
  coordinate-descent sweep with the same search; on failure again the solve
  stops with status STALLED.  A coloured sweep of CC or JGS2 is taken only
  at its full step (no halvings): when that raises E by more than tau, the
  iteration takes a Jacobi sweep of the same method with the search, and
  then the coordinate-descent fallback.  Each colour's condensed step assumes
  the colours after it follow through the basis; once the intermediate state
  is strained, the sweep's displacement can point almost nowhere downhill,
  and halving it then makes vanishing progress per iteration where the
  Jacobi (near-Newton) step does not.  SolveResult.sweep_fallbacks counts
  the iterations whose displacement came from a fallback sweep;
* termination: r_k = |g(x_k)|_2 / max(|g(x^_0)|_2, |f_g|_2, f_min) <= tol,
  where x^_0 is the inertial predictor with boundary targets (dynamic) or the
  initial guess (quasistatic), f_g = s_el m_i grav is the gravity load's part
  of the gradient over free DOFs, and f_min = 1e-8 s_el E V^((d-1)/d) (V the
  rest volume) is a floor at 1e-8 of the elastic force scale.  The load term
  keeps the test reachable for a loaded body that has settled: there
  |g(x^_0)| falls towards the rounding level of the force balance the body
  holds (the elastic forces cancelling the load), which a fixed fraction of
  it would ask the iteration to undercut.  The floor does the same for an
  unloaded body at rest, whose start gradient is only the rounding of its
  element forces; for any loaded or driven step it lies far below the other
  two terms.  The paper's own measure |g|/(V n E) (divided by h for
  dynamics) is also recorded.

Pins: tests/test_oracle_solvers.py -- with the exact basis one Jacobi
iteration equals the Newton step on quadratic problems (a spring rod, random
SPD chains, linear-elastic FEM) and converges in one iteration (Results,
Material Stiffness Scaling); the Schur form equals a direct solve of the
coupled block system; CD equals textbook block Jacobi / block Gauss-Seidel;
the line search never raises E by more than tau; converged CC states equal
Newton's minimiser on small meshes.
"""
from dataclasses import dataclass, field, replace

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .basis import basis_matrix

CD, CC, JGS2 = 0, 1, 2
JACOBI, GS = 0, 1
HESS_COLOUR, HESS_SWEEP = 0, 1

OK, NOT_CONVERGED, STALLED = 0, 1, 2

PIVOT_REL = 1e-12


@dataclass
class Params:
    method: int = CC
    sweep: int = GS
    hess_refresh: int = HESS_COLOUR
    line_search: bool = True
    max_iters: int = 10000
    max_halvings: int = 20
    corotate: bool = False      # rotate the basis blocks by per-vertex rotations


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    rel_grad: float
    status: int
    history: list = field(default_factory=list)   # per iteration (r, E, alpha, paper_measure)
    fallbacks: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=np.int64))
    sweep_fallbacks: int = 0   # iterations that took a Jacobi or CD fallback sweep


def chol_solve(M, B):
    """Solve M X = B for a stack of small SPD matrices by Cholesky.

    M (k, d, d), B (k, d, r).  Returns (X, ok) where ok[k] is False when a pivot
    of M[k] is not above PIVOT_REL * trace(M[k])."""
    M = np.asarray(M, dtype=np.float64)
    k, d, _ = M.shape
    tol = PIVOT_REL * np.einsum("kii->k", M)
    L = np.zeros_like(M)
    ok = np.ones(k, dtype=bool)
    for j in range(d):
        s = M[:, j, j] - np.sum(L[:, j, :j] ** 2, axis=1)
        ok &= s > tol
        ljj = np.sqrt(np.where(s > 0, s, 1.0))
        L[:, j, j] = ljj
        for i in range(j + 1, d):
            L[:, i, j] = (M[:, i, j] - np.sum(L[:, i, :j] * L[:, j, :j], axis=1)) / ljj
    Y = np.array(B, dtype=np.float64, copy=True)
    for i in range(d):                                   # forward: L y = b
        Y[:, i] = (Y[:, i] - np.einsum("kj,kjr->kr", L[:, i, :i], Y[:, :i])) / L[:, i, i, None]
    for i in reversed(range(d)):                         # backward: L^T x = y
        Y[:, i] = (Y[:, i] - np.einsum("kj,kjr->kr", L[:, i + 1:, i], Y[:, i + 1:])) / L[:, i, i, None]
    return Y, ok


def _blocks(S, row_dofs, col_dofs):
    """Dense (k, d, d) blocks S[row_dofs[k], col_dofs[k]] of a sparse matrix."""
    k, d = row_dofs.shape
    R = np.broadcast_to(row_dofs[:, :, None], (k, d, d)).ravel()
    C = np.broadcast_to(col_dofs[:, None, :], (k, d, d)).ravel()
    return np.asarray(S[R, C]).reshape(k, d, d)


def local_directions(prob, Umat, H, g, verts, method):
    """dx_i for the free-rank vertices `verts`, from g (n_free, d) and sparse H.

    Returns (dx (k, d), fallback counts [Ht or empty support, Schur, H_ii])."""
    d = prob.d
    verts = np.asarray(verts, dtype=np.int64)
    k = verts.size
    dofs = verts[:, None] * d + np.arange(d)[None, :]
    Hii = _blocks(H, dofs, dofs)
    gi = g[verts]
    dcd, ok_ii = chol_solve(Hii, -gi[:, :, None])
    dcd = np.where(ok_ii[:, None], dcd[:, :, 0], 0.0)
    counts = np.zeros(3, dtype=np.int64)
    counts[2] = int(np.sum(~ok_ii))
    if method == CD or Umat is None:
        return dcd, counts

    Uc = Umat[:, dofs.ravel()]                            # columns of the k bases
    Y = (H @ Uc).tocsc()                                   # H U_i for each i
    local = np.arange(k)[:, None] * d + np.arange(d)[None, :]
    A = _blocks(Y, dofs, local)                            # A_i = H_iC U_i  (rows of i)
    Ht = np.zeros((k, d, d))
    for p in range(d):                                     # Ht_i = U_i^T (H U_i)
        for q in range(d):
            Ht[:, p, q] = np.asarray(Uc[:, p::d].multiply(Y[:, q::d]).sum(axis=0)).ravel()
    b = (Uc.T @ g.ravel()).reshape(k, d)                   # b_i = U_i^T g_C
    empty = np.diff(Uc.indptr)[::d] == 0

    if method == JGS2:
        dx, ok = chol_solve(Hii + Ht, -(gi + b)[:, :, None])
        good = ok & ~empty
        counts[0] = int(np.sum(~good))
        return np.where(good[:, None], dx[:, :, 0], dcd), counts

    rhs = np.concatenate([np.swapaxes(A, 1, 2), b[:, :, None]], axis=2)
    Z, ok_t = chol_solve(Ht, rhs)                          # Ht^{-1} [A^T | b]
    S = np.einsum("kij,kjl->kil", A, Z[:, :, :d])
    gt = gi - np.einsum("kij,kj->ki", A, Z[:, :, d])
    dx, ok_s = chol_solve(Hii - S, -gt[:, :, None])
    t_ok = ok_t & ~empty
    s_ok = t_ok & ok_s
    counts[0] = int(np.sum(~t_ok))
    counts[1] = int(np.sum(t_ok & ~ok_s))
    return np.where(s_ok[:, None], dx[:, :, 0], dcd), counts


def mesh_neighbours(prob):
    """Sorted lists of all vertices sharing an element with each vertex
    (Dirichlet vertices included)."""
    nbr = [set() for _ in range(prob.n)]
    for e in prob.elems:
        for a in e:
            nbr[int(a)].update(int(b) for b in e if b != a)
    return [sorted(v) for v in nbr]


def polar_rotation(M):
    """Rotation factor of the polar decomposition M = R S (det R = +1), from
    the SVD M = U diag(s) V^T: R = U diag(1, .., 1, det(U V^T)) V^T."""
    U, _, Vt = np.linalg.svd(M)
    D = np.eye(M.shape[0])
    D[-1, -1] = np.sign(np.linalg.det(U @ Vt))
    return U @ D @ Vt


def vertex_rotations(prob, x, nbr=None):
    """Per-vertex rotations estimated from the displacement of each free
    vertex's neighbourhood (Method, Accounting for Large Deformations; this
    package's reading): R_j = polar factor of
    sum_{k in N(j)} (x_k - x_j)(X_k - X_j)^T, N(j) the mesh neighbours.
    Returns (n_free, d, d)."""
    nbr = mesh_neighbours(prob) if nbr is None else nbr
    out = np.zeros((prob.free.size, prob.d, prob.d))
    for r, j in enumerate(prob.free):
        ks = np.asarray(nbr[j], dtype=np.int64)
        M = (x[ks] - x[j]).T @ (prob.X[ks] - prob.X[j])
        out[r] = polar_rotation(M)
    return out


def rotate_basis(prob, Umat, R):
    """U_i^rot[j] = R_j U_i[j] for every basis column (Method, Eq. rotation):
    the rows of free vertex j are multiplied by R_j."""
    d, nf = prob.d, prob.free.size
    blocks = sp.block_diag([R[r] for r in range(nf)], format="csr") if nf else sp.csr_matrix((0, 0))
    return (blocks @ Umat).tocsc()


def _basis_at(prob, Umat, x, params):
    if Umat is None or not params.corotate:
        return Umat
    return rotate_basis(prob, Umat, vertex_rotations(prob, x))


def sweep(prob, x, Umat, colours_free, params, method=None):
    """One iteration; returns (x_new, fallback counts).  With params.corotate
    the basis is rotated at the state where g and H are evaluated."""
    method = params.method if method is None else method
    f = prob.free
    counts = np.zeros(3, dtype=np.int64)
    if params.sweep == JACOBI:
        g = prob.gradient(x)
        H = prob.hessian(x)
        dx, c = local_directions(prob, _basis_at(prob, Umat, x, params), H, g, np.arange(f.size), method)
        x_new = x.copy()
        x_new[f] += dx
        return x_new, counts + c
    x_cur = x.copy()
    H = None
    Ucur = Umat
    for col in range(int(colours_free.max()) + 1 if colours_free.size else 0):
        verts = np.flatnonzero(colours_free == col)
        if verts.size == 0:
            continue
        if H is None or params.hess_refresh == HESS_COLOUR:
            H = prob.hessian(x_cur)
            Ucur = _basis_at(prob, Umat, x_cur, params)
        g = prob.gradient(x_cur)
        dx, c = local_directions(prob, Ucur, H, g, verts, method)
        counts += c
        x_cur[f[verts]] += dx
    return x_cur, counts


def paper_measure(prob, g):
    """|g| / (V n E), divided by h for dynamic problems (Results, Termination criteria)."""
    V = float(np.sum(prob.vol))
    val = np.linalg.norm(g) / (V * prob.n * prob.E)
    return val if prob.quasistatic else val / prob.h


def _line_search(prob, x, d, max_halvings):
    E0 = prob.energy(x)
    tau = 1e-12 * max(abs(E0), 1.0)
    alpha = 1.0
    Ek = prob.energy(x + d)
    halvings = 0
    while Ek > E0 + tau and halvings < max_halvings:
        alpha *= 0.5
        Ek = prob.energy(x + alpha * d)
        halvings += 1
    return (Ek <= E0 + tau), alpha, Ek


def solve(prob, x0, basis, params, tol, colours=None, x_hat0=None, record=False):
    """Run the iteration from x0 (full (n, d) array with boundary values set)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    Umat = basis_matrix(prob, *basis) if basis is not None else None
    cf = (np.zeros(prob.free.size, dtype=np.int64) if colours is None
          else np.asarray(colours)[prob.free])
    g0 = max(np.linalg.norm(prob.gradient(x if x_hat0 is None else x_hat0)), prob.load_norm(),
             prob.residual_floor())
    res = SolveResult(x=x, iters=0, rel_grad=0.0, status=OK)
    gx = prob.gradient(x)
    if g0 == 0.0:
        res.rel_grad = 0.0
        return res
    r = np.linalg.norm(gx) / g0
    if record:
        res.history.append((r, prob.energy(x), 1.0, paper_measure(prob, gx)))
    k = 0
    while r > tol and k < params.max_iters:
        x_new, c = sweep(prob, x, Umat, cf, params)
        res.fallbacks += c
        alpha = 1.0
        if params.line_search:
            coloured = params.sweep == GS and params.method != CD
            ok, alpha, _ = _line_search(prob, x, x_new - x, 0 if coloured else params.max_halvings)
            if not ok:
                tries = [(replace(params, sweep=JACOBI), None)] if coloured else []
                tries.append((params, CD))
                for prm_fb, meth in tries:
                    x_fb, _ = sweep(prob, x, Umat, cf, prm_fb, method=meth)
                    ok, alpha, _ = _line_search(prob, x, x_fb - x, params.max_halvings)
                    if ok:
                        x_new = x_fb
                        res.sweep_fallbacks += 1
                        break
                if not ok:
                    res.status = STALLED
                    break
            x = x + alpha * (x_new - x)
        else:
            x = x_new
        k += 1
        gx = prob.gradient(x)
        r = np.linalg.norm(gx) / g0
        if record:
            res.history.append((r, prob.energy(x), alpha, paper_measure(prob, gx)))
        if not np.all(np.isfinite(x)):
            res.status = STALLED
            break
    res.x, res.iters, res.rel_grad = x, k, float(r)
    if res.status == OK and r > tol:
        res.status = NOT_CONVERGED
    return res


def newton(prob, x0, tol=1e-10, max_iters=100, x_hat0=None, c_armijo=1e-4, record=False):
    """Projected Newton with a sparse direct solve and Armijo backtracking."""
    x = np.array(x0, dtype=np.float64, copy=True)
    f = prob.free
    g0 = max(np.linalg.norm(prob.gradient(x if x_hat0 is None else x_hat0)), prob.load_norm(),
             prob.residual_floor())
    hist = []
    g = prob.gradient(x)
    r = np.linalg.norm(g) / g0 if g0 > 0 else 0.0
    if record:
        hist.append((r, prob.energy(x), 1.0, paper_measure(prob, g)))
    k = 0
    while r > tol and k < max_iters:
        H = prob.hessian(x).tocsc()
        p = spla.spsolve(H, -g.ravel()).reshape(-1, prob.d)
        E0 = prob.energy(x)
        slope = float(np.sum(g * p))
        alpha = 1.0
        while True:
            xt = x.copy()
            xt[f] += alpha * p
            if prob.energy(xt) <= E0 + c_armijo * alpha * slope or alpha < 1e-12:
                break
            alpha *= 0.5
        if alpha < 1e-12:
            break
        x = xt
        k += 1
        g = prob.gradient(x)
        r = np.linalg.norm(g) / g0
        if record:
            hist.append((r, prob.energy(x), alpha, paper_measure(prob, g)))
    return SolveResult(x=x, iters=k, rel_grad=float(r), status=OK if r <= tol else NOT_CONVERGED,
                       history=hist)
