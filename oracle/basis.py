"""Per-vertex perturbation basis (FP64), computed at rest or at a given state.

The paper builds, for every coordinate i, the response of the complementary
degrees of freedom C (all free DOFs except vertex i's) to a unit perturbation
of vertex i while keeping zero force on C:

    [H_ii H_iC; H_Ci H_CC] [I; U_i] = [df_i; 0]   =>   U_i = -H_CC^{-1} H_Ci

(Background, JGS2 subsection; Method, Coordinate Condensation: "computed at
the rest configuration").  H is the Hessian of the step energy at x = X (for
dynamics that includes the mass term, M + h^2 K(X)).  Given a state x, the
same construction on the projected Hessian at x gives the basis that the
paper's restarted variant reconstructs from the current configuration
(Results, Subspace Quality).

Two supports are provided:

* exact (R = infinity): C is every other free vertex.  Computed through the
  identity [I; U_i] = H^{-1} E_i ((H^{-1})_ii)^{-1}, i.e. with Z = H^{-1} E_i,
  U_i[j] = Z_j Z_i^{-1}.  This needs one factorisation of H.
* patch (finite R): C is the set of free vertices within R hops of i in the
  free-vertex graph, with every vertex outside the patch held fixed; then
  U_i = -H[C,C]^{-1} H[C,i].  This truncation is this package's reading for
  meshes where the dense exact basis does not fit (the paper's basis is the
  exact one).

Storage: CSR over the original vertex ids.  ptr (n+1, int64); idx (nnz,
int32) ascending vertex ids; U (nnz, d, d) with U[k] the block U_i[j] that
maps a displacement of vertex i to the displacement of vertex j = idx[k].
Dirichlet vertices have empty rows and never appear in a support.

Pins: tests/test_oracle_basis_colour.py -- exact basis satisfies H_CC U_i + H_Ci = 0
and matches a direct per-vertex solve of that equation (at rest and at a
deformed state); patch basis satisfies the patch equilibrium; Dirichlet
vertices absent; the state-given basis at x = X is the rest basis.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def rest_hessian(prob, x=None):
    """Projected step Hessian at rest, or at the state x when given."""
    return prob.hessian(prob.X if x is None else x, project=True)


def exact_basis(prob, x=None, verts=None):
    """Exact basis; with verts given (vertex ids), only those rows are filled."""
    d = prob.d
    H = rest_hessian(prob, x).tocsc()
    lu = spla.splu(H)
    nf = prob.free.size
    ptr = np.zeros(prob.n + 1, dtype=np.int64)
    idx_list, U_list = [], []
    want = None if verts is None else set(int(v) for v in verts)
    for fi, i in enumerate(prob.free):
        if want is not None and int(i) not in want:
            continue
        E = np.zeros((prob.ndof, d))
        E[fi * d:(fi + 1) * d, :] = np.eye(d)
        Z = lu.solve(E).reshape(nf, d, d)              # Z[j] = rows of vertex j
        Zi_inv = np.linalg.inv(Z[fi])
        others = np.array([j for j in range(nf) if j != fi], dtype=np.int64)
        idx_list.append(prob.free[others])
        U_list.append(np.einsum("jab,bc->jac", Z[others], Zi_inv))
        ptr[i + 1] = others.size
    return _finish(prob, ptr, idx_list, U_list)


def patch_supports(prob, R):
    adj = prob.adjacency()
    supp = [[] for _ in range(prob.n)]
    for i in prob.free:
        seen = {int(i)}
        frontier = [int(i)]
        for _ in range(R):
            nxt = []
            for v in frontier:
                for w in adj[v]:
                    if w not in seen:
                        seen.add(w)
                        nxt.append(w)
            frontier = nxt
        seen.discard(int(i))
        supp[i] = sorted(seen)
    return supp


def patch_basis(prob, R=1, verts=None, x=None):
    """Patch basis; with verts given, only those vertices get non-empty rows."""
    d = prob.d
    H = rest_hessian(prob, x).tocsr()
    supp = patch_supports(prob, R)
    ptr = np.zeros(prob.n + 1, dtype=np.int64)
    idx_list, U_list = [], []
    todo = prob.free if verts is None else np.intersect1d(prob.free, verts)
    for i in todo:
        C = np.asarray(supp[i], dtype=np.int64)
        ptr[i + 1] = C.size
        if C.size == 0:
            idx_list.append(C)
            U_list.append(np.zeros((0, d, d)))
            continue
        cd = (prob.fidx[C][:, None] * d + np.arange(d)[None, :]).ravel()
        idd = prob.fidx[i] * d + np.arange(d)
        Hcc = H[cd][:, cd].toarray()
        Hci = H[cd][:, idd].toarray()
        U = -np.linalg.solve(Hcc, Hci)                  # (|C| d, d)
        idx_list.append(C)
        U_list.append(U.reshape(C.size, d, d))
    return _finish(prob, ptr, idx_list, U_list)


def _finish(prob, ptr, idx_list, U_list):
    ptr = np.cumsum(ptr).astype(np.int64)
    # rows are emitted in ascending free-vertex order, which is ascending id
    idx = np.concatenate(idx_list).astype(np.int32) if idx_list else np.zeros(0, np.int32)
    U = np.concatenate(U_list, axis=0) if U_list else np.zeros((0, prob.d, prob.d))
    return ptr, idx, U


def basis_matrix(prob, ptr, idx, U):
    """Assemble the block matrix whose column block i (free rank) is U_i over free DOFs."""
    d = prob.d
    owner = np.repeat(np.arange(prob.n), np.diff(ptr))        # vertex i of each block
    fi = prob.fidx[owner]
    fj = prob.fidx[idx]
    r = np.arange(d)
    rows = fj[:, None, None] * d + r[None, :, None] + 0 * r[None, None, :]
    cols = fi[:, None, None] * d + r[None, None, :] + 0 * r[None, :, None]
    return sp.csc_matrix((U.ravel(), (rows.ravel(), cols.ravel())),
                         shape=(prob.ndof, prob.ndof))
