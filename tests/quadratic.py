"""Quadratic test problems exposing the interface the oracle solvers use.

E(x) = 1/2 (x_f - x0_f)^T K (x_f - x0_f) - c^T x_f over the free degrees of
freedom x_f.  On such a problem Coordinate Condensation with the exact basis
takes exactly the Newton step (Results, Material Stiffness Scaling: "single
iteration convergence" for the quadratic rod).
"""
import numpy as np
import scipy.sparse as sp


class QuadraticProblem:
    def __init__(self, K, n, d, fixed=None, c=None, x0=None):
        self.K = sp.csr_matrix(K)
        self.n, self.d = n, d
        self.fixed = np.zeros(n, dtype=bool) if fixed is None else np.asarray(fixed, bool)
        self.free = np.flatnonzero(~self.fixed)
        self.fidx = -np.ones(n, dtype=np.int64)
        self.fidx[self.free] = np.arange(self.free.size)
        assert self.K.shape == (self.free.size * d,) * 2
        self.c = np.zeros(self.free.size * d) if c is None else np.asarray(c, float)
        self.X = np.zeros((n, d)) if x0 is None else np.asarray(x0, float)
        self.quasistatic = True
        self.h = 1.0
        self.E = 1.0
        self.vol = np.ones(1)

    @property
    def ndof(self):
        return self.free.size * self.d

    def _u(self, x):
        return (np.asarray(x)[self.free] - self.X[self.free]).ravel()

    def energy(self, x):
        u = self._u(x)
        return 0.5 * u @ (self.K @ u) - self.c @ u

    def gradient(self, x):
        u = self._u(x)
        return (self.K @ u - self.c).reshape(-1, self.d)

    def hessian(self, x, project=True):
        return self.K.copy()

    def load_norm(self):
        """No gravity load: the residual is relative to the start gradient."""
        return 0.0

    def residual_floor(self):
        """No elastic force scale: the residual is relative to the start gradient."""
        return 0.0

    def adjacency(self):
        K = self.K.tocoo()
        nbr = [set() for _ in range(self.n)]
        for r, c in zip(K.row // self.d, K.col // self.d):
            if r != c:
                nbr[self.free[r]].add(int(self.free[c]))
        return [sorted(s) for s in nbr]


def spring_rod(n, k, m, h):
    """1D rod of n vertices joined by springs of stiffness k, lumped masses m,
    implicit-Euler Hessian M + h^2 K, left end fixed (vertex 0)."""
    fixed = np.zeros(n, dtype=bool)
    fixed[0] = True
    nf = n - 1
    K = sp.lil_matrix((nf, nf))
    for a in range(n - 1):            # spring between vertex a and a+1
        ia, ib = a - 1, a             # free ranks (vertex v -> v-1)
        for (p, q, s) in ((ia, ia, 1), (ib, ib, 1), (ia, ib, -1), (ib, ia, -1)):
            if p >= 0 and q >= 0:
                K[p, q] += s * k
    H = sp.identity(nf) * m + h * h * K.tocsr()
    return H, fixed


def random_spd_chain(nv, d, rng, coupling=0.9):
    """Block-tridiagonal SPD matrix with random d x d blocks."""
    nd = nv * d
    A = np.zeros((nd, nd))
    for i in range(nv):
        for j in (i - 1, i, i + 1):
            if 0 <= j < nv:
                B = rng.normal(size=(d, d))
                A[i * d:(i + 1) * d, j * d:(j + 1) * d] += coupling * B if i != j else B
    A = A + A.T
    w = np.linalg.eigvalsh(A)
    A += (abs(w.min()) + 0.5) * np.eye(nd)
    return sp.csr_matrix(A)
