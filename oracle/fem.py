"""Global energy, gradient and Hessian of one implicit-Euler step (FP64).

The step objective is the paper's variational implicit Euler energy
(Background, Optimization-Based Integration):

    E(x) = sum_i 1/2 m_i |x_i - x~_i|^2 + h^2 [ sum_e V_e Psi(F_e) - sum_i m_i g.x_i ]

with x~ = x^t + h v^t the inertial target (the footnote of that equation) and
the gravity potential one of the "additional potentials" it allows.  In the
quasistatic form the inertia term is dropped and the h^2 factor is 1.  Sums
over i run over free vertices only (Dirichlet vertices contribute constants).

Element terms (with the projected material Hessian C):
    g_e[a]      = V_e P beta_a
    H_e[a,b]_rs = V_e sum_{q,t} beta_{a,q} C_{(r,q),(s,t)} beta_{b,t}

Gradient and Hessian are restricted to free degrees of freedom, ordered by
free-vertex rank (ascending vertex id) then component.

Pins: tests/test_oracle_mesh_fem.py -- finite differences of E (gradient) and of
the gradient (unprojected Hessian); sum_a g_e[a] = 0; H_e annihilates
translations; symmetry; one Newton step solves a linear-elastic problem
exactly.
"""
import numpy as np
import scipy.sparse as sp

from .material import SNH, energy_density, lame, project_psd
from .mesh import deformation_gradient, lumped_mass, rest_data


class Problem:
    """One mesh with material, Dirichlet set and time-step constants."""

    def __init__(self, X, elems, fixed, E, nu, rho, gravity, dt, quasistatic, material=SNH):
        self.X = np.asarray(X, dtype=np.float64)
        self.elems = np.asarray(elems, dtype=np.int64)
        self.n, self.d = self.X.shape
        self.beta, self.vol = rest_data(self.X, self.elems)
        self.mass = lumped_mass(self.n, self.elems, self.vol, rho)
        self.E, self.nu, self.rho = E, nu, rho
        self.material = material
        self.mu, self.lam = lame(E, nu, material)
        self._psi, self._pk1, self._dpdf = energy_density(material)
        self.fixed = np.asarray(fixed).astype(bool)
        self.free = np.flatnonzero(~self.fixed)
        self.fidx = -np.ones(self.n, dtype=np.int64)
        self.fidx[self.free] = np.arange(self.free.size)
        self.grav = np.asarray(gravity, dtype=np.float64)[: self.d]
        self.h = float(dt)
        self.quasistatic = bool(quasistatic)
        self.w_in = 0.0 if quasistatic else 1.0
        self.s_el = 1.0 if quasistatic else self.h * self.h
        self.x_tilde = self.X.copy()
        self._pattern = None

    @classmethod
    def from_scene(cls, s):
        return cls(s.X, s.elems, s.fixed, s.E, s.nu, s.rho, s.gravity, s.dt, s.quasistatic,
                   getattr(s, "material", SNH))

    @property
    def ndof(self):
        return self.free.size * self.d

    def set_inertial_target(self, x_tilde):
        self.x_tilde = np.asarray(x_tilde, dtype=np.float64).copy()

    # ----- element level -------------------------------------------------
    def element_energy(self, x):
        F = deformation_gradient(x, self.elems, self.beta)
        return self.vol * self._psi(F, self.mu, self.lam)

    def element_gradient(self, x):
        F = deformation_gradient(x, self.elems, self.beta)
        P = self._pk1(F, self.mu, self.lam)
        return self.vol[:, None, None] * np.einsum("mrq,maq->mar", P, self.beta)

    def element_hessian(self, x, project=True):
        """H_e as (m, d+1, d+1, d, d): block [a, b] is the d x d block H_e[a,b]."""
        d = self.d
        F = deformation_gradient(x, self.elems, self.beta)
        C = self._dpdf(F, self.mu, self.lam)
        if project:
            C = project_psd(C)
        C4 = C.reshape(-1, d, d, d, d)                    # [r, q, s, t]
        return self.vol[:, None, None, None, None] * np.einsum(
            "maq,mrqst,mbt->mabrs", self.beta, C4, self.beta, optimize=True)

    # ----- global level --------------------------------------------------
    def energy(self, x):
        x = np.asarray(x)
        f = self.free
        dx = x[f] - self.x_tilde[f]
        inertia = 0.5 * np.sum(self.mass[f] * np.einsum("ij,ij->i", dx, dx))
        grav = np.sum(self.mass[f] * (x[f] @ self.grav))
        return self.w_in * inertia + self.s_el * (np.sum(self.element_energy(x)) - grav)

    def gradient_full(self, x):
        """Gradient on every vertex, (n, d) (rows of fixed vertices included)."""
        x = np.asarray(x)
        ge = self.element_gradient(x)
        gel = np.zeros((self.n, self.d))
        np.add.at(gel, self.elems.ravel(), ge.reshape(-1, self.d))
        return (self.w_in * self.mass[:, None] * (x - self.x_tilde)
                + self.s_el * (gel - self.mass[:, None] * self.grav[None, :]))

    def gradient(self, x):
        """Gradient restricted to free vertices, (n_free, d)."""
        return self.gradient_full(x)[self.free]

    def load_norm(self):
        """Norm over free DOFs of the gravity load's part of the gradient,
        |s_el m_i grav| (the scale of the force balance a loaded body holds)."""
        f = self.free
        return self.s_el * float(np.linalg.norm(self.mass[f])) * float(np.linalg.norm(self.grav))

    def residual_floor(self):
        """1e-8 of the elastic force scale s_el E V^((d-1)/d) (V the rest
        volume): the least gradient norm the convergence test divides by.  A
        body at rest with no load has a start gradient at the rounding level
        of its element forces, relative to which no iterate can pass."""
        V = float(np.sum(self.vol))
        return 1e-8 * self.s_el * self.E * V ** ((self.d - 1) / self.d)

    def hessian(self, x, project=True):
        """Sparse (CSR) Hessian over free DOFs: w_in M + s_el sum_e H_e."""
        d = self.d
        He = self.element_hessian(x, project=project)
        k = self.elems.shape[1]
        fa = self.fidx[self.elems]                         # (m, k)
        rows, cols, vals = [], [], []
        r_ = np.arange(d)
        for a in range(k):
            for b in range(k):
                ok = (fa[:, a] >= 0) & (fa[:, b] >= 0)
                ra = fa[ok, a][:, None, None] * d + r_[None, :, None]
                cb = fa[ok, b][:, None, None] * d + r_[None, None, :]
                rows.append(np.broadcast_to(ra, (ok.sum(), d, d)).ravel())
                cols.append(np.broadcast_to(cb, (ok.sum(), d, d)).ravel())
                vals.append(self.s_el * He[ok, a, b].ravel())
        mdiag = np.repeat(self.w_in * self.mass[self.free], d)
        rows.append(np.arange(self.ndof))
        cols.append(np.arange(self.ndof))
        vals.append(mdiag)
        H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.ndof, self.ndof)).tocsr()
        H.sum_duplicates()
        return H

    def adjacency(self):
        """Free-vertex graph: sorted neighbour lists (free vertices sharing an element)."""
        nbr = [set() for _ in range(self.n)]
        for e in self.elems:
            for a in e:
                if self.fixed[a]:
                    continue
                for b in e:
                    if b != a and not self.fixed[b]:
                        nbr[a].add(int(b))
        return [sorted(s) for s in nbr]
