"""Scene builders: meshes, Dirichlet sets, prescribed targets and material draws.

Every scene is deterministic given its arguments (and seed, where drawn).
Units are SI: metres, pascals, kg/m^3, seconds.
"""
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .grid import grid2d, grid3d

GRAV = 9.81


@dataclass
class Scene:
    name: str
    dim: int
    X: np.ndarray              # (n, dim) rest positions
    elems: np.ndarray          # (m, dim+1) int32, positively oriented
    fixed: np.ndarray          # (n,) uint8, 1 = Dirichlet vertex
    E: float                   # Young's modulus
    nu: float                  # Poisson ratio
    rho: float                 # density
    gravity: np.ndarray        # (3,) gravitational acceleration
    dt: float                  # time step h
    n_steps: int
    quasistatic: bool
    target_fn: Callable[[int], np.ndarray] = field(repr=False, default=None)
    x_init: Optional[np.ndarray] = field(repr=False, default=None)
    v_init: Optional[np.ndarray] = field(repr=False, default=None)
    meta: dict = field(default_factory=dict)
    material: str = "snh"      # "snh" stable neo-Hookean, "fcr" Fixed Corotational

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def m(self):
        return self.elems.shape[0]

    def targets(self, t):
        """(n, dim) array whose rows at Dirichlet vertices hold the step-t targets."""
        if self.target_fn is None:
            return self.X.copy()
        return self.target_fn(t)

    def initial_state(self):
        x = self.X.copy() if self.x_init is None else self.x_init.copy()
        v = np.zeros_like(x) if self.v_init is None else self.v_init.copy()
        return x, v


def _rotate_face(X, mask, theta, cy=0.5, cz=0.5):
    Y = X.copy()
    y = X[mask, 1] - cy
    z = X[mask, 2] - cz
    c, s = np.cos(theta), np.sin(theta)
    Y[mask, 1] = cy + c * y - s * z
    Y[mask, 2] = cz + s * y + c * z
    return Y


def stretch2d(n=17, E=1e5, nu=0.4, stretch=0.5, rho=1000.0):
    """Quasistatic stretch of the unit square: left edge held at rest, right edge
    moved by +stretch in x (both components prescribed).  The initial guess is
    the rest shape with the right-edge vertices already at their targets."""
    X, tris = grid2d(n, n)
    i = np.arange(X.shape[0]) % n
    left = i == 0
    right = i == n - 1
    fixed = (left | right).astype(np.uint8)
    tgt = X.copy()
    tgt[right, 0] += stretch

    x0 = X.copy()
    x0[right] = tgt[right]
    return Scene(name=f"stretch2d_{n}x{n}", dim=2, X=X, elems=tris, fixed=fixed, E=E, nu=nu,
                 rho=rho, gravity=np.zeros(3), dt=1.0, n_steps=1, quasistatic=True,
                 target_fn=lambda t: tgt.copy(), x_init=x0)


def tet_bar(nx=21, ny=6, nz=6, E=1e5, nu=0.45, rho=1000.0, dt=1.0 / 60, n_steps=10,
            length=(4.0, 1.0, 1.0), gravity=(0.0, -GRAV, 0.0), clamp_face=0,
            twist_per_step=0.0):
    """Tet bar on an nx*ny*nz vertex grid over [0,Lx]x[0,Ly]x[0,Lz].

    clamp_face in 0..5 selects the held face: 0 x=min, 1 x=max, 2 y=min,
    3 y=max, 4 z=min, 5 z=max.  With twist_per_step != 0 the face opposite the
    x=min face (x=max) is also prescribed and rotated about the bar axis by
    twist_per_step*t radians at step t (clamp_face must then be 0).
    """
    X, tets = grid3d(nx, ny, nz, *length)
    n = X.shape[0]
    ids = np.arange(n)
    ii = ids % nx
    jj = (ids // nx) % ny
    kk = ids // (nx * ny)
    faces = [ii == 0, ii == nx - 1, jj == 0, jj == ny - 1, kk == 0, kk == nz - 1]
    fixed = faces[clamp_face].copy()
    target_fn = None
    if twist_per_step != 0.0:
        assert clamp_face == 0
        far = faces[1]
        fixed |= far
        cy, cz = 0.5 * length[1], 0.5 * length[2]
        target_fn = lambda t: _rotate_face(X, far, twist_per_step * t, cy, cz)
    return Scene(name=f"bar_{nx}x{ny}x{nz}", dim=3, X=X, elems=tets,
                 fixed=fixed.astype(np.uint8), E=E, nu=nu, rho=rho,
                 gravity=np.asarray(gravity, dtype=np.float64), dt=dt, n_steps=n_steps,
                 quasistatic=False, target_fn=target_fn,
                 meta=dict(nx=nx, ny=ny, nz=nz, clamp_face=clamp_face,
                           twist_per_step=twist_per_step))


def rod_impulse(nx=41, E=1e3, nu=0.3, rho=1000.0, dt=1.0 / 60, length=1.0, width=0.05, speed=0.1):
    """Free rod [0,length]x[0,width]^2 on an nx*2*2 vertex grid (the 1D rod of
    the paper's stiffness sweep, as a chain of tets): no Dirichlet vertex, no
    gravity; the four vertices of the right end start with velocity -speed
    along x (the impulse), every other vertex at rest.  One step."""
    X, tets = grid3d(nx, 2, 2, length, width, width)
    v0 = np.zeros_like(X)
    v0[np.arange(X.shape[0]) % nx == nx - 1, 0] = -speed
    return Scene(name=f"rod_{nx}x2x2", dim=3, X=X, elems=tets, fixed=np.zeros(X.shape[0], np.uint8),
                 E=E, nu=nu, rho=rho, gravity=np.zeros(3), dt=dt, n_steps=1, quasistatic=False,
                 v_init=v0, meta=dict(nx=nx, speed=speed))


def cantilever_bend(nx=21, ny=6, nz=6, E=1e6, nu=0.45, rho=1000.0, n_steps=20, g_max=GRAV):
    """Quasistatic cantilever (the paper's subspace-quality scene): a tet bar
    over [0,4]x[0,1]x[0,1] clamped at x = 0 and bent by gravity along -y that
    grows linearly to g_max over n_steps load steps (gravity_at(t), t = 1..);
    each step starts from the previous step's solution."""
    s = tet_bar(nx, ny, nz, E=E, nu=nu, rho=rho, dt=1.0, n_steps=n_steps,
                gravity=(0.0, -g_max, 0.0))
    s.name = f"cantilever_{nx}x{ny}x{nz}"
    s.quasistatic = True
    s.meta = dict(s.meta, g_max=g_max)
    s.meta["gravity_at"] = lambda t: np.array([0.0, -g_max * t / n_steps, 0.0])
    return s


def twist_beam(nx=81, ny=21, nz=21, E=1e7, nu=0.45, rho=1000.0, dt=1.0 / 60, n_steps=30,
               total_angle=np.pi / 2):
    """Beam over [0,4]x[0,1]x[0,1]: face x=0 held at rest, face x=4 rotated about
    the axis (y,z) = (0.5,0.5) by total_angle*t/n_steps at step t.  No gravity."""
    return tet_bar(nx, ny, nz, E=E, nu=nu, rho=rho, dt=dt, n_steps=n_steps,
                   gravity=(0.0, 0.0, 0.0), clamp_face=0,
                   twist_per_step=total_angle / n_steps)


def batch_bars(count=64, master_seed=20251012, spacing=0.1, dt=1.0 / 60, n_steps=10):
    """Seed-drawn batch of uneven tet bars: nx ~ U{6..41}, ny, nz ~ U{6..11},
    log10 E ~ U(4,7), nu ~ U(0.3,0.48), held face ~ U{0..5}, gravity 9.81 times a
    uniform unit vector, rho 1000.  Bar b uses seed master_seed + b."""
    out = []
    for b in range(count):
        rng = np.random.default_rng(master_seed + b)
        nx = int(rng.integers(6, 42))
        ny = int(rng.integers(6, 12))
        nz = int(rng.integers(6, 12))
        E = float(10.0 ** rng.uniform(4.0, 7.0))
        nu = float(rng.uniform(0.3, 0.48))
        face = int(rng.integers(0, 6))
        g = rng.normal(size=3)
        g = GRAV * g / np.linalg.norm(g)
        length = ((nx - 1) * spacing, (ny - 1) * spacing, (nz - 1) * spacing)
        s = tet_bar(nx, ny, nz, E=E, nu=nu, rho=1000.0, dt=dt, n_steps=n_steps,
                    length=length, gravity=g, clamp_face=face)
        s.name = f"batch{b}_{nx}x{ny}x{nz}"
        s.meta["seed"] = master_seed + b
        out.append(s)
    return out


def warm_start_train_scene(seed, nx=21, ny=6, nz=6, n_steps=10):
    """Training episode for the learned warm start: a 21x6x6 bar with
    log-uniform E in [1e4,1e7], gravity of random direction and magnitude in
    [0, 2g], and a far-end twist rate drawn in [0, 3] degrees per step."""
    rng = np.random.default_rng(seed)
    E = float(10.0 ** rng.uniform(4.0, 7.0))
    g = rng.normal(size=3)
    g = rng.uniform(0.0, 2.0 * GRAV) * g / np.linalg.norm(g)
    rate = float(np.deg2rad(rng.uniform(0.0, 3.0)))
    s = tet_bar(nx, ny, nz, E=E, nu=0.45, rho=1000.0, dt=1.0 / 60, n_steps=n_steps,
                gravity=g, clamp_face=0, twist_per_step=rate)
    s.name = f"wstrain{seed}"
    s.meta["seed"] = seed
    return s


def warm_start_eval_scene(seed, nx=81, ny=21, nz=21, n_steps=30):
    """Held-out evaluation episode drawn like the training ones at beam size."""
    rng = np.random.default_rng(seed)
    E = float(10.0 ** rng.uniform(4.0, 7.0))
    g = rng.normal(size=3)
    g = rng.uniform(0.0, 2.0 * GRAV) * g / np.linalg.norm(g)
    rate = float(np.deg2rad(rng.uniform(0.0, 3.0)))
    s = tet_bar(nx, ny, nz, E=E, nu=0.45, rho=1000.0, dt=1.0 / 60, n_steps=n_steps,
                gravity=g, clamp_face=0, twist_per_step=rate)
    s.name = f"wseval{seed}"
    s.meta["seed"] = seed
    return s


def mlp_init(seed=7, n_in=32, n_hid=64, n_out=16, n_used_in=16, n_used_out=3):
    """Seeded initial parameters of the warm-start network, packed as
    W1 (n_in x n_hid), b1, W2 (n_hid x n_hid), b2, W3 (n_hid x n_out), b3, all
    row-major float64.  Scaled normal draws (variance 1/fan_in); padding rows
    of W1 and padding columns of W3 are zero; biases zero; W3 scaled by 0.1 so
    that the untrained proposal stays near the inertial predictor."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((n_in, n_hid))
    W1[:n_used_in] = rng.normal(size=(n_used_in, n_hid)) / np.sqrt(n_used_in)
    W2 = rng.normal(size=(n_hid, n_hid)) / np.sqrt(n_hid)
    W3 = np.zeros((n_hid, n_out))
    W3[:, :n_used_out] = 0.1 * rng.normal(size=(n_hid, n_used_out)) / np.sqrt(n_hid)
    return np.concatenate([W1.ravel(), np.zeros(n_hid), W2.ravel(), np.zeros(n_hid), W3.ravel(),
                           np.zeros(n_out)])
