"""The exact-basis condensation at the mesh sizes where fewer basis rows fit
in a workgroup's LDS (Method, Eqs. update and schur; Algorithm 1): one
Jacobi sweep's CC directions against the oracle on sampled vertices, for
every vertices-per-workgroup count the kernel instantiates, and a batch of
the largest bars against single-mesh steps.

Rows per workgroup (160 KB of LDS, 512 threads):
  31x6x6 bar, 1,080 free vertices: float64 2, float32-mixed 4;
  35x6x6 bar, 1,224 free vertices: float64 1, float32-mixed 3;
  41x7x7 bar, 1,960 free vertices: float64 1 (near its limit), float32-mixed 2.
Tolerances: float64 1e-9, float32-mixed 1e-4 of the largest direction."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from ccscenes import tet_bar
from oracle import solvers as S
from oracle.basis import basis_matrix, exact_basis
from oracle.fem import Problem
from oracle.timestep import predictor

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def cg():
    import paper_2510_12053_amd.ccgpu as cg
    cg.lib()
    return cg


@pytest.fixture(scope="module")
def ctx(cg):
    c = cg.cc_create(0)
    yield c
    cg.cc_destroy(c)


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("shape", [(31, 6, 6), (35, 6, 6), (41, 7, 7)])
@pytest.mark.parametrize("prec", [0, 1])
def test_directions_at_large_sizes(cg, ctx, shape, prec):
    s = tet_bar(*shape, E=1e6)
    p = Problem.from_scene(s)
    mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
    cg.cc_subspace_build(ctx, mid, 0, s.dt, False)
    x0, v0 = s.initial_state()
    xh = predictor(p, x0, v0 + 0.3, s.targets(1))
    x = xh + 0.01 * np.random.default_rng(3).normal(size=xh.shape)
    x[p.fixed] = xh[p.fixed]
    par = cg.cc_params_default(method=cg.METHOD_CC, precision=prec, gravity=s.gravity)
    E, g, dx = cg.cc_probe_sweep(ctx, mid, _t(x), _t(p.x_tilde), s.dt, par)
    dx = dx.cpu().numpy()
    # sampled free vertices, the first and the last included
    rng = np.random.default_rng(17)
    ranks = np.unique(np.concatenate([[0, p.free.size - 1], rng.choice(p.free.size, 22, replace=False)]))
    B = exact_basis(p, verts=p.free[ranks])
    dxo, _ = S.local_directions(p, basis_matrix(p, *B), p.hessian(x), p.gradient(x), ranks, S.CC)
    tol = 1e-9 if prec == 0 else 1e-4
    assert np.max(np.abs(dx[p.free[ranks]] - dxo)) <= tol * np.max(np.abs(dxo))


def test_batch_of_largest_bars(cg, ctx):
    """Two 41x7x7 bars (one basis row per float64 workgroup) stepped as a
    batch equal the same bars stepped one at a time."""
    scenes = [tet_bar(41, 7, 7, E=1e5), tet_bar(41, 7, 7, E=1e6)]
    mids, mids1 = [], []
    for s in scenes:
        for lst in (mids, mids1):
            mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
            cg.cc_subspace_build(ctx, mid, 0, s.dt, False)
            lst.append(mid)
    par = cg.cc_params_default(max_iters=200, gravity=scenes[0].gravity)
    xs = [_t(s.initial_state()[0]) for s in scenes]
    vs = [_t(s.initial_state()[1]) for s in scenes]
    xs1 = [x.clone() for x in xs]
    vs1 = [v.clone() for v in vs]
    for t in (1, 2):
        bcs = [_t(s.targets(t)) for s in scenes]
        worst, its, rgs, sts = cg.cc_step_batch(ctx, mids, xs, vs, bcs, scenes[0].dt, par, 1e-8)
        assert worst == cg.CC_OK
        for k, s in enumerate(scenes):
            st, it, rg = cg.cc_step(ctx, mids1[k], xs1[k], vs1[k], bcs[k], s.dt, par, 1e-8)
            assert st == sts[k] and it == its[k]
            a, b = xs[k].cpu().numpy(), xs1[k].cpu().numpy()
            assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b - s.X)
