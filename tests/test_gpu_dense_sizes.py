"""Every configuration of the exact-basis condensation (Method, Eqs. block,
update and schur; Eq. rotation; Algorithm 1): one Jacobi sweep's CC
directions against the oracle on sampled vertices, with the rows per
workgroup and the chunk of band positions forced through cc_dense_tuning,
and a batch of the largest bars against single-mesh steps.

The 41x7x7 bar has 1,960 free vertices: 16 chunks of 128 positions (the last
holding 40), 8 of 256 (the last 168) or 4 of 512 (the last 424), so the ring
(chunk + band width positions) wraps several times and the tail is ragged.
Rows per workgroup: float64 1 and 2, float32-mixed 1 to 4 (with chunks of
128, two waves take four rows' final sums in turn); chunks 128, 256 and 512;
with and without corotation (rotated band
records and R^T g).  Tolerances: float64 1e-9, float32-mixed 1e-4 of the
largest direction."""
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


@pytest.fixture(scope="module")
def bar(cg, ctx):
    s = tet_bar(41, 7, 7, E=1e6, twist_per_step=0.15)
    p = Problem.from_scene(s)
    mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
    cg.cc_subspace_build(ctx, mid, 0, s.dt, False)
    x0, v0 = s.initial_state()
    xh = predictor(p, x0, v0 + 0.3, s.targets(3))       # far face turned by 0.45 rad
    x = xh + 0.01 * np.random.default_rng(3).normal(size=xh.shape)
    x[p.fixed] = xh[p.fixed]
    rng = np.random.default_rng(17)
    ranks = np.unique(np.concatenate([[0, p.free.size - 1], rng.choice(p.free.size, 22, replace=False)]))
    Um = basis_matrix(p, *exact_basis(p, verts=p.free[ranks]))
    return dict(s=s, p=p, mid=mid, x=x, ranks=ranks, Um=Um)


CONFIGS = [(0, 1, 128), (0, 1, 256), (0, 1, 512), (0, 2, 128), (0, 2, 256), (0, 2, 512),
           (1, 1, 128), (1, 1, 256), (1, 1, 512), (1, 2, 128), (1, 2, 256), (1, 2, 512),
           (1, 3, 128), (1, 3, 256), (1, 3, 512), (1, 4, 128), (1, 4, 256), (1, 4, 512)]


@pytest.mark.parametrize("corot", [0, 1])
@pytest.mark.parametrize("prec,rows,chunk", CONFIGS)
def test_directions_every_configuration(cg, ctx, bar, prec, rows, chunk, corot):
    s, p, x, ranks = bar["s"], bar["p"], bar["x"], bar["ranks"]
    par = cg.cc_params_default(method=cg.METHOD_CC, precision=prec, gravity=s.gravity, corotate=corot)
    cg.cc_dense_tuning(ctx, rows, chunk)
    try:
        _, _, dx = cg.cc_probe_sweep(ctx, bar["mid"], _t(x), _t(p.x_tilde), s.dt, par)
    finally:
        cg.cc_dense_tuning(ctx, 0, 0)
    dx = dx.cpu().numpy()
    Ur = S._basis_at(p, bar["Um"], x, S.Params(method=S.CC, corotate=bool(corot)))
    dxo, _ = S.local_directions(p, Ur, p.hessian(x), p.gradient(x), ranks, S.CC)
    tol = 1e-9 if prec == 0 else 1e-4
    assert np.max(np.abs(dx[p.free[ranks]] - dxo)) <= tol * np.max(np.abs(dxo))


def test_dense_tuning_rejects_bad_values(cg, ctx):
    with pytest.raises(cg.CCError):
        cg.cc_dense_tuning(ctx, 5, 0)
    with pytest.raises(cg.CCError):
        cg.cc_dense_tuning(ctx, 0, 384)
    cg.cc_dense_tuning(ctx, 0, 0)


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
