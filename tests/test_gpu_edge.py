"""GPU parity on the degenerate cases of the method, against the oracle:
no free vertex (zero gradient: converged in zero iterations), a single free
vertex in 2D and 3D (empty basis: the coordinate-descent fallback), a body at
rest, a one-cell bar, and a batch that mixes a converged mesh with iterating
ones."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from ccscenes import tet_bar
from ccscenes.scenes import Scene
from oracle import solvers as S
from oracle.basis import exact_basis
from oracle.fem import Problem
from oracle.timestep import step

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def cg():
    import paper_2510_12053_amd.ccgpu as cg
    cg.lib()
    return cg


@pytest.fixture(scope="module")
def ctx(cg):
    c = cg.cc_create(0, torch.cuda.Stream(device=DEV))
    yield c
    cg.cc_destroy(c)


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _simplex(dim, fixed, gravity=(0.0, -9.81, 0.0), shift=None):
    """One triangle / tet with the given Dirichlet flags; targets move the
    fixed vertices by `shift` (per step)."""
    X = np.vstack([np.zeros(dim), np.eye(dim)]) * 0.5
    el = np.arange(dim + 1, dtype=np.int32)[None, :]
    fx = np.asarray(fixed, dtype=np.uint8)
    tf = None
    if shift is not None:
        def tf(t, X=X, fx=fx):
            Y = X.copy()
            Y[fx.astype(bool)] += t * np.asarray(shift)[:dim]
            return Y
    return Scene(name=f"simplex{dim}", dim=dim, X=X, elems=el, fixed=fx, E=1e5, nu=0.4, rho=1000.0,
                 gravity=np.asarray(gravity, dtype=np.float64), dt=1.0 / 60, n_steps=3,
                 quasistatic=False, target_fn=tf)


def _steps(cg, ctx, s, nsteps, basis_kind="exact"):
    p = Problem.from_scene(s)
    B = exact_basis(p)
    mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
    cg.cc_subspace_upload(ctx, mid, *B, s.dt)
    x, v = s.initial_state()
    xg, vg = _t(x), _t(v)
    op = S.Params(method=S.CC, sweep=S.JACOBI, line_search=True, max_iters=200)
    par = cg.cc_params_default(gravity=s.gravity, max_iters=200)
    out = []
    for t in range(1, nsteps + 1):
        tg = s.targets(t)
        x, v, res, _ = step(p, x, v, tg, B, op, 1e-8)
        st, it, rg = cg.cc_step(ctx, mid, xg, vg, _t(tg), s.dt, par, 1e-8)
        out.append((res, st, it, x.copy(), v.copy(), xg.cpu().numpy(), vg.cpu().numpy()))
    return p, out


def test_no_free_vertex(cg, ctx):
    """Every vertex prescribed: zero iterations, positions are the targets and
    velocities their finite differences."""
    s = _simplex(3, [1, 1, 1, 1], shift=(0.01, 0.0, -0.02))
    p, out = _steps(cg, ctx, s, 2)
    for res, st, it, x, v, xg, vg in out:
        assert st == cg.CC_OK and it == 0 and res.iters == 0
        np.testing.assert_array_equal(xg, x)
        np.testing.assert_allclose(vg, v, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_single_free_vertex(cg, ctx, dim):
    """One free vertex: its exact basis is empty, so CC takes the
    coordinate-descent step (a block Newton step), as in the oracle."""
    s = _simplex(dim, [1] * dim + [0], shift=(0.02, 0.01, 0.0))
    p, out = _steps(cg, ctx, s, 3)
    for res, st, it, x, v, xg, vg in out:
        assert st == cg.CC_OK and it == res.iters
        assert np.linalg.norm(xg - x) <= 1e-10 * max(np.linalg.norm(x - s.X), 1e-3)
        np.testing.assert_allclose(vg, v, rtol=0, atol=1e-8)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("batched", [False, True])
def test_rest_stays_at_rest(cg, ctx, prec, batched):
    """At rest, no gravity, targets at rest: the predictor is the rest state
    and its gradient is rounding noise (F = I only to rounding with spacings
    of 0.1).  The convergence test's floor (1e-8 of the elastic force scale)
    makes the step converge with no iteration, as in the oracle: status OK,
    zero iterations, positions and velocities exactly at rest."""
    s = tet_bar(7, 3, 3, E=1e6, gravity=(0.0, 0.0, 0.0), length=(0.7, 0.3, 0.3))
    p = Problem.from_scene(s)
    B = exact_basis(p)
    mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
    cg.cc_subspace_upload(ctx, mid, *B, s.dt)
    x, v = s.initial_state()
    xg, vg = _t(x), _t(v)
    op = S.Params(method=S.CC, sweep=S.JACOBI, line_search=True, max_iters=5)
    par = cg.cc_params_default(gravity=s.gravity, max_iters=5, precision=prec)
    for t in (1, 2):
        x, v, res, _ = step(p, x, v, s.targets(t), B, op, 1e-6)
        assert res.status == S.OK and res.iters == 0
        if batched:
            _, its, _, sts = cg.cc_step_batch(ctx, [mid], [xg], [vg], [_t(s.targets(t))], s.dt, par, 1e-6,
                                              gravity=s.gravity[None, :])
            st, it = int(sts[0]), int(its[0])
        else:
            st, it, rg = cg.cc_step(ctx, mid, xg, vg, _t(s.targets(t)), s.dt, par, 1e-6)
        assert st == cg.CC_OK and it == 0, (t, st, it)
        assert np.array_equal(xg.cpu().numpy(), s.X) and np.array_equal(x, s.X)
        assert not np.any(vg.cpu().numpy())


def test_one_cell_bar(cg, ctx):
    """A 2x2x2 vertex bar (one hex, six tets) with one face held."""
    s = tet_bar(2, 2, 2, E=1e6)
    p, out = _steps(cg, ctx, s, 3)
    for res, st, it, x, v, xg, vg in out:
        assert st == cg.CC_OK and it == res.iters
        assert np.linalg.norm(xg - x) <= 1e-6 * np.linalg.norm(x - s.X)


def test_batch_with_converged_mesh(cg, ctx):
    """A batch holding a mesh with no free vertex (zero gradient: converged
    in zero iterations) next to meshes that iterate, one of them with a
    single free vertex: each equals its single-mesh step."""
    scenes = [_simplex(3, [1, 1, 1, 1], shift=(0.01, 0.0, 0.0)), tet_bar(7, 3, 3, E=1e5),
              _simplex(3, [1, 1, 1, 0], shift=(0.02, 0.0, 0.0))]
    mids, mids1 = [], []
    for s in scenes:
        B = exact_basis(Problem.from_scene(s))
        for lst in (mids, mids1):
            mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
            cg.cc_subspace_upload(ctx, mid, *B, s.dt)
            lst.append(mid)
    cg.cc_batch_tuning(ctx, 16, 2)
    par = cg.cc_params_default(max_iters=200)
    xs = [_t(s.initial_state()[0]) for s in scenes]
    vs = [_t(s.initial_state()[1]) for s in scenes]
    xs1 = [x.clone() for x in xs]
    vs1 = [v.clone() for v in vs]
    grav = np.stack([s.gravity for s in scenes])
    for t in (1, 2):
        bcs = [_t(s.targets(t)) for s in scenes]
        worst, its, rgs, sts = cg.cc_step_batch(ctx, mids, xs, vs, bcs, scenes[0].dt, par, 1e-8,
                                                gravity=grav)
        assert worst == cg.CC_OK and its[0] == 0
        for k, s in enumerate(scenes):
            par1 = cg.cc_params_default(max_iters=200, gravity=s.gravity)
            st, it, rg = cg.cc_step(ctx, mids1[k], xs1[k], vs1[k], bcs[k], s.dt, par1, 1e-8)
            assert st == sts[k] and it == its[k]
            a, b = xs[k].cpu().numpy(), xs1[k].cpu().numpy()
            assert np.linalg.norm(a - b) <= 1e-10 * max(np.linalg.norm(b - s.X), 1e-3)


def test_batch_with_non_finite_input(cg, ctx):
    """A batch in which one mesh gets a non-finite position fails with
    CC_E_NONFINITE and leaves the caller's arrays as they were; the next
    batched step of valid inputs equals single-mesh stepping."""
    scenes = [tet_bar(6, 3, 3, E=1e5), tet_bar(7, 3, 3, E=1e6)]
    mids, mids1 = [], []
    for s in scenes:
        B = exact_basis(Problem.from_scene(s))
        for lst in (mids, mids1):
            mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
            cg.cc_subspace_upload(ctx, mid, *B, s.dt)
            lst.append(mid)
    par = cg.cc_params_default(max_iters=200, gravity=scenes[0].gravity)
    xs = [_t(s.initial_state()[0]) for s in scenes]
    vs = [_t(s.initial_state()[1]) for s in scenes]
    bcs = [_t(s.targets(1)) for s in scenes]
    bad = xs[1].clone()
    bad[4, 2] = float("nan")
    xb = [xs[0].clone(), bad]
    vb = [v.clone() for v in vs]
    with pytest.raises(cg.CCError) as ei:
        cg.cc_step_batch(ctx, mids, xb, vb, bcs, scenes[0].dt, par, 1e-8)
    assert ei.value.status == -5
    np.testing.assert_array_equal(xb[0].cpu().numpy(), xs[0].cpu().numpy())
    np.testing.assert_array_equal(vb[0].cpu().numpy(), vs[0].cpu().numpy())
    xa, va = [x.clone() for x in xs], [v.clone() for v in vs]
    worst, its, rgs, sts = cg.cc_step_batch(ctx, mids, xa, va, bcs, scenes[0].dt, par, 1e-8)
    assert worst == cg.CC_OK
    for k, s in enumerate(scenes):
        x1, v1 = xs[k].clone(), vs[k].clone()
        st, it, rg = cg.cc_step(ctx, mids1[k], x1, v1, bcs[k], s.dt, par, 1e-8)
        assert st == sts[k] and it == its[k]
        assert np.linalg.norm(xa[k].cpu().numpy() - x1.cpu().numpy()) <= 1e-10 * np.linalg.norm(
            x1.cpu().numpy() - s.X)
