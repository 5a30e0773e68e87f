"""GPU parity of the Fixed Corotational material (Results, Implementation
Details) against the oracle: element gradients and projected Hessians
(closed-form eigensystem on the GPU, exact Sylvester derivative of the polar
rotation in the oracle) at rest, deformed and inverted states; energies,
gradients and CC directions of one sweep; time steps in float64 and
float32-mixed; steps with corotation; the 2D quasistatic stretch; warm-start
features; a batch mixing both materials; and the material switch itself.

Tolerances as in the other parity tests: float64 kernels 1e-10 relative to
the largest entry, float32-mixed 2e-5; converged states rel|dx| <= 1e-6
(float64) and 1e-4 (float32-mixed).
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from ccscenes import rod_impulse, stretch2d, tet_bar
from oracle import mlp as M
from oracle import solvers as S
from oracle.basis import basis_matrix, exact_basis
from oracle.fem import Problem
from oracle.timestep import predictor, step

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


def _fcr(s):
    return dataclasses.replace(s, material="fcr")


def _upload(cg, ctx, s):
    mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
    if s.material == "fcr":
        cg.cc_mesh_set_material(ctx, mid, cg.MATERIAL_FCR)
    return mid


def _rel(a, b, X):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b - X), 1e-300)


def _states(s):
    """Rest, mildly and strongly perturbed states; the strong 3D one holds 83
    inverted elements and a pair of rotation-variant singular values summing
    to 0.027 (close to where the polar rotation has no derivative)."""
    out = []
    for scale, seed in ((0.0, 0), (0.02, 1), (0.08, 4), (0.15, 2)):
        rng = np.random.default_rng(seed)
        out.append(s.X + scale * rng.normal(size=s.X.shape))
    return out


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_element_kernel(cg, ctx, dim, prec):
    s = _fcr(stretch2d(n=9) if dim == 2 else tet_bar(9, 4, 4, E=1e6))
    p = Problem.from_scene(s)
    mid = _upload(cg, ctx, s)
    for x in _states(s):
        ge, He = cg.cc_probe_element(ctx, mid, _t(x), prec, s.m)
        ge, He = ge.cpu().numpy(), He.cpu().numpy()
        ge_o = p.element_gradient(x)
        He_o = p.element_hessian(x)
        tol = 1e-10 if prec == 0 else 2e-5
        fscale = max(np.max(np.abs(ge_o)), p.mu * p.vol.max() * np.abs(p.beta).max())
        assert np.max(np.abs(ge - ge_o)) <= tol * fscale
        assert np.max(np.abs(He - He_o)) <= tol * np.max(np.abs(He_o))


def test_material_switch(cg, ctx):
    """The switch changes the element terms to the selected model and back;
    unknown models are rejected and leave the mesh as it was."""
    s = tet_bar(6, 3, 3, E=1e5)
    p_snh = Problem.from_scene(s)
    p_fcr = Problem.from_scene(_fcr(s))
    x = _states(s)[2]
    mid = _upload(cg, ctx, s)
    for model, p in ((cg.MATERIAL_FCR, p_fcr), (cg.MATERIAL_SNH, p_snh), (cg.MATERIAL_FCR, p_fcr)):
        cg.cc_mesh_set_material(ctx, mid, model)
        ge, _ = cg.cc_probe_element(ctx, mid, _t(x), 0, s.m)
        go = p.element_gradient(x)
        assert np.max(np.abs(ge.cpu().numpy() - go)) <= 1e-10 * np.max(np.abs(go))
    with pytest.raises(cg.CCError) as e:
        cg.cc_mesh_set_material(ctx, mid, 7)
    assert e.value.status == -1          # CC_E_INVALID_ARG
    ge, _ = cg.cc_probe_element(ctx, mid, _t(x), 0, s.m)
    go = p_fcr.element_gradient(x)
    assert np.max(np.abs(ge.cpu().numpy() - go)) <= 1e-10 * np.max(np.abs(go))


@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_directions(cg, ctx, prec):
    """Energy, gradient and CC directions of one Jacobi sweep (exact basis)."""
    s = _fcr(tet_bar(8, 4, 4, E=1e6))
    p = Problem.from_scene(s)
    B = exact_basis(p)
    mid = _upload(cg, ctx, s)
    cg.cc_subspace_upload(ctx, mid, *B, s.dt)
    x0, v0 = s.initial_state()
    xh = predictor(p, x0, v0 + 0.3, s.targets(1))
    x = xh + 0.01 * np.random.default_rng(3).normal(size=xh.shape)
    x[p.fixed] = xh[p.fixed]
    par = cg.cc_params_default(method=cg.METHOD_CC, precision=prec, gravity=s.gravity)
    E, g, dx = cg.cc_probe_sweep(ctx, mid, _t(x), _t(p.x_tilde), s.dt, par)
    g, dx = g.cpu().numpy(), dx.cpu().numpy()
    assert abs(E - p.energy(x)) <= 1e-11 * abs(p.energy(x))
    go = p.gradient(x)
    assert np.max(np.abs(g[p.free] - go)) <= 1e-10 * np.max(np.abs(go))
    dxo, _ = S.local_directions(p, basis_matrix(p, *B), p.hessian(x), go, np.arange(p.free.size), S.CC)
    tol = 1e-9 if prec == 0 else 1e-4
    assert np.max(np.abs(dx[p.free] - dxo)) <= tol * np.max(np.abs(dxo))


def _run_steps(cg, ctx, s, par, op, tol, nsteps):
    p = Problem.from_scene(s)
    B = exact_basis(p)
    mid = _upload(cg, ctx, s)
    cg.cc_subspace_upload(ctx, mid, *B, s.dt)
    x, v = s.initial_state()
    xg, vg = _t(x), _t(v)
    out = []
    for t in range(1, nsteps + 1):
        tg = s.targets(t)
        x, v, res, _ = step(p, x, v, tg, B, op, tol)
        st, it, rg = cg.cc_step(ctx, mid, xg, vg, _t(tg), s.dt, par, tol)
        out.append((res, st, it, rg, x.copy(), xg.cpu().numpy()))
    return out


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("corotate", [0, 1])
def test_twisting_bar_steps(cg, ctx, prec, corotate):
    """Bar whose free end turns 0.3 rad per step, exact basis, Jacobi CC with
    line search, three steps, with and without the corotated basis."""
    s = _fcr(tet_bar(8, 4, 4, E=1e5, twist_per_step=0.3))
    par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, line_search=1, precision=prec,
                               max_iters=300, gravity=s.gravity, corotate=corotate)
    op = S.Params(method=S.CC, sweep=S.JACOBI, line_search=True, max_iters=300, corotate=bool(corotate))
    for res, st, it, rg, xo, xg in _run_steps(cg, ctx, s, par, op, 1e-8 if prec == 0 else 1e-6, 3):
        assert st == cg.CC_OK and res.status == S.OK
        if prec == 0:
            assert it == res.iters
            assert _rel(xg, xo, s.X) <= 1e-6
        else:
            assert abs(it - res.iters) <= 2
            assert _rel(xg, xo, s.X) <= 1e-4


def test_sagging_bar_steps(cg, ctx):
    """21x6x6 bar under gravity (E = 1e5), the benchmark geometry, float64."""
    s = _fcr(tet_bar(E=1e5))
    par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, line_search=1, max_iters=200,
                               gravity=s.gravity)
    op = S.Params(method=S.CC, sweep=S.JACOBI, line_search=True, max_iters=200)
    for res, st, it, rg, xo, xg in _run_steps(cg, ctx, s, par, op, 1e-6, 2):
        assert st == cg.CC_OK and it == res.iters
        assert _rel(xg, xo, s.X) <= 1e-6


def test_stretch2d_quasistatic(cg, ctx):
    """The 2D stretch of the resolution experiment (right edge +50%) with the
    paper's material, CC without line search for a fixed 40 iterations."""
    s = _fcr(stretch2d(n=9))
    par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, line_search=0, max_iters=40,
                               quasistatic=1)
    op = S.Params(method=S.CC, sweep=S.JACOBI, line_search=False, max_iters=40)
    (res, st, it, rg, xo, xg), = _run_steps(cg, ctx, s, par, op, 0.0, 1)
    assert it == res.iters == 40
    assert _rel(xg, xo, s.X) <= 1e-8


def test_features_match_oracle(cg, ctx):
    """Warm-start features carry the material through the diagonal Hessian blocks."""
    s = _fcr(tet_bar(8, 4, 4, E=3e5, twist_per_step=0.05))
    p = Problem.from_scene(s)
    rng = np.random.default_rng(4)
    x = s.X + 0.01 * rng.normal(size=s.X.shape)
    v = 0.3 * rng.normal(size=s.X.shape)
    mid = _upload(cg, ctx, s)
    tg = s.targets(2)
    nf = int((~s.fixed.astype(bool)).sum())
    feat, xt, ell = cg.cc_mlp_features(ctx, mid, _t(x), _t(v), _t(tg), s.dt, nf)
    fo, _ = M.features(p, x, predictor(p, x, v, tg))
    scale = np.maximum(np.abs(fo).max(axis=0), 1e-3)
    assert np.max(np.abs(feat.cpu().numpy() - fo) / scale) <= 1e-5
    fs, _ = M.features(Problem.from_scene(dataclasses.replace(s, material="snh")), x, predictor(p, x, v, tg))
    assert np.max(np.abs(fs - fo)[:, 6:12]) > 1e-6


@pytest.mark.parametrize("prec", [0, 1])
def test_mixed_batch_equals_single_meshes(cg, ctx, prec):
    """A batch of stable neo-Hookean and Fixed Corotational bars: every mesh
    follows its own model and equals its single-mesh step (float64: 1e-10,
    float32-mixed: 1e-5 relative to the displacement)."""
    scenes = [tet_bar(7, 3, 3, E=1e5), _fcr(tet_bar(7, 3, 3, E=1e5)), _fcr(tet_bar(9, 3, 3, E=1e6)),
              tet_bar(9, 3, 3, E=1e6)]
    mids, mids1 = [], []
    for s in scenes:
        B = exact_basis(Problem.from_scene(s))
        for lst in (mids, mids1):
            mid = _upload(cg, ctx, s)
            cg.cc_subspace_upload(ctx, mid, *B, s.dt)
            lst.append(mid)
    cg.cc_batch_tuning(ctx, 16, 2)
    par = cg.cc_params_default(max_iters=200, gravity=scenes[0].gravity, precision=prec)
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
            assert st == sts[k]
            assert it == its[k] if prec == 0 else abs(it - its[k]) <= 1
            a, b = xs[k].cpu().numpy(), xs1[k].cpu().numpy()
            tol = 1e-10 if prec == 0 else 1e-5
            assert np.linalg.norm(a - b) <= tol * max(np.linalg.norm(b - s.X), 1e-3)
    # the two materials give different motions of the same bar
    assert np.linalg.norm(xs[0].cpu().numpy() - xs[1].cpu().numpy()) > 1e-6 * np.linalg.norm(
        xs[0].cpu().numpy() - scenes[0].X)


@pytest.mark.parametrize("E,method", [(1e1, S.CC), (1e6, S.CC), (1e3, S.JGS2), (1e3, S.CD)])
def test_rod_impulse_step(cg, ctx, E, method):
    """One step of the struck free rod of the stiffness sweep (no Dirichlet
    vertex), Jacobi with line search to rel|g| <= 1e-6: equal iterations and
    positions against the oracle."""
    s = _fcr(rod_impulse(E=E))
    gm = {S.CC: cg.METHOD_CC, S.JGS2: cg.METHOD_JGS2, S.CD: cg.METHOD_CD}[method]
    par = cg.cc_params_default(method=gm, sweep=cg.SWEEP_JACOBI, line_search=1, max_iters=500)
    op = S.Params(method=method, sweep=S.JACOBI, line_search=True, max_iters=500)
    (res, st, it, rg, xo, xg), = _run_steps(cg, ctx, s, par, op, 1e-6, 1)
    assert st == cg.CC_OK and res.status == S.OK and it == res.iters
    assert _rel(xg, xo, s.X) <= 1e-6


def test_material_switch_between_batch_calls(cg, ctx):
    """Switching a mesh's material after a batch has run on it: the next
    batched step follows the new model (its result equals the single-mesh
    step with that model, and differs from the old model's)."""
    scenes = [tet_bar(7, 3, 3, E=1e5), tet_bar(7, 3, 3, E=1e6)]
    B = [exact_basis(Problem.from_scene(s)) for s in scenes]
    mids = []
    for s, b in zip(scenes, B):
        mid = _upload(cg, ctx, s)
        cg.cc_subspace_upload(ctx, mid, *b, s.dt)
        mids.append(mid)
    par = cg.cc_params_default(max_iters=200, gravity=scenes[0].gravity)
    x0 = [_t(s.initial_state()[0]) for s in scenes]
    v0 = [_t(s.initial_state()[1]) for s in scenes]
    bcs = [_t(s.targets(1)) for s in scenes]
    xa, va = [x.clone() for x in x0], [v.clone() for v in v0]
    cg.cc_step_batch(ctx, mids, xa, va, bcs, scenes[0].dt, par, 1e-8)          # SNH plan
    cg.cc_mesh_set_material(ctx, mids[1], cg.MATERIAL_FCR)
    xb, vb = [x.clone() for x in x0], [v.clone() for v in v0]
    worst, its, rgs, sts = cg.cc_step_batch(ctx, mids, xb, vb, bcs, scenes[0].dt, par, 1e-8)
    assert worst == cg.CC_OK
    # reference: fresh single meshes with the same materials
    for k, (s, b) in enumerate(zip(scenes, B)):
        s_k = _fcr(s) if k == 1 else s
        mid = _upload(cg, ctx, s_k)
        cg.cc_subspace_upload(ctx, mid, *b, s.dt)
        x, v = x0[k].clone(), v0[k].clone()
        st, it, rg = cg.cc_step(ctx, mid, x, v, bcs[k], s.dt, par, 1e-8)
        assert st == sts[k] and it == its[k]
        ref = x.cpu().numpy()
        assert np.linalg.norm(xb[k].cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref - s.X)
    d_old = np.linalg.norm(xa[1].cpu().numpy() - xb[1].cpu().numpy())
    assert d_old > 1e-6 * np.linalg.norm(xb[1].cpu().numpy() - scenes[1].X)
