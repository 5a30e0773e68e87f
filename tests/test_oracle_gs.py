"""Coloured Gauss-Seidel with the global energy test on the sweep's
displacement (the oracle's reading of the line search for that
sweep): the energy never rises from one iteration to the next, the
iteration reaches Newton's minimiser on a stiff bar in a handful of sweeps,
and with a basis so poor that its condensed steps raise E the search (with
its coordinate-descent fallback) still never raises it.  A coloured sweep of
CC is taken at its full step only; when that raises E the iteration takes a
Jacobi sweep of the same method with the search."""
from dataclasses import replace

import numpy as np

from ccscenes import stretch2d, tet_bar
from oracle import solvers as S
from oracle.basis import basis_matrix, exact_basis, patch_basis
from oracle.colour import greedy_colour
from oracle.fem import Problem
from oracle.timestep import predictor, step


def _monotone(res):
    E = np.array([h[1] for h in res.history])
    return np.all(E[1:] <= E[:-1] + 1e-12 * np.maximum(np.abs(E[:-1]), 1.0))


def test_gs_search_reaches_newton_minimiser_stiff():
    """E = 1e7, exact basis: searched Gauss-Seidel converges to the minimiser
    that a sparse-direct Newton solve finds (rel |dx| <= 1e-6), monotonically."""
    s = tet_bar(7, 3, 3, E=1e7)
    p = Problem.from_scene(s)
    B = exact_basis(p)
    col = greedy_colour(p.n, p.elems, p.fixed)
    x, v = s.initial_state()
    xt = predictor(p, x, v, s.targets(1))
    p.set_inertial_target(xt)
    xn = S.newton(p, xt, tol=1e-12, x_hat0=xt).x
    prm = S.Params(method=S.CC, sweep=S.GS, line_search=True, max_iters=200)
    xc, _, rc, _ = step(p, x, v, s.targets(1), B, prm, 1e-10, colours=col, record=True)
    assert rc.status == S.OK and rc.iters <= 10
    assert np.linalg.norm(xc - xn) / np.linalg.norm(xn - p.X) <= 1e-6
    assert _monotone(rc)


def test_gs_search_with_a_bad_basis_never_raises_energy():
    """A basis with large random errors: the energy still never rises, and the
    search and its coordinate-descent fallback still converge."""
    s = stretch2d(n=7)
    p = Problem.from_scene(s)
    ptr, idx, U = patch_basis(p, 2)
    rng = np.random.default_rng(3)
    U = U + 2.0 * rng.normal(size=U.shape)
    col = greedy_colour(p.n, p.elems, p.fixed)
    x0, v0 = s.initial_state()
    prm = S.Params(method=S.CC, sweep=S.GS, line_search=True, max_iters=3000)
    _, _, res, _ = step(p, x0, v0, s.targets(1), (ptr, idx, U), prm, 1e-6, colours=col, record=True)
    assert _monotone(res)
    assert res.status == S.OK


def test_gs_full_step_or_jacobi_fallback():
    """A coloured sweep is taken at its full step only, else the iteration
    takes the Jacobi sweep.  Cantilevers 8x4x4 at E = 1e7 under gravity -y:
    held at x = min, the first coloured sweep from the predictor raises E (its
    search would need four halvings) while the Jacobi sweep does not, so the
    first iterate is x + d_J; held at y = min, the coloured sweep's full step
    lowers E and the first iterate is x + d_GS.  Whether a step raises E is
    found here by evaluating E along each displacement."""
    for face, gs_passes in ((0, False), (2, True)):
        s = tet_bar(8, 4, 4, E=1e7, length=(0.7, 0.3, 0.3), clamp_face=face)
        p = Problem.from_scene(s)
        B = exact_basis(p)
        col = greedy_colour(p.n, p.elems, p.fixed)
        cf = np.asarray(col)[p.free]
        x, v = s.initial_state()
        xt = predictor(p, x, v, s.targets(1))
        p.set_inertial_target(xt)
        U = basis_matrix(p, *B)
        prm = S.Params(method=S.CC, sweep=S.GS, line_search=True, max_iters=1, corotate=True)
        d_gs = S.sweep(p, xt, U, cf, prm)[0] - xt
        d_j = S.sweep(p, xt, U, cf, replace(prm, sweep=S.JACOBI))[0] - xt
        E0 = p.energy(xt)
        slack = 1e-12 * max(abs(E0), 1.0)
        assert (p.energy(xt + d_gs) <= E0 + slack) == gs_passes
        assert p.energy(xt + d_j) <= E0 + slack
        if not gs_passes:
            assert p.energy(xt + d_gs / 16.0) <= E0 + slack   # a search would have taken d_GS/16
        xo, _, res, _ = step(p, x, v, s.targets(1), B, prm, 1e-12, colours=col)
        expect = xt + (d_gs if gs_passes else d_j)
        assert np.linalg.norm(xo - expect) <= 1e-12 * np.linalg.norm(d_j), face
        assert res.sweep_fallbacks == (0 if gs_passes else 1)
