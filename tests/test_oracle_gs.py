"""Coloured Gauss-Seidel with the global backtracking search along the
sweep's displacement (the oracle's reading of the line search for that
sweep): the energy never rises from one iteration to the next, the
iteration reaches Newton's minimiser on a stiff bar in a handful of sweeps,
and with a basis so poor that its condensed steps raise E the search (with
its coordinate-descent fallback) still never raises it."""
import numpy as np

from ccscenes import stretch2d, tet_bar
from oracle import solvers as S
from oracle.basis import exact_basis, patch_basis
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
