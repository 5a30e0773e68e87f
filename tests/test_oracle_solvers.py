"""Pins of the oracle's Coordinate Condensation, CD, line search and Newton."""
import numpy as np
import pytest
import scipy.sparse as sp

from ccscenes import stretch2d, tet_bar
from oracle import solvers as S
from oracle.basis import basis_matrix, exact_basis, patch_basis
from oracle.colour import greedy_colour
from oracle.fem import Problem
from oracle.timestep import newton_step, step
from tests.quadratic import QuadraticProblem, random_spd_chain, spring_rod


def _exact_basis_dense(K, d):
    """Exact basis straight from U_i = -K_CC^{-1} K_Ci, as (ptr, idx, U)."""
    K = K.toarray()
    nv = K.shape[0] // d
    ptr = [0]
    idx, U = [], []
    for i in range(nv):
        C = [j for j in range(nv) if j != i]
        cd = np.concatenate([np.arange(j * d, j * d + d) for j in C])
        idd = np.arange(i * d, i * d + d)
        Ui = -np.linalg.solve(K[np.ix_(cd, cd)], K[np.ix_(cd, idd)])
        idx += C
        U.append(Ui.reshape(len(C), d, d))
        ptr.append(ptr[-1] + len(C))
    return np.array(ptr), np.array(idx, dtype=np.int32), np.concatenate(U)


def _quadratic_cases():
    rng = np.random.default_rng(0)
    out = []
    H, fixed = spring_rod(12, k=1e5, m=0.1, h=1 / 60)     # the paper's quadratic rod
    n = fixed.size
    c = rng.normal(size=n - 1)
    out.append(QuadraticProblem(H, n, 1, fixed=fixed, c=c))
    K = random_spd_chain(9, 3, rng)
    out.append(QuadraticProblem(K, 9, 3, c=rng.normal(size=27)))
    s = tet_bar(5, 3, 3, E=1e6)
    p = Problem.from_scene(s)
    Kfem = p.hessian(p.X)                                 # linear elasticity + mass
    out.append(QuadraticProblem(Kfem, p.n, 3, fixed=s.fixed, c=rng.normal(size=p.ndof)))
    return out


def test_chol_solve():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(30, 3, 3))
    M = np.einsum("kij,klj->kil", A, A) + 0.1 * np.eye(3)
    B = rng.normal(size=(30, 3, 2))
    X, ok = S.chol_solve(M, B)
    assert ok.all()
    np.testing.assert_allclose(X, np.linalg.solve(M, B), rtol=1e-10, atol=1e-12)
    M[0] = np.diag([1.0, 1.0, 0.0])
    _, ok = S.chol_solve(M, B)
    assert not ok[0] and ok[1:].all()


def _block_system_direction(K, U_cols, g, i, d):
    """dx_i from a direct solve of the coupled block system (Method, Eq. block)."""
    nd = K.shape[0]
    Bi = np.zeros((nd, 2 * d))
    Bi[i * d:(i + 1) * d, :d] = np.eye(d)
    Bi[:, d:] = U_cols
    q = np.linalg.solve(Bi.T @ K @ Bi, -Bi.T @ g)
    return q[:d]


@pytest.mark.parametrize("case", [0, 1, 2])
def test_schur_equals_block_solve(case):
    """The Schur-condensed update equals the first block of the 2d x 2d solve,
    for a generic (here: random) basis, not only the exact one."""
    p = _quadratic_cases()[case]
    d = p.d
    rng = np.random.default_rng(case)
    K = p.K
    nf = p.free.size
    # random supports and blocks
    ptr, idx, U = [0] * (p.n + 1), [], []
    for i in p.free:
        C = [int(j) for j in p.free if j != i and rng.uniform() < 0.6]
        ptr[i + 1] = len(C)
        idx += C
        U.append(rng.normal(size=(len(C), d, d)))
    ptr = np.cumsum(ptr)
    idx = np.array(idx, dtype=np.int32)
    U = np.concatenate(U)
    Um = basis_matrix(p, ptr, idx, U)
    x = p.X + rng.normal(size=p.X.shape)
    g = p.gradient(x)
    dx, counts = S.local_directions(p, Um, K, g, np.arange(nf), S.CC)
    assert counts.sum() == 0
    Ud = Um.toarray()
    for fi in range(nf):
        want = _block_system_direction(K.toarray(), Ud[:, fi * d:(fi + 1) * d], g.ravel(), fi, d)
        assert np.max(np.abs(dx[fi] - want)) <= 1e-8 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("case", [0, 1, 2])
@pytest.mark.parametrize("sweep", [S.JACOBI, S.GS])
def test_cc_exact_basis_is_newton_on_quadratics(case, sweep):
    """With the exact basis CC takes the Newton step: one iteration converges."""
    p = _quadratic_cases()[case]
    d = p.d
    B = _exact_basis_dense(p.K, d)
    # the dense construction above is over free ranks; map to vertex ids
    ptr = np.zeros(p.n + 1, dtype=np.int64)
    ptr[p.free + 1] = np.diff(B[0])
    B = (np.cumsum(ptr), p.free[B[1]].astype(np.int32), B[2])
    col = greedy_colour(p.n, _edges_as_elems(p), p.fixed)
    x0 = p.X.copy()
    newton_x = x0.copy()
    newton_x[p.free] += np.linalg.solve(p.K.toarray(), p.c).reshape(-1, d)
    prm = S.Params(method=S.CC, sweep=sweep, line_search=False, max_iters=1)
    res = S.solve(p, x0, B, prm, tol=0.0, colours=col)
    assert res.iters == 1
    scale = np.max(np.abs(newton_x - x0))
    assert np.max(np.abs(res.x - newton_x)) <= 1e-9 * scale
    assert res.rel_grad <= 1e-9


def _edges_as_elems(p):
    adj = p.adjacency()
    return np.array([(i, j) for i in range(p.n) for j in adj[i] if j > i] or [(0, 0)])


@pytest.mark.parametrize("sweep", [S.JACOBI, S.GS])
def test_cd_is_textbook_block_relaxation(sweep):
    rng = np.random.default_rng(4)
    K = random_spd_chain(8, 3, rng, coupling=0.3)
    p = QuadraticProblem(K, 8, 3, c=rng.normal(size=24))
    col = greedy_colour(p.n, _edges_as_elems(p), p.fixed)
    x = p.X + rng.normal(size=p.X.shape)
    prm = S.Params(method=S.CD, sweep=sweep, line_search=False)
    x_new, _ = S.sweep(p, x, None, col, prm)
    Kd = K.toarray()
    u = (x - p.X).ravel()
    if sweep == S.JACOBI:
        want = u.copy()
        r = Kd @ u - p.c
        for i in range(8):
            sl = slice(3 * i, 3 * i + 3)
            want[sl] -= np.linalg.solve(Kd[sl, sl], r[sl])
    else:
        want = u.copy()
        for c in range(col.max() + 1):
            r = Kd @ want - p.c
            upd = {}
            for i in np.flatnonzero(col == c):
                sl = slice(3 * i, 3 * i + 3)
                upd[i] = np.linalg.solve(Kd[sl, sl], r[sl])
            for i, v in upd.items():
                want[3 * i:3 * i + 3] -= v
    np.testing.assert_allclose((x_new - p.X).ravel(), want, rtol=1e-11, atol=1e-12)


def test_jgs2_printed_form():
    """JGS2: dx_i = -(H_ii + U^T H_CC U)^{-1}(g_i + U^T g_C) (Background, JGS2)."""
    p = _quadratic_cases()[1]
    d = 3
    B = _exact_basis_dense(p.K, d)
    Um = basis_matrix(p, *B)
    rng = np.random.default_rng(9)
    x = p.X + rng.normal(size=p.X.shape)
    g = p.gradient(x)
    dx, _ = S.local_directions(p, Um, p.K, g, np.arange(9), S.JGS2)
    Kd = p.K.toarray()
    Ud = Um.toarray()
    for i in range(9):
        sl = slice(3 * i, 3 * i + 3)
        Ui = Ud[:, sl]
        want = -np.linalg.solve(Kd[sl, sl] + Ui.T @ Kd @ Ui, g.ravel()[sl] + Ui.T @ g.ravel())
        np.testing.assert_allclose(dx[i], want, rtol=1e-9, atol=1e-12)


def test_line_search_never_raises_energy():
    s = stretch2d(n=9)
    p = Problem.from_scene(s)
    B = patch_basis(p, 1)
    col = greedy_colour(p.n, p.elems, p.fixed)
    x0, v0 = s.initial_state()
    for sweep in (S.JACOBI, S.GS):
        prm = S.Params(method=S.CC, sweep=sweep, line_search=True, max_iters=15)
        _, _, res, _ = step(p, x0, v0, s.targets(1), B, prm, 1e-12, colours=col, record=True)
        E = np.array([h[1] for h in res.history])
        tau = 1e-12 * np.maximum(np.abs(E[:-1]), 1.0)
        assert np.all(E[1:] <= E[:-1] + tau)


def test_cc_converges_to_newton_minimiser_2d():
    s = stretch2d(n=9)
    p = Problem.from_scene(s)
    B = exact_basis(p)
    x0, v0 = s.initial_state()
    xn, _, rn = newton_step(p, x0, v0, s.targets(1), tol=1e-11)
    prm = S.Params(method=S.CC, sweep=S.JACOBI, line_search=True, max_iters=200)
    xc, _, rc, _ = step(p, x0, v0, s.targets(1), B, prm, 1e-11)
    assert rn.rel_grad <= 1e-11 and rc.rel_grad <= 1e-11
    assert np.linalg.norm(xc - xn) / np.linalg.norm(xn - p.X) <= 1e-6


@pytest.mark.parametrize("sweep", [S.JACOBI, S.GS])
def test_cc_converges_to_newton_minimiser_3d_dynamic(sweep):
    s = tet_bar(7, 3, 3, E=1e6)
    p = Problem.from_scene(s)
    B = exact_basis(p)
    col = greedy_colour(p.n, p.elems, p.fixed)
    x, v = s.initial_state()
    xn, vn, rn = newton_step(p, x, v, s.targets(1), tol=1e-11)
    prm = S.Params(method=S.CC, sweep=sweep, line_search=(sweep == S.JACOBI), max_iters=100)
    xc, vc, rc, _ = step(p, x, v, s.targets(1), B, prm, 1e-11, colours=col)
    assert rc.status == S.OK and rc.iters <= 10
    assert np.linalg.norm(xc - xn) / np.linalg.norm(xn - p.X) <= 1e-6


def test_qualitative_ordering_on_stretch():
    """CC well ahead of JGS2, JGS2 ahead of CD after a fixed budget (teaser,
    Mesh Resolution Scaling)."""
    s = stretch2d(n=9)
    p = Problem.from_scene(s)
    B = exact_basis(p)
    x0, v0 = s.initial_state()
    r = {}
    for name, m in (("cc", S.CC), ("jgs2", S.JGS2), ("cd", S.CD)):
        prm = S.Params(method=m, sweep=S.JACOBI, line_search=True, max_iters=20)
        _, _, res, _ = step(p, x0, v0, s.targets(1), B, prm, 0.0)
        r[name] = res.rel_grad
    assert r["cc"] < 1e-3 * r["jgs2"] and r["jgs2"] < r["cd"]
