"""Pins of the oracle's warm-start network and features."""
import numpy as np
import pytest

from ccscenes import mlp_init, tet_bar
from oracle import mlp as M
from oracle.fem import Problem


def _batch(rng, B=7):
    X = np.zeros((B, M.N_IN_PAD))
    X[:, :M.N_IN] = rng.normal(size=(B, M.N_IN))
    T = rng.normal(size=(B, M.N_OUT))
    return X, T


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp_init(3) + 0.05 * rng.normal(size=M.N_PARAMS)   # non-zero padding too
    X, T = _batch(rng)
    Y, cache = M.forward(theta, X)
    loss, dY = M.loss_and_dY(Y, T)
    g = M.backward(theta, cache, dY)
    eps = 1e-6
    idx = rng.choice(M.N_PARAMS, size=200, replace=False)
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        lp = M.loss_and_dY(M.forward(tp, X)[0], T)[0]
        lm = M.loss_and_dY(M.forward(tm, X)[0], T)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    fd = (M.silu(z + 1e-6) - M.silu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(M.dsilu(z), fd, rtol=1e-7, atol=1e-9)


def test_adam_first_step_is_sign_step():
    """With zero moments the first bias-corrected Adam step is lr * sign(g)
    (up to eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = M.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert th[3] == 0.0


def test_features_at_rest_and_affine():
    s = tet_bar(6, 3, 3, E=1e5)
    p = Problem.from_scene(s)
    f, ell = M.features(p, p.X, p.X)
    assert np.allclose(f[:, 0:6], 0.0) and np.allclose(f[:, 12:14], 0.0)
    assert np.allclose(f[:, 14], 1.0) and np.allclose(f[:, 15], 0.0, atol=1e-12)
    # uniform translation: relative displacement and strain features vanish,
    # velocity feature equals the translation / l
    t = np.array([0.1, -0.2, 0.05])
    xt = p.X + t
    f, ell = M.features(p, p.X, xt)
    assert np.allclose(f[:, 0:3], 0.0, atol=1e-12)
    assert np.allclose(f[:, 3:6], t / ell)
    # uniform scaling by s: J = s^3, |F|^2 - 3 = 3 s^2 - 3
    sc = 1.1
    f, _ = M.features(p, p.X, p.X * sc)
    assert np.allclose(f[:, 14], sc ** 3) and np.allclose(f[:, 15], 3 * sc * sc - 3)
    # diagonal Hessian block: mass-dominated limit at h -> 0 gives I m/(m) = identity upper triangle
    p.h = 1e-9
    f, _ = M.features(p, p.X, p.X)
    assert np.allclose(f[:, 6:12], [1, 0, 0, 1, 0, 1], atol=1e-9)


def test_proposal_adds_previous_correction_on_free_vertices():
    """x_p = x~ + c + l Delta on free vertices, x~ on Dirichlet ones."""
    from ccscenes import tet_bar
    from oracle.fem import Problem
    s = tet_bar(5, 3, 3)
    p = Problem.from_scene(s)
    rng = np.random.default_rng(2)
    xt = s.X + 0.01 * rng.normal(size=s.X.shape)
    corr = rng.normal(size=s.X.shape)
    Delta = rng.normal(size=(p.free.size, 16))
    xp = M.proposal(p, xt, Delta, 0.5, corr)
    np.testing.assert_array_equal(xp[p.fixed], xt[p.fixed])
    np.testing.assert_allclose(xp[p.free], xt[p.free] + corr[p.free] + 0.5 * Delta[:, :3], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(M.proposal(p, xt, Delta, 0.5), M.proposal(p, xt, Delta, 0.5, np.zeros_like(xt)))
