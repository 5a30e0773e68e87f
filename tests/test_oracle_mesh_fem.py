"""Pins of the oracle's rest data, element terms and global energy derivatives."""
import numpy as np
import pytest

from ccscenes import grid2d, grid3d, stretch2d, tet_bar, twist_beam
from oracle.fem import Problem
from oracle.mesh import MeshError, deformation_gradient, rest_data


def test_counts_and_volume():
    X, T = grid2d(17, 17)
    assert (X.shape[0], T.shape[0]) == (289, 512)
    beta, vol = rest_data(X, T)
    assert vol.min() > 0 and abs(vol.sum() - 1.0) < 1e-13
    X, T = grid3d(21, 6, 6, 4.0, 1.0, 1.0)
    assert (X.shape[0], T.shape[0]) == (756, 3000)
    beta, vol = rest_data(X, T)
    assert vol.min() > 0 and abs(vol.sum() - 4.0) < 1e-12
    s = twist_beam()
    assert (s.n, s.m) == (35721, 192000)


def test_rest_deformation_gradient_is_identity():
    for X, T in (grid2d(5, 4, 2.0, 1.0), grid3d(4, 3, 3, 1.0, 0.5, 0.7)):
        beta, vol = rest_data(X, T)
        F = deformation_gradient(X, T, beta)
        np.testing.assert_allclose(F, np.broadcast_to(np.eye(X.shape[1]), F.shape), atol=1e-13)
        # an affine map x = A X + t gives F = A
        A = np.eye(X.shape[1]) + 0.3 * np.arange(X.shape[1] ** 2).reshape(X.shape[1], -1) / 9
        F = deformation_gradient(X @ A.T + 0.1, T, beta)
        np.testing.assert_allclose(F, np.broadcast_to(A, F.shape), atol=1e-12)


def test_inverted_element_rejected():
    X, T = grid2d(3, 3)
    T = T.copy()
    T[0, [1, 2]] = T[0, [2, 1]]
    with pytest.raises(MeshError):
        rest_data(X, T)


def test_total_mass():
    s = tet_bar(7, 3, 3, rho=800.0)
    p = Problem.from_scene(s)
    assert abs(p.mass.sum() - 800.0 * 4.0) < 1e-9


def _perturbed(p, rng, scale):
    return p.X + scale * rng.normal(size=p.X.shape)


@pytest.mark.parametrize("quasi", [False, True])
@pytest.mark.parametrize("dim", [2, 3])
def test_fd_gradient(dim, quasi):
    rng = np.random.default_rng(dim)
    if dim == 2:
        s = stretch2d(n=5)
    else:
        s = tet_bar(5, 3, 3, E=1e5)
    p = Problem(s.X, s.elems, s.fixed, s.E, s.nu, s.rho, (0.0, -9.81, 0.0), 1 / 60, quasi)
    p.set_inertial_target(_perturbed(p, rng, 0.02))
    x = _perturbed(p, rng, 0.05)
    g = p.gradient(x)
    eps = 1e-6
    gfd = np.zeros_like(g)
    for fi, v in enumerate(p.free):
        for c in range(p.d):
            xp, xm = x.copy(), x.copy()
            xp[v, c] += eps
            xm[v, c] -= eps
            gfd[fi, c] = (p.energy(xp) - p.energy(xm)) / (2 * eps)
    assert np.max(np.abs(g - gfd)) <= 1e-6 * np.max(np.abs(g))


@pytest.mark.parametrize("dim", [2, 3])
def test_fd_hessian_unprojected(dim):
    rng = np.random.default_rng(10 + dim)
    s = stretch2d(n=4) if dim == 2 else tet_bar(4, 3, 3, E=1e5)
    p = Problem(s.X, s.elems, s.fixed, s.E, s.nu, s.rho, (0.0, -9.81, 0.0), 1 / 60, False)
    p.set_inertial_target(p.X)
    x = _perturbed(p, rng, 0.08)
    H = p.hessian(x, project=False).toarray()
    eps = 1e-6
    Hfd = np.zeros_like(H)
    for fi, v in enumerate(p.free):
        for c in range(p.d):
            xp, xm = x.copy(), x.copy()
            xp[v, c] += eps
            xm[v, c] -= eps
            Hfd[:, fi * p.d + c] = (p.gradient(xp) - p.gradient(xm)).ravel() / (2 * eps)
    assert np.max(np.abs(H - Hfd)) <= 1e-5 * np.max(np.abs(H))
    assert np.max(np.abs(H - H.T)) <= 1e-12 * np.max(np.abs(H))


@pytest.mark.parametrize("dim", [2, 3])
def test_element_invariants(dim):
    rng = np.random.default_rng(20 + dim)
    s = stretch2d(n=4) if dim == 2 else tet_bar(4, 3, 3, E=1e5)
    p = Problem.from_scene(s)
    x = _perturbed(p, rng, 0.1)
    ge = p.element_gradient(x)
    assert np.max(np.abs(ge.sum(axis=1))) <= 1e-9 * np.max(np.abs(ge))
    He = p.element_hessian(x)                         # (m, k, k, d, d)
    m, k = He.shape[:2]
    Hm = np.transpose(He, (0, 1, 3, 2, 4)).reshape(m, k * dim, k * dim)
    for c in range(dim):
        t = np.zeros(k * dim)
        t[c::dim] = 1.0
        assert np.max(np.abs(Hm @ t)) <= 1e-8 * np.max(np.abs(Hm))
    assert np.max(np.abs(Hm - np.swapaxes(Hm, 1, 2))) <= 1e-10 * np.max(np.abs(Hm))
    assert min(np.linalg.eigvalsh(h).min() for h in Hm) >= -1e-9 * np.max(np.abs(Hm))
