"""Pins of the oracle's stable neo-Hookean energy and PSD projection."""
import numpy as np
import pytest

from oracle.material import dpdf, lame, pk1, project_psd, psi


def _rand_F(rng, d, m, scale):
    return np.eye(d)[None] + scale * rng.normal(size=(m, d, d))


def _rot(rng, d):
    Q, R = np.linalg.qr(rng.normal(size=(d, d)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("scale", [0.05, 0.6])
def test_fd_psi_to_P(d, scale):
    rng = np.random.default_rng(1 + d)
    mu, lam = lame(1e5, 0.4)
    F = _rand_F(rng, d, 20, scale)
    P = pk1(F, mu, lam)
    eps = 1e-6
    Pfd = np.zeros_like(F)
    for i in range(d):
        for j in range(d):
            dF = np.zeros((d, d))
            dF[i, j] = eps
            Pfd[:, i, j] = (psi(F + dF, mu, lam) - psi(F - dF, mu, lam)) / (2 * eps)
    assert np.max(np.abs(P - Pfd)) <= 1e-6 * np.max(np.abs(P))


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("scale", [0.05, 0.6])
def test_fd_P_to_hessian(d, scale):
    rng = np.random.default_rng(7 + d)
    mu, lam = lame(1e6, 0.45)
    F = _rand_F(rng, d, 20, scale)
    C = dpdf(F, mu, lam)
    eps = 1e-6
    Cfd = np.zeros_like(C)
    for k in range(d * d):
        dF = np.zeros((d, d))
        dF.flat[k] = eps
        Cfd[:, :, k] = ((pk1(F + dF, mu, lam) - pk1(F - dF, mu, lam)) / (2 * eps)).reshape(-1, d * d)
    assert np.max(np.abs(C - Cfd)) <= 1e-5 * np.max(np.abs(C))


@pytest.mark.parametrize("d", [2, 3])
def test_rest_state(d):
    mu, lam = lame(1e5, 0.4)
    I = np.eye(d)[None]
    assert abs(psi(I, mu, lam)[0]) == 0.0
    assert np.max(np.abs(pk1(I, mu, lam))) == 0.0


@pytest.mark.parametrize("d", [2, 3])
def test_rotation_invariance(d):
    rng = np.random.default_rng(3)
    mu, lam = lame(1e5, 0.3)
    F = _rand_F(rng, d, 10, 0.4)
    for _ in range(3):
        Q = _rot(rng, d)
        QF = np.einsum("ij,mjk->mik", Q, F)
        np.testing.assert_allclose(psi(QF, mu, lam), psi(F, mu, lam), rtol=1e-11, atol=1e-6)


@pytest.mark.parametrize("d", [2, 3])
def test_rest_linearisation_is_linear_elasticity(d):
    """Second variation at F = I equals mu(|dF|^2 + tr(dF^2)) + lambda_L (tr dF)^2."""
    rng = np.random.default_rng(11)
    E, nu = 2e5, 0.42
    mu, lam = lame(E, nu)
    lam_l = E * nu / ((1 + nu) * (1 - 2 * nu))
    C = dpdf(np.eye(d)[None], mu, lam)[0]
    for _ in range(10):
        dF = rng.normal(size=(d, d))
        lhs = dF.ravel() @ C @ dF.ravel()
        rhs = mu * (np.sum(dF * dF) + np.trace(dF @ dF)) + lam_l * np.trace(dF) ** 2
        assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_lame_textbook_case():
    # nu = 0.25 gives lambda_L = mu = E / 2.5
    mu, lam = lame(1.0, 0.25)
    assert abs(mu - 0.4) < 1e-15 and abs(lam - 0.8) < 1e-15


@pytest.mark.parametrize("n", [4, 9])
def test_projection_kkt(n):
    """P(A) is the Frobenius-nearest PSD matrix: P >= 0, P - A >= 0, <P, P - A> = 0."""
    rng = np.random.default_rng(n)
    A = rng.normal(size=(50, n, n))
    A = A + np.swapaxes(A, 1, 2)
    P = project_psd(A)
    for a, p in zip(A, P):
        assert np.linalg.eigvalsh(p).min() >= -1e-12 * np.abs(a).max()
        assert np.linalg.eigvalsh(p - a).min() >= -1e-12 * np.abs(a).max()
        assert abs(np.sum(p * (p - a))) <= 1e-11 * np.sum(a * a)
    np.testing.assert_allclose(project_psd(P), P, atol=1e-12 * np.abs(P).max())
    S = np.einsum("mij,mkj->mik", A, A)        # PSD input is left unchanged
    np.testing.assert_allclose(project_psd(S), S, atol=1e-11 * np.abs(S).max())


def test_projection_is_nearest():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(9, 9))
    A = A + A.T
    P = project_psd(A[None])[0]
    for _ in range(200):
        B = rng.normal(size=(9, 9))
        B = P + 0.1 * B @ B.T * rng.uniform() - 0.0
        w, Q = np.linalg.eigh(0.5 * (B + B.T))
        B = Q @ np.diag(np.maximum(w, 0)) @ Q.T
        assert np.linalg.norm(A - P) <= np.linalg.norm(A - B) + 1e-12
