"""Pins of the oracle's Fixed Corotational energy (Results, Implementation
Details names the model): derivatives by finite differences, the closest
rotation against scipy's polar decomposition and Procrustes optimality, the
Sylvester solve against scipy's solver, the rest linearisation shared with
stable neo-Hookean (so the exact basis is the same), invariances, and the
projected-free spectrum against the published closed-form eigenvalues of
the as-rigid-as-possible and volume terms."""
import numpy as np
import pytest
from scipy.linalg import polar, solve_sylvester
from scipy.spatial.transform import Rotation

from ccscenes import tet_bar
from oracle import material as mt
from oracle.basis import exact_basis
from oracle.fem import Problem

MU, LAM = mt.lame(1e5, 0.4, mt.FCR)


def _rot(rng, d):
    if d == 3:
        return Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix()
    a = rng.uniform(-np.pi, np.pi)
    return np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])


def _F(rng, d, m, scale, inverted=False):
    """Random deformation gradients away from the non-differentiable set
    (rotation-variant singular values whose pairwise sums stay >= 0.2 in
    magnitude)."""
    out = []
    while len(out) < m:
        F = np.eye(d) + scale * rng.normal(size=(d, d))
        if inverted:
            F[:, 0] *= -1.0
        s = np.linalg.svd(F, compute_uv=False)
        if np.linalg.det(F) < 0:
            s[-1] = -s[-1]
        if min(abs(s[i] + s[j]) for i in range(d) for j in range(i + 1, d)) < 0.2:
            continue
        out.append(F)
    return np.array(out)


def test_lame_parameters():
    mu, lam = mt.lame(2.0e5, 0.3, mt.FCR)
    mu_s, lam_s = mt.lame(2.0e5, 0.3, mt.SNH)
    assert mu == mu_s and abs(lam + mu - lam_s) <= 1e-9 * lam_s
    assert abs(lam - 2.0e5 * 0.3 / (1.3 * 0.4)) <= 1e-9 * lam
    with pytest.raises(ValueError):
        mt.lame(1.0, 0.3, "corotated-linear")


@pytest.mark.parametrize("d", [2, 3])
def test_closest_rotation(d):
    rng = np.random.default_rng(11 + d)
    F = np.concatenate([_F(rng, d, 15, 0.5), _F(rng, d, 15, 0.5, inverted=True)])
    R = mt.closest_rotation(F)
    for k in range(F.shape[0]):
        assert np.allclose(R[k] @ R[k].T, np.eye(d), atol=1e-12)
        assert abs(np.linalg.det(R[k]) - 1.0) < 1e-12
        S = R[k].T @ F[k]
        assert np.allclose(S, S.T, atol=1e-12)                # first-order optimality
        if np.linalg.det(F[k]) > 0:
            Up, _ = polar(F[k])
            assert np.allclose(R[k], Up, atol=1e-11)
        # no random rotation is closer
        best = np.linalg.norm(F[k] - R[k])
        for _ in range(50):
            Q = _rot(rng, d)
            assert np.linalg.norm(F[k] - Q) >= best - 1e-12
            Qn = R[k] @ _rot_small(rng, d)
            assert np.linalg.norm(F[k] - Qn) >= best - 1e-12


def _rot_small(rng, d):
    if d == 3:
        return Rotation.from_rotvec(0.05 * rng.normal(size=3)).as_matrix()
    a = 0.05 * rng.normal()
    return np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])


@pytest.mark.parametrize("d", [2, 3])
def test_sylvester_against_scipy(d):
    rng = np.random.default_rng(3 + d)
    A = rng.normal(size=(10, d, d))
    S = np.einsum("mij,mkj->mik", A, A) + 0.3 * np.eye(d)
    M = rng.normal(size=(10, d, d))
    W = mt.sylvester_sym(S, M)
    for k in range(10):
        ref = solve_sylvester(S[k], S[k], M[k])
        assert np.allclose(W[k], ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("inverted", [False, True])
def test_fd_psi_to_P(d, inverted):
    rng = np.random.default_rng(21 + d + 5 * inverted)
    F = _F(rng, d, 20, 0.4, inverted)
    P = mt.fcr_pk1(F, MU, LAM)
    eps = 1e-6
    Pfd = np.zeros_like(F)
    for i in range(d):
        for j in range(d):
            dF = np.zeros((d, d))
            dF[i, j] = eps
            Pfd[:, i, j] = (mt.fcr_psi(F + dF, MU, LAM) - mt.fcr_psi(F - dF, MU, LAM)) / (2 * eps)
    assert np.max(np.abs(P - Pfd)) <= 1e-6 * np.max(np.abs(P))


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("inverted", [False, True])
def test_fd_P_to_hessian(d, inverted):
    rng = np.random.default_rng(31 + d + 5 * inverted)
    F = _F(rng, d, 20, 0.4, inverted)
    C = mt.fcr_dpdf(F, MU, LAM)
    eps = 1e-6
    Cfd = np.zeros_like(C)
    for st in range(d * d):
        dF = np.zeros((d, d))
        dF[st // d, st % d] = eps
        dP = mt.fcr_pk1(F + dF, MU, LAM) - mt.fcr_pk1(F - dF, MU, LAM)
        Cfd[:, :, st] = dP.reshape(-1, d * d) / (2 * eps)
    assert np.max(np.abs(C - Cfd)) <= 1e-5 * np.max(np.abs(C))
    assert np.allclose(C, np.swapaxes(C, 1, 2), atol=1e-9 * np.abs(C).max())


@pytest.mark.parametrize("d", [2, 3])
def test_rotation_derivative_fd(d):
    rng = np.random.default_rng(41 + d)
    F = np.concatenate([_F(rng, d, 8, 0.5), _F(rng, d, 8, 0.5, inverted=True)])
    dR = mt.rotation_derivative(F)
    eps = 1e-6
    for st in range(d * d):
        dF = np.zeros((d, d))
        dF[st // d, st % d] = eps
        fd = (mt.closest_rotation(F + dF) - mt.closest_rotation(F - dF)) / (2 * eps)
        assert np.max(np.abs(dR[:, :, st] - fd.reshape(-1, d * d))) <= 1e-7


@pytest.mark.parametrize("d", [2, 3])
def test_rest_linearisation_equals_neo_hookean(d):
    """At F = I the second variation is mu(|dF|^2 + tr(dF^2)) + lambda_L (tr dF)^2,
    the stable neo-Hookean one: both materials share the rest Hessian."""
    rng = np.random.default_rng(51 + d)
    I = np.eye(d)[None]
    C = mt.fcr_dpdf(I, MU, LAM)[0]
    mu_s, lam_s = mt.lame(1e5, 0.4, mt.SNH)
    assert np.allclose(C, mt.dpdf(I, mu_s, lam_s)[0], atol=1e-9 * MU)
    for _ in range(10):
        dF = rng.normal(size=(d, d))
        v = dF.ravel()
        ref = MU * (np.sum(dF * dF) + np.trace(dF @ dF)) + LAM * np.trace(dF) ** 2
        assert abs(v @ C @ v - ref) <= 1e-10 * abs(ref) + 1e-6


def test_exact_basis_is_material_independent():
    s = tet_bar(5, 3, 3, E=1e5)
    p_snh = Problem.from_scene(s)
    p_fcr = Problem(s.X, s.elems, s.fixed, s.E, s.nu, s.rho, s.gravity, s.dt, s.quasistatic, mt.FCR)
    H1 = p_snh.hessian(s.X).toarray()
    H2 = p_fcr.hessian(s.X).toarray()
    assert np.abs(H1 - H2).max() <= 1e-9 * np.abs(H1).max()
    B1, B2 = exact_basis(p_snh), exact_basis(p_fcr)
    assert np.array_equal(B1[0], B2[0]) and np.array_equal(B1[1], B2[1])
    assert np.abs(B1[2] - B2[2]).max() <= 1e-7 * max(np.abs(B1[2]).max(), 1.0)


@pytest.mark.parametrize("d", [2, 3])
def test_rotations_and_invariance(d):
    rng = np.random.default_rng(61 + d)
    Q = np.array([_rot(rng, d) for _ in range(10)])
    assert np.allclose(mt.fcr_psi(Q, MU, LAM), 0.0, atol=1e-12 * MU)
    assert np.allclose(mt.fcr_pk1(Q, MU, LAM), 0.0, atol=1e-10 * MU)
    F = _F(rng, d, 10, 0.4)
    QF = np.einsum("mij,mjk->mik", Q, F)
    assert np.allclose(mt.fcr_psi(QF, MU, LAM), mt.fcr_psi(F, MU, LAM), rtol=1e-10)
    assert np.allclose(mt.fcr_pk1(QF, MU, LAM), np.einsum("mij,mjk->mik", Q, mt.fcr_pk1(F, MU, LAM)),
                       atol=1e-9 * MU)
    # isotropy: Psi(F Q) = Psi(F)
    FQ = np.einsum("mij,mjk->mik", F, Q)
    assert np.allclose(mt.fcr_psi(FQ, MU, LAM), mt.fcr_psi(F, MU, LAM), rtol=1e-10)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("inverted", [False, True])
def test_closed_form_spectrum(d, inverted):
    """Eigenvalues of the unprojected Hessian against the closed form of the
    as-rigid-as-possible term (2 mu on scalings and flips, 2 mu - 4 mu/(s_k+s_l)
    on twists) plus the volume term (lambda c c^T + lambda (J-1) d2J on the
    scaling block, -+ lambda (J-1) s_m on flips and twists), with s the
    rotation-variant singular values, c_k = prod_{l != k} s_l and s_m the
    remaining singular value (1 in 2D)."""
    rng = np.random.default_rng(71 + d + 5 * inverted)
    F = _F(rng, d, 10, 0.5, inverted)
    C = mt.fcr_dpdf(F, MU, LAM)
    for k in range(F.shape[0]):
        s = np.linalg.svd(F[k], compute_uv=False)
        J = np.linalg.det(F[k])
        if J < 0:
            s[-1] = -s[-1]
        c = np.array([np.prod(np.delete(s, i)) for i in range(d)])
        A = 2 * MU * np.eye(d) + LAM * np.outer(c, c)
        ref = []
        for i in range(d):
            for j in range(i + 1, d):
                sm = 1.0 if d == 2 else s[3 - i - j]
                A[i, j] += LAM * (J - 1) * sm
                A[j, i] += LAM * (J - 1) * sm
                ref.append(2 * MU - 4 * MU / (s[i] + s[j]) + LAM * (J - 1) * sm)
                ref.append(2 * MU - LAM * (J - 1) * sm)
        ref.extend(np.linalg.eigvalsh(A))
        w = np.linalg.eigvalsh(0.5 * (C[k] + C[k].T))
        assert np.allclose(np.sort(w), np.sort(ref), atol=1e-8 * np.abs(ref).max())


def test_rod_stiffness_ordering():
    """The struck free rod (Results, Material Stiffness Scaling): with the
    exact basis CC needs a few iterations at every stiffness, while JGS2's
    count grows with E and CD's exceeds a 100-iteration cap once E = 1e4."""
    import dataclasses

    from ccscenes import rod_impulse
    from oracle import solvers as S
    from oracle.timestep import predictor

    def iters(E, method, cap):
        s = dataclasses.replace(rod_impulse(E=E), material=mt.FCR)
        p = Problem.from_scene(s)
        B = exact_basis(p)
        x0, v0 = s.initial_state()
        xh = predictor(p, x0, v0, s.targets(1))
        res = S.solve(p, xh, B, S.Params(method=method, sweep=S.JACOBI, line_search=True, max_iters=cap), 1e-6)
        return res.iters, res.status

    cc = [iters(E, S.CC, 50) for E in (1e1, 1e4, 1e6)]
    assert all(st == S.OK and it <= 4 for it, st in cc)
    j1, j2 = iters(1e1, S.JGS2, 200), iters(1e4, S.JGS2, 200)
    assert j1[1] == S.OK and j2[1] == S.OK and j2[0] > 10 * j1[0]
    cd = iters(1e4, S.CD, 100)
    assert cd == (100, S.NOT_CONVERGED)
