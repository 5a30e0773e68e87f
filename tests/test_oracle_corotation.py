"""Pins of the corotated basis (Method, Accounting for Large Deformations,
Eq. rotation): the polar rotation against its definition, the rotations of a
rigid motion, the identity at rest, and the rotation equivariance of the
corotated Coordinate Condensation directions (which the unrotated basis does
not have)."""
import numpy as np
from scipy.spatial.transform import Rotation

from ccscenes import tet_bar
from oracle import solvers as S
from oracle.basis import basis_matrix, exact_basis
from oracle.fem import Problem
from oracle.timestep import predictor


def test_polar_rotation_definition():
    """Against the closed form R = M (M^T M)^(-1/2) where det M > 0, and
    M = Q P (P symmetric positive definite) -> Q in 2D and 3D."""
    from scipy.linalg import sqrtm
    rng = np.random.default_rng(0)
    for d in (2, 3):
        n = 0
        while n < 20:
            M = rng.normal(size=(d, d))
            if np.linalg.det(M) <= 0.1:
                continue
            n += 1
            R = S.polar_rotation(M)
            ref = M @ np.linalg.inv(np.real(sqrtm(M.T @ M)))
            assert np.allclose(R, ref, atol=1e-10)
            assert np.allclose(R @ R.T, np.eye(d), atol=1e-12)
            assert abs(np.linalg.det(R) - 1.0) < 1e-12
        Q = Rotation.random(random_state=3).as_matrix() if d == 3 else \
            np.array([[np.cos(0.7), -np.sin(0.7)], [np.sin(0.7), np.cos(0.7)]])
        A = rng.normal(size=(d, d))
        P = A @ A.T + d * np.eye(d)
        assert np.allclose(S.polar_rotation(Q @ P), Q, atol=1e-12)
        # a reflection in M still gives a proper rotation
        Rf = S.polar_rotation(np.diag([1.0] * (d - 1) + [-1.0]) @ P)
        assert abs(np.linalg.det(Rf) - 1.0) < 1e-12


def test_rigid_motion_rotations():
    s = tet_bar(5, 3, 3)
    p = Problem.from_scene(s)
    Q = Rotation.from_rotvec([0.3, -1.1, 0.5]).as_matrix()
    x = s.X @ Q.T + np.array([0.2, -0.4, 1.0])
    R = S.vertex_rotations(p, x)
    assert np.allclose(R, Q[None], atol=1e-12)
    Rrest = S.vertex_rotations(p, s.X)
    assert np.allclose(Rrest, np.eye(3)[None], atol=1e-12)


def _directions(p, B, x, corotate):
    Umat = basis_matrix(p, *B)
    if corotate:
        Umat = S.rotate_basis(p, Umat, S.vertex_rotations(p, x))
    g = p.gradient(x)
    H = p.hessian(x)
    dx, _ = S.local_directions(p, Umat, H, g, np.arange(p.free.size), S.CC)
    return dx


def test_identity_at_rest():
    s = tet_bar(5, 3, 3, E=1e5)
    p = Problem.from_scene(s)
    B = exact_basis(p)
    # rotations at the rest shape are the identity, so the rotated basis is the basis
    Umat = basis_matrix(p, *B)
    Ur = S.rotate_basis(p, Umat, S.vertex_rotations(p, s.X))
    assert abs(Ur - Umat).max() <= 1e-14 * abs(Umat).max()


def test_corotated_directions_rotate_with_the_body():
    """Rotating a deformed state, its inertial target and its boundary values
    by Q (no gravity: the step energy is then invariant) rotates the
    corotated CC directions by Q; the basis fixed at rest does not."""
    s = tet_bar(5, 3, 3, E=1e6, gravity=(0.0, 0.0, 0.0))
    p = Problem.from_scene(s)
    B = exact_basis(p)
    rng = np.random.default_rng(5)
    x = s.X + 0.02 * rng.normal(size=s.X.shape)
    xt = x + 0.01 * rng.normal(size=s.X.shape)
    Q = Rotation.from_rotvec([0.9, 0.4, -1.3]).as_matrix()

    p.set_inertial_target(xt)
    d0 = _directions(p, B, x, True)
    n0 = _directions(p, B, x, False)
    p.set_inertial_target(xt @ Q.T)
    d1 = _directions(p, B, x @ Q.T, True)
    n1 = _directions(p, B, x @ Q.T, False)
    scale = np.abs(d0).max()
    assert np.abs(d1 - d0 @ Q.T).max() <= 1e-9 * scale
    assert np.abs(n1 - n0 @ Q.T).max() > 1e-3 * np.abs(n0).max()


def test_corotated_solve_converges_to_newton():
    """Corotated CC with line search reaches the same minimiser as Newton on
    a bar whose free end is turned by 60 degrees."""
    s = tet_bar(6, 3, 3, E=1e5, gravity=(0.0, 0.0, 0.0), twist_per_step=np.pi / 3)
    p = Problem.from_scene(s)
    B = exact_basis(p)
    x0, v0 = s.initial_state()
    xh = predictor(p, x0, v0, s.targets(1))
    prm = S.Params(method=S.CC, sweep=S.JACOBI, line_search=True, max_iters=300, corotate=True)
    res = S.solve(p, xh, B, prm, 1e-10)
    ref = S.newton(p, xh, tol=1e-12)
    assert res.status == S.OK
    assert np.linalg.norm(res.x - ref.x) <= 1e-6 * np.linalg.norm(ref.x - s.X)
