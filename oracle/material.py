"""Elastic materials (FP64): stable neo-Hookean and Fixed Corotational.

Stable neo-Hookean stands in for the paper's material on the workloads built
here; Fixed Corotational is the model the paper's own experiments use
(Results, Implementation Details).  Both take mu = E/(2(1+nu)) and
lambda_L = E nu/((1+nu)(1-2nu)).

Stable neo-Hookean, with lambda = lambda_L + mu (so that the rest
linearisation is linear elasticity with Lame parameters (mu, lambda_L)):

    Psi(F) = mu/2 (|F|_F^2 - d) - mu (J - 1) + lambda/2 (J - 1)^2,   J = det F.

    P = dPsi/dF = mu F + (lambda (J-1) - mu) dJ/dF
    d2Psi/dF2  = mu I + lambda vec(dJ/dF) vec(dJ/dF)^T + (lambda (J-1) - mu) d2J/dF2

with dJ/dF the cofactor matrix (3D columns f1 x f2, f2 x f0, f0 x f1; 2D
[[F11, -F10], [-F01, F00]]) and d2J/dF_ij dF_kl = eps_ikm eps_jln F_mn (3D) or
eps_ik eps_jl (2D).  vec() is row-major: index (r, q) -> r*d + q.  In 2D the
same formulas are used with d = 2 (plane strain, unit thickness).

Fixed Corotational, with lambda = lambda_L (its rest linearisation is then
the same linear elasticity, so both materials share the rest Hessian and
hence the exact basis):

    Psi(F) = mu |F - R|_F^2 + lambda/2 (J - 1)^2,   R the rotation closest to F
    P      = 2 mu (F - R) + lambda (J - 1) dJ/dF
    d2Psi/dF2 = 2 mu (I - dR/dF) + lambda vec(dJ/dF) vec(dJ/dF)^T + lambda (J-1) d2J/dF2

R is the proper rotation minimising |F - R| (orthogonal Procrustes with the
determinant constraint: from the SVD F = U S V^T, R = U diag(1, .., det(U V^T)) V^T),
so S := R^T F is symmetric.  P carries no dR term because (F - R)^T R = S - I is
symmetric and R^T dR is skew.  dR/dF is the exact derivative: differentiating
F = R S gives, for W = R^T dR (skew),

    W S + S W = R^T dF - dF^T R,

a Sylvester equation solved in the eigenbasis of S (eigenvalues s_i):
W~_ij = M~_ij / (s_i + s_j).  Where s_i + s_j = 0 (an element inverted so far
that two rotation-variant singular values cancel) R is not differentiable;
the reading taken there is W~_ij = 0.

The solver uses the Hessian projected to the PSD cone element by element:
eigenvalues below zero are set to zero (the paper is silent on indefinite
Hessians; this is the reading taken here).  The projected matrix is unique, so
any correct eigen-routine gives the same result.

Pins: tests/test_oracle_material.py (stable neo-Hookean) and
tests/test_oracle_fcr.py (Fixed Corotational) -- central finite differences
Psi -> P and P -> d2Psi/dF2; Psi and P vanish on rotations; rotation
invariance; the rest second variation mu(|dF|^2 + tr(dF^2)) + lambda_L (tr dF)^2;
R against scipy's polar decomposition and Procrustes optimality; the Sylvester
solve against scipy's solver; the projected Fixed Corotational spectrum against
its published closed form; projection is PSD, idempotent and the identity on
PSD input.
"""
import numpy as np


SNH = "snh"
FCR = "fcr"
MATERIALS = (SNH, FCR)


def lame(E, nu, model=SNH):
    """Return (mu, lambda) of the material: lambda = lambda_L + mu for stable
    neo-Hookean, lambda_L for Fixed Corotational."""
    mu = E / (2.0 * (1.0 + nu))
    lam_l = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    if model == FCR:
        return mu, lam_l
    if model != SNH:
        raise ValueError(f"unknown material {model!r}")
    return mu, lam_l + mu


def _levi_civita(d):
    if d == 2:
        return np.array([[0.0, 1.0], [-1.0, 0.0]])
    e = np.zeros((3, 3, 3))
    e[0, 1, 2] = e[1, 2, 0] = e[2, 0, 1] = 1.0
    e[0, 2, 1] = e[2, 1, 0] = e[1, 0, 2] = -1.0
    return e


def det_grad(F):
    """dJ/dF (cofactor matrix) for a stack F (m, d, d)."""
    d = F.shape[-1]
    if d == 2:
        C = np.empty_like(F)
        C[:, 0, 0] = F[:, 1, 1]
        C[:, 0, 1] = -F[:, 1, 0]
        C[:, 1, 0] = -F[:, 0, 1]
        C[:, 1, 1] = F[:, 0, 0]
        return C
    f0, f1, f2 = F[:, :, 0], F[:, :, 1], F[:, :, 2]
    return np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=2)


def det_hess(F):
    """d2J/dF2 as (m, d*d, d*d) in row-major vec ordering."""
    m, d, _ = F.shape
    eps = _levi_civita(d)
    if d == 2:
        T = np.einsum("ik,jl->ijkl", eps, eps)
        return np.broadcast_to(T.reshape(1, 4, 4), (m, 4, 4)).copy()
    T = np.einsum("ikM,jlN,zMN->zijkl", eps, eps, F, optimize=True)
    return T.reshape(m, 9, 9)


def psi(F, mu, lam):
    d = F.shape[-1]
    J = np.linalg.det(F)
    return (0.5 * mu * (np.einsum("mij,mij->m", F, F) - d) - mu * (J - 1.0)
            + 0.5 * lam * (J - 1.0) ** 2)


def pk1(F, mu, lam):
    J = np.linalg.det(F)
    return mu * F + (lam * (J - 1.0) - mu)[:, None, None] * det_grad(F)


def dpdf(F, mu, lam):
    """Unprojected d2Psi/dF2, (m, d*d, d*d)."""
    m, d, _ = F.shape
    J = np.linalg.det(F)
    g = det_grad(F).reshape(m, d * d)
    return (mu * np.eye(d * d)[None] + lam * np.einsum("mi,mj->mij", g, g)
            + (lam * (J - 1.0) - mu)[:, None, None] * det_hess(F))


def project_psd(C):
    """Clamp the negative eigenvalues of each symmetric matrix of the stack to 0."""
    Cs = 0.5 * (C + np.swapaxes(C, -1, -2))
    w, Q = np.linalg.eigh(Cs)
    return np.einsum("mik,mk,mjk->mij", Q, np.maximum(w, 0.0), Q, optimize=True)


# ----- Fixed Corotational ----------------------------------------------------
def closest_rotation(F):
    """Proper rotation nearest to each F of the stack (Frobenius norm)."""
    U, _, Vt = np.linalg.svd(F)
    sgn = np.sign(np.linalg.det(U @ Vt))
    sgn[sgn == 0] = 1.0
    U = U.copy()
    U[:, :, -1] *= sgn[:, None]
    return U @ Vt


def sylvester_sym(S, M):
    """Solve W S + S W = M for each symmetric S of the stack (eigenbasis of S;
    pairs with s_i + s_j = 0 get W~_ij = 0)."""
    s, Q = np.linalg.eigh(S)
    Mt = np.einsum("mki,mkl,mlj->mij", Q, M, Q)
    den = s[:, :, None] + s[:, None, :]
    Wt = np.divide(Mt, den, out=np.zeros_like(Mt), where=den != 0.0)
    return np.einsum("mik,mkl,mjl->mij", Q, Wt, Q)


def fcr_psi(F, mu, lam):
    R = closest_rotation(F)
    J = np.linalg.det(F)
    D = F - R
    return mu * np.einsum("mij,mij->m", D, D) + 0.5 * lam * (J - 1.0) ** 2


def fcr_pk1(F, mu, lam):
    R = closest_rotation(F)
    J = np.linalg.det(F)
    return 2.0 * mu * (F - R) + (lam * (J - 1.0))[:, None, None] * det_grad(F)


def rotation_derivative(F):
    """dR/dF as (m, d*d, d*d): entry [(r,q),(s,t)] = dR_rq / dF_st."""
    m, d, _ = F.shape
    R = closest_rotation(F)
    S = np.swapaxes(R, 1, 2) @ F
    S = 0.5 * (S + np.swapaxes(S, 1, 2))
    out = np.empty((m, d * d, d * d))
    for st in range(d * d):
        E = np.zeros((d, d))
        E[st // d, st % d] = 1.0
        M = np.swapaxes(R, 1, 2) @ E - E.T[None] @ R
        W = sylvester_sym(S, M)
        out[:, :, st] = (R @ W).reshape(m, d * d)
    return out


def fcr_dpdf(F, mu, lam):
    """Unprojected d2Psi/dF2 of Fixed Corotational, (m, d*d, d*d)."""
    m, d, _ = F.shape
    J = np.linalg.det(F)
    g = det_grad(F).reshape(m, d * d)
    return (2.0 * mu * (np.eye(d * d)[None] - rotation_derivative(F))
            + lam * np.einsum("mi,mj->mij", g, g)
            + (lam * (J - 1.0))[:, None, None] * det_hess(F))


def energy_density(model):
    """(psi, pk1, dpdf) of the named material."""
    if model == SNH:
        return psi, pk1, dpdf
    if model == FCR:
        return fcr_psi, fcr_pk1, fcr_dpdf
    raise ValueError(f"unknown material {model!r}")
