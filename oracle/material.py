"""Stable neo-Hookean material (FP64), used in place of the paper's Fixed
Corotational model (Results, Implementation Details names FCR; the workloads
built here call for stable neo-Hookean, so this is a reading, not the paper's
choice).

Energy density, with mu = E/(2(1+nu)), lambda_L = E nu/((1+nu)(1-2nu)) and
lambda = lambda_L + mu (so that the rest linearisation is linear elasticity
with Lame parameters (mu, lambda_L)):

    Psi(F) = mu/2 (|F|_F^2 - d) - mu (J - 1) + lambda/2 (J - 1)^2,   J = det F.

    P = dPsi/dF = mu F + (lambda (J-1) - mu) dJ/dF
    d2Psi/dF2  = mu I + lambda vec(dJ/dF) vec(dJ/dF)^T + (lambda (J-1) - mu) d2J/dF2

with dJ/dF the cofactor matrix (3D columns f1 x f2, f2 x f0, f0 x f1; 2D
[[F11, -F10], [-F01, F00]]) and d2J/dF_ij dF_kl = eps_ikm eps_jln F_mn (3D) or
eps_ik eps_jl (2D).  vec() is row-major: index (r, q) -> r*d + q.  In 2D the
same formulas are used with d = 2 (plane strain, unit thickness).

The solver uses the Hessian projected to the PSD cone element by element:
eigenvalues below zero are set to zero (the paper is silent on indefinite
Hessians; this is the reading taken here).  The projected matrix is unique, so
any correct eigen-routine gives the same result.

Pins: tests/test_oracle_material.py -- central finite differences Psi -> P and
P -> d2Psi/dF2; Psi(I) = 0, P(I) = 0; rotation invariance; the rest second
variation mu(|dF|^2 + tr(dF^2)) + lambda_L (tr dF)^2; projection is PSD,
idempotent and the identity on PSD input.
"""
import numpy as np


def lame(E, nu):
    """Return (mu, lambda) of the stable neo-Hookean energy (lambda = lambda_L + mu)."""
    mu = E / (2.0 * (1.0 + nu))
    lam_l = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
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
