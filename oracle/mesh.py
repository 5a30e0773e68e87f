"""Rest-shape data of a simplicial mesh (FP64).

Follows the finite-element discretisation the paper assumes in its
Background section (positions x in R^{dn}, mass matrix M):

* Dm = [X_1 - X_0, ..., X_d - X_0]; an element with det Dm <= 0 is rejected;
* rest volume V_e = det Dm / d!;
* shape-gradient vectors beta_a: beta_1..beta_d are the rows of Dm^{-1} and
  beta_0 = -(beta_1 + ... + beta_d), so that F = sum_a x_a beta_a^T;
* lumped mass m_i = rho * sum_{e containing i} V_e / (d+1).  The paper only
  names "the mass matrix"; the lumped form is this package's reading.

Pins: tests/test_oracle_mesh_fem.py (counts, orientation, total volume equals the
box volume, F(X) = I, total mass equals rho * volume).
"""
import math

import numpy as np


class MeshError(ValueError):
    pass


def rest_data(X, elems):
    """Return (beta (m, d+1, d), vol (m,)) for rest positions X and elements."""
    X = np.asarray(X, dtype=np.float64)
    elems = np.asarray(elems)
    d = X.shape[1]
    Xe = X[elems]                                     # (m, d+1, d)
    Dm = np.transpose(Xe[:, 1:, :] - Xe[:, :1, :], (0, 2, 1))   # columns X_a - X_0
    det = np.linalg.det(Dm)
    if np.any(~(det > 0.0)):
        bad = int(np.flatnonzero(~(det > 0.0))[0])
        raise MeshError(f"element {bad} has non-positive rest volume")
    Dinv = np.linalg.inv(Dm)                          # rows are beta_1..beta_d
    beta = np.empty((elems.shape[0], d + 1, d))
    beta[:, 1:, :] = Dinv
    beta[:, 0, :] = -Dinv.sum(axis=1)
    vol = det / math.factorial(d)
    return beta, vol


def lumped_mass(n, elems, vol, rho):
    """m_i = rho * sum_{e ni i} V_e / (d+1)."""
    k = elems.shape[1]
    m = np.zeros(n)
    np.add.at(m, np.asarray(elems).ravel(), np.repeat(rho * vol / k, k))
    return m


def deformation_gradient(x, elems, beta):
    """F_e = sum_a x_{e,a} beta_{e,a}^T, shape (m, d, d)."""
    xe = np.asarray(x)[elems]                          # (m, d+1, d)
    return np.einsum("mar,maq->mrq", xe, beta)
