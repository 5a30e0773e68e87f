"""Learned per-vertex warm start (FP64 oracle).  The paper has no learned
component; this module defines the proposal the GPU path trains and uses:

features f_i (16 values) of a free vertex i at the inertial predictor x~:
  f[0:3]   (u_i - mean_{j in N(i)} u_j) / l, u = x~ - X, N(i) the mesh neighbours
  f[3:6]   (x~_i - x^t_i) / l  (= h v_i / l)
  f[6:12]  upper triangle (00,01,02,11,12,22) of the step-Hessian diagonal block
           H_ii(x~) = m_i I + h^2 sum_e H_e[i,i]  divided by (m_i + h^2 E l)
  f[12:16] over the elements containing i, volume-weighted mean of (|F|^2 - 3),
           volume-weighted mean of (J - 1), min J, max (|F|^2 - 3), at x~
with l the mean rest edge length.  Inputs are z-scored with training
statistics and padded with zeros to 32 columns.

network: 32 -> 64 -> 64 -> 16 (only the first 3 outputs are used), SiLU
activations, output Delta_i; proposal x_i = x~_i + l Delta_i for free vertices;
loss = mean over samples and the 3 used outputs of (Delta - target)^2 with
target (x*_i - x~_i) / l.  Adam(lr, 0.9, 0.999, 1e-8).
The proposal is accepted only when E(proposal) < E(x~) (oracle.timestep).

Pins: tests/test_oracle_mlp.py -- backward by central finite differences of
the loss; features by their definitions on affine and rest configurations;
one Adam step against the textbook update.
"""
import numpy as np

N_IN, N_IN_PAD, N_HID, N_OUT, N_OUT_PAD = 16, 32, 64, 3, 16
SHAPES = [("W1", (N_IN_PAD, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT_PAD)), ("b3", (N_OUT_PAD,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def mean_edge_length(X, elems):
    k = elems.shape[1]
    L = [np.linalg.norm(X[elems[:, a]] - X[elems[:, b]], axis=1)
         for a in range(k) for b in range(a + 1, k)]
    return float(np.mean(np.concatenate(L)))


def features(prob, x_t, x_tilde):
    """(n_free, 16) features of the free vertices (ascending id)."""
    from .mesh import deformation_gradient
    X, el = prob.X, prob.elems
    ell = mean_edge_length(X, el)
    u = x_tilde - X
    nbr = [set() for _ in range(prob.n)]
    for e in el:
        for a in e:
            nbr[a].update(int(b) for b in e if b != a)
    h = prob.h
    He = prob.element_hessian(x_tilde)                   # (m, k, k, d, d), no h^2
    k = el.shape[1]
    Hii = np.zeros((prob.n, 3, 3))
    for a in range(k):
        np.add.at(Hii, el[:, a], He[:, a, a])
    F = deformation_gradient(x_tilde, el, prob.beta)
    Ic = np.einsum("mij,mij->m", F, F) - 3.0
    J = np.linalg.det(F)
    out = np.zeros((prob.free.size, N_IN))
    for r, i in enumerate(prob.free):
        nb = sorted(nbr[i])
        out[r, 0:3] = (u[i] - u[nb].mean(axis=0)) / ell
        out[r, 3:6] = (x_tilde[i] - x_t[i]) / ell
        H = prob.mass[i] * np.eye(3) + h * h * Hii[i]
        scale = prob.mass[i] + h * h * prob.E * ell
        out[r, 6:12] = H[np.triu_indices(3)] / scale
        es = np.flatnonzero((el == i).any(axis=1))
        w = prob.vol[es]
        out[r, 12] = np.sum(w * Ic[es]) / np.sum(w)
        out[r, 13] = np.sum(w * (J[es] - 1.0)) / np.sum(w)
        out[r, 14] = J[es].min()
        out[r, 15] = Ic[es].max()
    return out, ell


def normalise(feat, mean, std):
    Xn = np.zeros((feat.shape[0], N_IN_PAD))
    Xn[:, :N_IN] = (feat - mean) / std
    return Xn


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, Xn):
    """Returns (Y (B, 16), cache)."""
    p = unpack(params) if not isinstance(params, dict) else params
    Z1 = Xn @ p["W1"] + p["b1"]
    A1 = silu(Z1)
    Z2 = A1 @ p["W2"] + p["b2"]
    A2 = silu(Z2)
    Y = A2 @ p["W3"] + p["b3"]
    return Y, (Xn, Z1, A1, Z2, A2)


def loss_and_dY(Y, T):
    """MSE over the 3 used outputs; dY is zero on the padding columns."""
    B = Y.shape[0]
    R = Y[:, :N_OUT] - T
    loss = float(np.sum(R * R) / (B * N_OUT))
    dY = np.zeros_like(Y)
    dY[:, :N_OUT] = 2.0 * R / (B * N_OUT)
    return loss, dY


def backward(params, cache, dY):
    """Gradient of the loss w.r.t. the packed parameters, given dL/dY."""
    p = unpack(params) if not isinstance(params, dict) else params
    Xn, Z1, A1, Z2, A2 = cache
    g = {}
    g["W3"] = A2.T @ dY
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ p["W3"].T) * dsilu(Z2)
    g["W2"] = A1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"].T) * dsilu(Z1)
    g["W1"] = Xn.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)


def adam(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def proposal(prob, x_tilde, Delta, ell, corr=None):
    """x~ + c + l Delta on free vertices, x~ on Dirichlet ones; c (n x d, or
    None for zero) is the previous step's correction x_end - x~."""
    xp = x_tilde.copy()
    xp[prob.free] += ell * Delta[:, :N_OUT]
    if corr is not None:
        xp[prob.free] += corr[prob.free]
    return xp
