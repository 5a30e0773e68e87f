"""Python binding of libccgpu (argument marshalling only).

Every function has the name of the C entry point it wraps (include/ccgpu.h)
and forwards to it through ctypes.  Host arrays are NumPy arrays; device
arrays are torch tensors on the context's GPU, used only as device memory.
Negative statuses raise CCError; warnings (CC_NOT_CONVERGED, CC_STALLED) are
returned to the caller.  The library must have been built (``build.py``); a
missing library raises at import time of the first call -- there is no
fallback implementation.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccgpu.so")

CC_OK, CC_NOT_CONVERGED, CC_STALLED, CC_GRAPH_FALLBACK = 0, 1, 2, 3
METHOD_CD, METHOD_CC, METHOD_JGS2 = 0, 1, 2
SWEEP_JACOBI, SWEEP_COLORED_GS = 0, 1
HESS_PER_COLOR, HESS_PER_SWEEP = 0, 1
FP64, FP32_MIXED = 0, 1
MATERIAL_SNH, MATERIAL_FCR = 0, 1

_STATUS_NAMES = {
    0: "CC_OK", 1: "CC_NOT_CONVERGED", 2: "CC_STALLED", 3: "CC_GRAPH_FALLBACK", -1: "CC_E_INVALID_ARG",
    -2: "CC_E_MESH",
    -3: "CC_E_SUBSPACE", -4: "CC_E_HIP", -5: "CC_E_NONFINITE", -6: "CC_E_STATE", -7: "CC_E_NO_DEVICE",
}


class CCError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class cc_params(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("sweep", ctypes.c_int32),
                ("hess_refresh", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("line_search", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32),
                ("quasistatic", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("gravity", ctypes.c_double * 3), ("corotate", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libccgpu.so not built at {LIB_PATH}; run paper_2510_12053_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        pI32, pI64, pD = ctypes.POINTER(I32), ctypes.POINTER(I64), ctypes.POINTER(D)
        sig = {
            "cc_params_default": (None, [ctypes.POINTER(cc_params)]),
            "cc_create": (I32, [I32, P, ctypes.POINTER(P)]),
            "cc_destroy": (None, [P]),
            "cc_last_error": (ctypes.c_char_p, [P]),
            "cc_mesh_upload": (I32, [P, I32, I32, P, I32, P, P, D, D, D, pI32]),
            "cc_color": (I32, [P, I32, P, pI32]),
            "cc_mesh_set_material": (I32, [P, I32, I32]),
            "cc_layout": (I32, [P, I32, P, P]),
            "cc_subspace_upload": (I32, [P, I32, P, P, P, D]),
            "cc_subspace_build": (I32, [P, I32, I32, D, I32]),
            "cc_subspace_build_at": (I32, [P, I32, P, I32, D, I32]),
            "cc_subspace_nnz": (I32, [P, I32, pI64]),
            "cc_subspace_download": (I32, [P, I32, P, P, P]),
            "cc_subspace_row": (I32, [P, I32, I32, pI64, P, P]),
            "cc_step": (I32, [P, I32, P, P, P, D, ctypes.POINTER(cc_params), D, pI32, pD]),
            "cc_step_info": (I32, [P, I32, pD, pD, P, pI64, pI32, pI64]),
            "cc_probe_element": (I32, [P, I32, P, I32, P, P]),
            "cc_probe_sweep": (I32, [P, I32, P, P, D, ctypes.POINTER(cc_params), pD, P, P]),
            "cc_step_batch": (I32, [P, I32, P, P, P, P, P, D, ctypes.POINTER(cc_params), D, P, P, P]),
            "cc_batch_tuning": (I32, [P, I32, I32]),
            "cc_dense_tuning": (I32, [P, I32, I32]),
            "cc_autotune_batch": (I32, [P, I32, P, ctypes.POINTER(cc_params), pI32, P]),
            "cc_profile_enable": (I32, [P, I32]),
            "cc_profile_read": (I32, [P, I32, pD, pI64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class Context:
    """Owns a cc_ctx*; released by cc_destroy (also on garbage collection)."""

    def __init__(self, handle, device):
        self.handle = handle
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cc_destroy(self.handle)
            self.handle = None


def _check(ctx, status):
    if status < 0:
        msg = lib().cc_last_error(ctx.handle if ctx is not None else None)
        raise CCError(status, msg.decode() if msg else "")
    return status


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t, dtype_name="float64"):
    import torch
    if t is None:
        return None
    if not t.is_cuda or str(t.dtype) != f"torch.{dtype_name}" or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype_name} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def cc_params_default(**overrides):
    p = cc_params()
    lib().cc_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if k == "gravity":
            for c in range(3):
                p.gravity[c] = float(v[c]) if c < len(v) else 0.0
        else:
            setattr(p, k, int(v))
    return p


def cc_create(device=0, stream=None):
    """stream: a torch.cuda.Stream (default: the current stream of `device`)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    h = ctypes.c_void_p()
    st = lib().cc_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
    if st < 0:
        raise CCError(st, "cc_create failed")
    ctx = Context(h, device)
    ctx.stream = stream
    return ctx


def cc_destroy(ctx):
    if ctx.handle:
        lib().cc_destroy(ctx.handle)
        ctx.handle = None


def cc_mesh_upload(ctx, X, elems, fixed, youngs, poisson, density):
    X = _host(X, np.float64)
    E = _host(elems, np.int32)
    F = _host(fixed, np.uint8)
    mid = ctypes.c_int32(-1)
    _check(ctx, lib().cc_mesh_upload(ctx.handle, X.shape[1], X.shape[0], _ptr(X), E.shape[0], _ptr(E),
                                     _ptr(F), youngs, poisson, density, ctypes.byref(mid)))
    return mid.value


def cc_mesh_set_material(ctx, mesh_id, model):
    _check(ctx, lib().cc_mesh_set_material(ctx.handle, mesh_id, model))


def cc_color(ctx, mesh_id, n_verts):
    col = np.empty(n_verts, dtype=np.int32)
    nc = ctypes.c_int32(0)
    _check(ctx, lib().cc_color(ctx.handle, mesh_id, _ptr(col), ctypes.byref(nc)))
    return col, nc.value


def cc_layout(ctx, mesh_id, n_verts, n_elems):
    vp = np.empty(n_verts, dtype=np.int32)
    ep = np.empty(n_elems, dtype=np.int32)
    _check(ctx, lib().cc_layout(ctx.handle, mesh_id, _ptr(vp), _ptr(ep)))
    return vp, ep


def cc_subspace_upload(ctx, mesh_id, ptr, idx, U, dt_used=0.0):
    ptr = _host(ptr, np.int64)
    idx = _host(idx, np.int32)
    U = _host(U, np.float64)
    _check(ctx, lib().cc_subspace_upload(ctx.handle, mesh_id, _ptr(ptr), _ptr(idx), _ptr(U), dt_used))


def cc_subspace_build(ctx, mesh_id, radius, dt, quasistatic=False):
    _check(ctx, lib().cc_subspace_build(ctx.handle, mesh_id, radius, dt, int(quasistatic)))


def cc_subspace_build_at(ctx, mesh_id, x, radius, dt, quasistatic=False):
    """Basis from the Hessian at the state x (float64 CUDA tensor, n x dim)."""
    _check(ctx, lib().cc_subspace_build_at(ctx.handle, mesh_id, _dptr(x), radius, dt, int(quasistatic)))


def cc_subspace_download(ctx, mesh_id, n_verts, dim):
    nnz = ctypes.c_int64(0)
    _check(ctx, lib().cc_subspace_nnz(ctx.handle, mesh_id, ctypes.byref(nnz)))
    ptr = np.empty(n_verts + 1, dtype=np.int64)
    idx = np.empty(nnz.value, dtype=np.int32)
    U = np.empty((nnz.value, dim, dim), dtype=np.float64)
    _check(ctx, lib().cc_subspace_download(ctx.handle, mesh_id, _ptr(ptr), _ptr(idx), _ptr(U)))
    return ptr, idx, U


def cc_subspace_row(ctx, mesh_id, vertex, n_free, dim):
    """Basis row of caller vertex `vertex`: (idx (caller ids, ascending), U (len, dim, dim))."""
    ln = ctypes.c_int64(0)
    idx = np.empty(max(n_free - 1, 1), dtype=np.int32)
    U = np.empty((max(n_free - 1, 1), dim, dim), dtype=np.float64)
    _check(ctx, lib().cc_subspace_row(ctx.handle, mesh_id, vertex, ctypes.byref(ln), _ptr(idx), _ptr(U)))
    return idx[:ln.value].copy(), U[:ln.value].copy()


def cc_step(ctx, mesh_id, x, v, x_bc, dt, params, tol):
    """x, v (and x_bc or None): float64 CUDA tensors (n, dim), updated in place.
    Returns (status, iters, rel_grad)."""
    it = ctypes.c_int32(0)
    rg = ctypes.c_double(0.0)
    st = _check(ctx, lib().cc_step(ctx.handle, mesh_id, _dptr(x), _dptr(v), _dptr(x_bc), dt,
                                   ctypes.byref(params), tol, ctypes.byref(it), ctypes.byref(rg)))
    return st, it.value, rg.value


def cc_step_info(ctx, mesh_id):
    e, pr = ctypes.c_double(0), ctypes.c_double(0)
    fb = np.zeros(3, dtype=np.int64)
    hv = ctypes.c_int64(0)
    wa = ctypes.c_int32(0)
    sf = ctypes.c_int64(0)
    _check(ctx, lib().cc_step_info(ctx.handle, mesh_id, ctypes.byref(e), ctypes.byref(pr), _ptr(fb),
                                   ctypes.byref(hv), ctypes.byref(wa), ctypes.byref(sf)))
    return dict(energy=e.value, paper_residual=pr.value, fallbacks=fb, halvings=hv.value,
                warm_accepted=int(wa.value), sweep_fallbacks=sf.value)


def cc_probe_element(ctx, mesh_id, x, precision, n_elems):
    import torch
    n, d = x.shape
    k = d + 1
    ge = torch.empty((n_elems, k, d), dtype=torch.float64, device=x.device)
    He = torch.empty((n_elems, k, k, d, d), dtype=torch.float64, device=x.device)
    _check(ctx, lib().cc_probe_element(ctx.handle, mesh_id, _dptr(x), precision, _dptr(ge), _dptr(He)))
    return ge, He


def cc_probe_sweep(ctx, mesh_id, x, x_tilde, dt, params, want_g=True, want_dx=True):
    import torch
    e = ctypes.c_double(0)
    g = torch.zeros_like(x) if want_g else None
    dx = torch.zeros_like(x) if want_dx else None
    _check(ctx, lib().cc_probe_sweep(ctx.handle, mesh_id, _dptr(x), _dptr(x_tilde), dt,
                                     ctypes.byref(params), ctypes.byref(e), _dptr(g), _dptr(dx)))
    return e.value, g, dx


K_ELEM_HESS, K_ASSEMBLE, K_GRADIENT, K_CC_PREP, K_CC_UPDATE, K_ENERGY = range(6)
K_NAMES = ["elem_hess", "assemble", "gradient", "cc_prep", "cc_update", "energy"]


def cc_profile_enable(ctx, mask):
    _check(ctx, lib().cc_profile_enable(ctx.handle, mask))


def cc_profile_read(ctx, kernel_id):
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(ctx, lib().cc_profile_read(ctx.handle, kernel_id, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def cc_step_batch(ctx, mesh_ids, xs, vs, x_bcs, dt, params, tol, gravity=None):
    """Step several meshes together.  xs, vs, x_bcs: lists of float64 CUDA
    tensors (x_bcs may be None or hold None); gravity: (n, 3) array or None.
    Returns (worst status, iters[n], rel_grad[n], status[n])."""
    n = len(mesh_ids)
    ids = np.ascontiguousarray(mesh_ids, dtype=np.int32)
    xp = (ctypes.c_void_p * n)(*[_dptr(t).value for t in xs])
    vp = (ctypes.c_void_p * n)(*[_dptr(t).value for t in vs])
    bp = None
    if x_bcs is not None:
        bp = (ctypes.c_void_p * n)(*[(_dptr(t).value if t is not None else None) for t in x_bcs])
    g = None if gravity is None else np.ascontiguousarray(gravity, dtype=np.float64).reshape(n, 3)
    it = np.zeros(n, dtype=np.int32)
    rg = np.zeros(n, dtype=np.float64)
    st = np.zeros(n, dtype=np.int32)
    worst = _check(ctx, lib().cc_step_batch(ctx.handle, n, _ptr(ids), xp, vp, bp,
                                            None if g is None else _ptr(g), dt, ctypes.byref(params),
                                            tol, _ptr(it), _ptr(rg), _ptr(st)))
    return worst, it, rg, st


def cc_batch_tuning(ctx, lanes, iters_per_graph):
    _check(ctx, lib().cc_batch_tuning(ctx.handle, lanes, iters_per_graph))


def cc_dense_tuning(ctx, rows_per_workgroup, chunk=0):
    _check(ctx, lib().cc_dense_tuning(ctx.handle, rows_per_workgroup, chunk))


def cc_autotune_batch(ctx, mesh_ids, params):
    ids = np.ascontiguousarray(mesh_ids, dtype=np.int32)
    lanes = ctypes.c_int32(0)
    ms = np.zeros(3, dtype=np.float64)
    _check(ctx, lib().cc_autotune_batch(ctx.handle, len(ids), _ptr(ids), ctypes.byref(params),
                                        ctypes.byref(lanes), _ptr(ms)))
    return lanes.value, dict(zip((16, 32, 64), ms.tolist()))


# ---- learned warm start -----------------------------------------------------
MLP_NPARAM = 7312
MLP_NFEAT = 16


def _mlp_sig(L):
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sig = {
        "cc_mlp_set": (I32, [P, P, P, P]),
        "cc_mlp_get": (I32, [P, P, P, P]),
        "cc_mlp_norm_from_data": (I32, [P, P, I32]),
        "cc_mlp_features": (I32, [P, I32, P, P, P, D, P, P, ctypes.POINTER(D)]),
        "cc_mlp_forward": (I32, [P, P, I32, P]),
        "cc_mlp_gradient": (I32, [P, P, P, P, I32, P, ctypes.POINTER(ctypes.c_float)]),
        "cc_mlp_adam": (I32, [P, P, ctypes.c_float]),
        "cc_mlp_gradient_noalloc": (I32, [P, P, P, P, I32, P, P]),
        "cc_mlp_train_step": (I32, [P, P, P, P, I32, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]),
        "cc_mlp_targets": (I32, [P, I32, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ml():
    L = lib()
    if not getattr(L, "_mlp_sig_done", False):
        _mlp_sig(L)
        L._mlp_sig_done = True
    return L


def cc_mlp_set(ctx, params, mean=None, istd=None):
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == MLP_NPARAM
    m = None if mean is None else np.ascontiguousarray(mean, dtype=np.float32)
    s = None if istd is None else np.ascontiguousarray(istd, dtype=np.float32)
    _check(ctx, _ml().cc_mlp_set(ctx.handle, _ptr(p), None if m is None else _ptr(m),
                                 None if s is None else _ptr(s)))


def cc_mlp_get(ctx):
    p = np.empty(MLP_NPARAM, dtype=np.float32)
    m = np.empty(MLP_NFEAT, dtype=np.float32)
    s = np.empty(MLP_NFEAT, dtype=np.float32)
    _check(ctx, _ml().cc_mlp_get(ctx.handle, _ptr(p), _ptr(m), _ptr(s)))
    return p, m, s


def cc_mlp_norm_from_data(ctx, X):
    _check(ctx, _ml().cc_mlp_norm_from_data(ctx.handle, _dptr(X, "float32"), X.shape[0]))


def cc_mlp_features(ctx, mesh_id, x, v, x_bc, dt, n_free, out=None):
    """Returns (feat (n_free,16) float32 CUDA tensor, x_base (n,3) float64, ell):
    x_base is the predictor plus the mesh's last step correction on free
    vertices, the point the warm start adds ell * Delta to.
    out: optional preallocated (n_free,16) float32 tensor (e.g. a view into a
    dataset)."""
    import torch
    feat = out if out is not None else torch.zeros((n_free, MLP_NFEAT), dtype=torch.float32,
                                                   device=x.device)
    xt = torch.empty_like(x)
    ell = ctypes.c_double(0)
    _check(ctx, _ml().cc_mlp_features(ctx.handle, mesh_id, _dptr(x), _dptr(v), _dptr(x_bc), dt,
                                      _dptr(feat, "float32"), _dptr(xt), ctypes.byref(ell)))
    return feat, xt, ell.value


def cc_mlp_forward(ctx, X):
    import torch
    Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device=X.device)
    _check(ctx, _ml().cc_mlp_forward(ctx.handle, _dptr(X, "float32"), X.shape[0], _dptr(Y, "float32")))
    return Y


def cc_mlp_gradient(ctx, X, T, idx):
    import torch
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
    loss = ctypes.c_float(0)
    _check(ctx, _ml().cc_mlp_gradient(ctx.handle, _dptr(X, "float32"), _dptr(T, "float32"),
                                      _dptr(idx, "int32"), idx.shape[0], _dptr(g, "float32"),
                                      ctypes.byref(loss)))
    return g, loss.value


def cc_mlp_gradient_noalloc(ctx, X, T, idx, grad, loss=None):
    """Gradient into the caller's device tensors grad (MLP_NPARAM float32) and
    loss (1 float32, or None); the library allocates nothing and does not
    synchronise the stream."""
    _check(ctx, _ml().cc_mlp_gradient_noalloc(ctx.handle, _dptr(X, "float32"), _dptr(T, "float32"),
                                              _dptr(idx, "int32"), idx.shape[0], _dptr(grad, "float32"),
                                              None if loss is None else _dptr(loss, "float32")))


def cc_mlp_adam(ctx, grad, lr):
    _check(ctx, _ml().cc_mlp_adam(ctx.handle, _dptr(grad, "float32"), lr))


def cc_mlp_train_step(ctx, X, T, idx, lr):
    loss = ctypes.c_float(0)
    _check(ctx, _ml().cc_mlp_train_step(ctx.handle, _dptr(X, "float32"), _dptr(T, "float32"),
                                        _dptr(idx, "int32"), idx.shape[0], lr, ctypes.byref(loss)))
    return loss.value


def cc_mlp_targets(ctx, mesh_id, x_new, x_base, n_free, out=None):
    import torch
    T = out if out is not None else torch.zeros((n_free, 3), dtype=torch.float32, device=x_new.device)
    L = _ml()
    if not hasattr(L, "_tgt_sig"):
        L.cc_mlp_targets.restype = ctypes.c_int32
        L.cc_mlp_targets.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]
        L._tgt_sig = True
    _check(ctx, L.cc_mlp_targets(ctx.handle, mesh_id, _dptr(x_new), _dptr(x_base), _dptr(T, "float32")))
    return T
