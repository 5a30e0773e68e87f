"""Learned warm start on the GPU: data generation with the solver itself,
training with the library's BF16 MFMA kernels, and held-out evaluation.

Everything numerical runs in libccgpu (features, targets, forward, backward,
Adam, stepping); this module only orders the calls and owns the buffers.
"""
import time

import numpy as np

from . import ccgpu as cg


def _upload(ctx, scenes, dev):
    import torch
    out = []
    for s in scenes:
        mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
        cg.cc_subspace_build(ctx, mid, 0, s.dt, False)          # exact basis
        x, v = s.initial_state()
        xs = torch.tensor(x, dtype=torch.float64, device=dev)
        vs = torch.tensor(v, dtype=torch.float64, device=dev)
        nf = int((~s.fixed.astype(bool)).sum())
        out.append(dict(s=s, mid=mid, x=xs, v=vs, nf=nf))
    return out


def _params(precision, warm, corotate=0):
    return cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, line_search=1,
                                max_iters=10000, precision=precision, warm_start=int(warm),
                                corotate=int(corotate))


def generate(ctx, scenes, steps, dev, tol=1e-6, precision=cg.FP64, corotate=1):
    """Step `scenes` together with CC (corotated by default: the training
    scenes twist, and a rest-frame basis needs hundreds of iterations per
    step there, while the step's solution is the same); record for every
    free vertex of every step the features at the predictor and the target
    (x* - x_base)/l, x_base the predictor plus the mesh's previous step
    correction (the base of the warm start's proposal).  Returns (X (N,16)
    float32, T (N,3) float32, iterations per step)."""
    import torch
    ms = _upload(ctx, scenes, dev)
    rows = sum(m["nf"] for m in ms)
    X = torch.zeros((steps * rows, cg.MLP_NFEAT), dtype=torch.float32, device=dev)
    T = torch.zeros((steps * rows, 3), dtype=torch.float32, device=dev)
    par = _params(precision, False, corotate)
    grav = np.stack([m["s"].gravity for m in ms])
    iters = []
    r0 = 0
    for t in range(1, steps + 1):
        bcs = [torch.tensor(m["s"].targets(t), dtype=torch.float64, device=dev) for m in ms]
        bases, offs = [], []
        for m, bc in zip(ms, bcs):
            _, xt, _ = cg.cc_mlp_features(ctx, m["mid"], m["x"], m["v"], bc, m["s"].dt, m["nf"],
                                          out=X[r0:r0 + m["nf"]])
            bases.append(xt)
            offs.append(r0)
            r0 += m["nf"]
        _, its, _, _ = cg.cc_step_batch(ctx, [m["mid"] for m in ms], [m["x"] for m in ms],
                                        [m["v"] for m in ms], bcs, ms[0]["s"].dt, par, tol, gravity=grav)
        iters.extend(int(i) for i in its)
        for m, xt, o in zip(ms, bases, offs):
            cg.cc_mlp_targets(ctx, m["mid"], m["x"], xt, m["nf"], out=T[o:o + m["nf"]])
    return X, T, iters


def train(ctx, X, T, params0, epochs=30, batch=4096, lr=1e-3, seed=0):
    """Adam on minibatches drawn from a seeded permutation per epoch; returns
    the mean training loss of every epoch and the wall time."""
    import torch
    cg.cc_mlp_set(ctx, np.asarray(params0, dtype=np.float32))
    cg.cc_mlp_norm_from_data(ctx, X)
    rng = np.random.default_rng(seed)
    N = X.shape[0]
    batch = min(batch, N)
    losses = []
    t0 = time.perf_counter()
    for _ in range(epochs):
        perm = torch.tensor(rng.permutation(N).astype(np.int32), device=X.device)
        ep = [cg.cc_mlp_train_step(ctx, X, T, perm[b * batch:(b + 1) * batch], lr)
              for b in range(N // batch)]
        losses.append(float(np.mean(ep)))
    return losses, time.perf_counter() - t0


def evaluate(ctx, scenes, steps, dev, warm, tol=1e-6, precision=cg.FP64):
    """Step held-out scenes together with or without the learned proposal.
    Returns per-step (iterations of every mesh, warm-start acceptances, wall ms)."""
    import torch
    ms = _upload(ctx, scenes, dev)
    par = _params(precision, warm)
    grav = np.stack([m["s"].gravity for m in ms])
    out = []
    for t in range(1, steps + 1):
        bcs = [torch.tensor(m["s"].targets(t), dtype=torch.float64, device=dev) for m in ms]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, _, sts = cg.cc_step_batch(ctx, [m["mid"] for m in ms], [m["x"] for m in ms],
                                          [m["v"] for m in ms], bcs, ms[0]["s"].dt, par, tol,
                                          gravity=grav)
        ms_ = (time.perf_counter() - t0) * 1e3
        acc = [cg.cc_step_info(ctx, m["mid"])["warm_accepted"] for m in ms]
        out.append(dict(iters=[int(i) for i in its], accepted=acc, ms=ms_,
                        ok=all(int(s) == cg.CC_OK for s in sts)))
    return out
