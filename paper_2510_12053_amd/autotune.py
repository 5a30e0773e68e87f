"""Schedule and tile autotuner of the batched path, with a JSON cache.

The tunables, all set through the C ABI:
  * lanes per vertex of the sparse-basis condensation and update kernels
    (16, 32, 64; cc_batch_tuning);
  * iterations captured per graph replay, i.e. per host check (1, 2, 4;
    cc_batch_tuning);
  * rows per workgroup of the exact-basis condensation (1, 2, 3 or the most
    that fit; cc_dense_tuning).
A candidate is timed by stepping the real batch for a few implicit steps
from copies of the given state (the caller's state is not changed); the
fastest is kept.  Results are cached in a JSON file keyed by the device
architecture, the precision, the sweep, whether any basis is exact, and the
size bucket of the batch (log2 of its free vertices and of its mesh count),
so a later process on the same kind of device and workload takes the cached
choice without timing.

This module only orders library calls and times them; every kernel runs in
libccgpu.
"""
import json
import math
import os
import time

from . import ccgpu as cg

LANES = (16, 32, 64)
ITERS_PER_GRAPH = (1, 2, 4)
DENSE_ROWS = (0, 3, 2, 1)       # 0: the most whose LDS ring fits


def default_cache_path():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "ccgpu", "autotune.json")


def cache_key(device_arch, precision, sweep, any_dense, n_free, n_meshes):
    return "|".join([str(device_arch), "fp64" if precision == cg.FP64 else "fp32",
                     "gs" if sweep == cg.SWEEP_COLORED_GS else "jacobi",
                     "exact" if any_dense else "sparse",
                     f"nf2^{int(round(math.log2(max(n_free, 1))))}",
                     f"meshes2^{int(round(math.log2(max(n_meshes, 1))))}"])


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(ctx, choice):
    cg.cc_batch_tuning(ctx, int(choice["lanes"]), int(choice["iters_per_graph"]))
    cg.cc_dense_tuning(ctx, int(choice["dense_rows"]), int(choice.get("dense_chunk", 0)))


def tune(ctx, mesh_ids, xs, vs, bcs, dt, params, tol, gravity, n_free, any_dense, any_sparse, steps=2,
         cache_path=None, device_arch=None, use_cache=True):
    """Choose and apply the fastest tuning for this batch.  xs, vs: the start
    state (device tensors; copied, not changed); bcs: per step t = 1..steps a
    list of Dirichlet target tensors; any_dense / any_sparse: whether the
    batch holds exact / R-hop bases (lane counts matter only for the
    latter, rows per workgroup only for the former).  Returns (choice, table
    of timings, or None when taken from the cache)."""
    import torch
    cache_path = cache_path or default_cache_path()
    if device_arch is None:
        device_arch = torch.cuda.get_device_properties(xs[0].device).gcnArchName
    key = cache_key(device_arch, params.precision, params.sweep, any_dense, n_free, len(mesh_ids))
    table = _load(cache_path) if use_cache else {}
    if key in table:
        apply(ctx, table[key])
        return table[key], None
    lanes = LANES if any_sparse else (16,)
    rows = DENSE_ROWS if any_dense else (0,)
    timings = []
    best = None
    for ln in lanes:
        for ipg in ITERS_PER_GRAPH:
            for dr in rows:
                choice = {"lanes": ln, "iters_per_graph": ipg, "dense_rows": dr}
                apply(ctx, choice)
                x1 = [x.clone() for x in xs]
                v1 = [v.clone() for v in vs]
                # one untimed step builds the plan and the graph
                cg.cc_step_batch(ctx, mesh_ids, x1, v1, bcs[0], dt, params, tol, gravity=gravity)
                x1 = [x.clone() for x in xs]
                v1 = [v.clone() for v in vs]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for t in range(steps):
                    cg.cc_step_batch(ctx, mesh_ids, x1, v1, bcs[t], dt, params, tol, gravity=gravity)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / steps
                timings.append(dict(choice, ms_per_step=round(ms, 3)))
                if best is None or ms < best[1]:
                    best = (choice, ms)
    choice = dict(best[0], ms_per_step=round(best[1], 3))
    apply(ctx, choice)
    if use_cache:
        table = _load(cache_path)
        table[key] = choice
        _save(cache_path, table)
    return choice, timings

