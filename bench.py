#!/usr/bin/env python
"""Benchmark of the Coordinate Condensation hot path on one MI355X.

Workload (default, "bar21x6x6_Esweep"): four 21x6x6 tet bars (756 vertices,
3000 tets, x=0 face clamped, gravity, rho 1000, nu 0.45, h = 1/60) with
E = 1e4, 1e5, 1e6, 1e7, each with its exact perturbation basis.  One bench
step advances all four bars by one implicit Euler step, each solved by plain
Coordinate Condensation (Jacobi sweeps with backtracking line search) to
rel|grad E| <= 1e-6.  Inputs are resident on the GPU before timing starts.

Prints one JSON line: vertex updates per second (value), time to tolerance
per bar-step, the roofline position of the dominant kernel (timed live with
HIP events on the library's stream) and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-rel‖∇E‖≤1e-6 per step and vertex-updates/s; "
          "learned+batched vs plain CC")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
E_SWEEP = (1e4, 1e5, 1e6, 1e7)
TOL = 1e-6


def block_pattern(s):
    """Row lengths (diagonal included) of the free-vertex block Hessian, by vertex id."""
    fixed = s.fixed.astype(bool)
    nbr = [set() for _ in range(s.n)]
    for e in s.elems:
        fr = [int(a) for a in e if not fixed[a]]
        for a in fr:
            nbr[a].update(fr)
    return np.array([len(nbr[i]) for i in range(s.n)])


def kernel_models(scenes, prec_bytes):
    """Algorithmic bytes and flops per launch (summed over the meshes of one
    launch group) of the kernels of one Jacobi iteration."""
    S = prec_bytes
    out = {}
    byts = {"cc_prep": 0.0, "elem_hess": 0.0, "assemble": 0.0, "gradient": 0.0, "cc_update": 0.0,
            "energy": 0.0}
    flops = dict.fromkeys(byts, 0.0)
    for s in scenes:
        d = s.X.shape[1]
        k = d + 1
        dd = d * d
        nb = k * (k + 1) // 2
        rl = block_pattern(s)
        free = ~s.fixed.astype(bool)
        nf = int(free.sum())
        nnzb = int(rl[free].sum())
        nnzU = nf * (nf - 1)                       # exact basis
        # cc_prep: basis (blocks + indices), block rows once, K and L out
        byts["cc_prep"] += nnzU * (dd * S + 4) + nnzb * (dd * S + 4) + nf * 2 * dd * S
        flops["cc_prep"] += 2.0 * 2 * d ** 3 * nf * (nnzb - 1)
        # cc_update: basis once, gradient once, K,L, dx out (float64)
        byts["cc_update"] += nnzU * (dd * S + 4) + nf * d * 8 * 2 + nf * 2 * dd * S
        flops["cc_update"] += 2.0 * dd * nnzU
        # element Hessian: ids, Dm^-1, volume, positions of 4 vertices, packed blocks out
        byts["elem_hess"] += s.m * (k * 4 + dd * S + S + k * d * 8 + nb * dd * S)
        flops["elem_hess"] += s.m * 3.4e3
        # assembly: element blocks in (each block read once), block rows out
        byts["assemble"] += s.m * nb * dd * S + nnzb * dd * S
        flops["assemble"] += nnzb * dd * 1.0
        # gradient: per free vertex its star (ids, Dm^-1, volume, 4 positions), g out
        byts["gradient"] += s.m * (k * 4 + dd * 8 + 8) + s.n * d * 8 * 2 + nf * d * 8
        flops["gradient"] += 4 * s.m * 150.0
        byts["energy"] += s.m * (k * 4 + dd * 8 + 8) + s.n * d * 8 * 2
        flops["energy"] += s.m * 100.0
    out["bytes"] = byts
    out["flops"] = flops
    return out


def cpu_baseline(scenes, budget_s):
    """Time the oracle on the first time step of each bar (bounded sample)."""
    from oracle import solvers as S
    from oracle.basis import exact_basis
    from oracle.fem import Problem
    from oracle.timestep import step
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    prm = S.Params(method=S.CC, sweep=S.JACOBI, line_search=True, max_iters=200)
    upd = 0
    t_solve = 0.0
    done = []
    for s in scenes:
        p = Problem.from_scene(s)
        B = exact_basis(p)                          # precompute, untimed
        x, v = s.initial_state()
        t0 = time.perf_counter()
        _, _, res, _ = step(p, x, v, s.targets(1), B, prm, TOL)
        t_solve += time.perf_counter() - t0
        upd += res.iters * p.free.size
        done.append(f"E={s.E:.0e}:{res.iters}it")
        if t_solve > budget_s:
            break
    return {"value": upd / t_solve, "unit": "vertex-updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "first implicit step of " + ", ".join(done) + " (21x6x6 bars, exact basis, "
                      f"Jacobi CC + line search to 1e-6), {t_solve:.1f} s of oracle time; "
                      f"host os.cpu_count()={os.cpu_count()}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--sweep", choices=["jacobi", "gs"], default="jacobi")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--iters-per-graph", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of this path is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    if args.warmup + args.steps > 10 or args.steps < 1:
        print("the bar trajectory has 10 steps: warmup + steps must be <= 10", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_12053_amd.ccgpu as cg
    from ccscenes import tet_bar

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)          # capturable stream for the batched graphs
    torch.cuda.set_stream(stream)
    ctx = cg.cc_create(0, stream)
    prec = cg.FP64 if args.precision == "fp64" else cg.FP32_MIXED
    sweep = cg.SWEEP_JACOBI if args.sweep == "jacobi" else cg.SWEEP_COLORED_GS
    scenes = [tet_bar(E=E) for E in E_SWEEP]
    nfree = [int((~s.fixed.astype(bool)).sum()) for s in scenes]

    def make_meshes():
        out = []
        for s in scenes:
            mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
            cg.cc_subspace_build(ctx, mid, 0, s.dt, False)   # exact basis, untimed precompute
            x, v = s.initial_state()
            xs = torch.tensor(x, dtype=torch.float64, device=dev)
            vs = torch.tensor(v, dtype=torch.float64, device=dev)
            bcs = [torch.tensor(s.targets(t), dtype=torch.float64, device=dev) for t in range(1, 11)]
            par = cg.cc_params_default(method=cg.METHOD_CC, sweep=sweep, precision=prec, line_search=1,
                                       max_iters=10000, gravity=s.gravity)
            out.append((s, mid, xs, vs, bcs, par))
        return out

    MASK = (1 << 6) - 1

    def run_plain(meshes, t, rec):
        for (s, mid, xs, vs, bcs, par), nf in zip(meshes, nfree):
            t0 = time.perf_counter()
            st, it, rg = cg.cc_step(ctx, mid, xs, vs, bcs[t], s.dt, par, TOL)
            if rec is not None:
                rec.append((st, it, rg, (time.perf_counter() - t0) * 1e3, it * nf))

    def run_batch(meshes, t, rec):
        ids = [m[1] for m in meshes]
        par = meshes[0][5]
        grav = np.stack([m[0].gravity for m in meshes])
        t0 = time.perf_counter()
        worst, its, rgs, sts = cg.cc_step_batch(ctx, ids, [m[2] for m in meshes], [m[3] for m in meshes],
                                                [m[4][t] for m in meshes], scenes[0].dt, par, TOL,
                                                gravity=grav)
        ms = (time.perf_counter() - t0) * 1e3
        if rec is not None:
            for k in range(len(meshes)):
                rec.append((int(sts[k]), int(its[k]), float(rgs[k]), ms, int(its[k]) * nfree[k]))

    def timed(runner, meshes, profile=True):
        for t in range(args.warmup):
            runner(meshes, t, None)
        torch.cuda.synchronize()
        cg.cc_profile_enable(ctx, MASK if profile else 0)
        rec = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(args.warmup, args.warmup + args.steps):
            runner(meshes, t, rec)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kern = {cg.K_NAMES[k]: cg.cc_profile_read(ctx, k) for k in range(6)}
        cg.cc_profile_enable(ctx, 0)
        return rec, elapsed, kern

    # plain CC: one mesh at a time, single-mesh launches, host-driven iteration
    plain_meshes = make_meshes()
    rec_p, el_p, kern_p = timed(run_plain, plain_meshes)
    # batched: all bars in every launch, graph replays, autotuned lanes
    batch_meshes = make_meshes()
    lanes, lane_ms = cg.cc_autotune_batch(ctx, [m[1] for m in batch_meshes], batch_meshes[0][5])
    cg.cc_batch_tuning(ctx, lanes, args.iters_per_graph)
    rec_b, el_b, _ = timed(run_batch, batch_meshes, profile=False)
    # second timed region of the same batched launches, uncaptured, with HIP
    # events around every kernel: per-kernel durations for the roofline
    prof_meshes = make_meshes()
    rec_k, el_k, kern_b = timed(run_batch, prof_meshes, profile=True)

    def summary(rec, elapsed, steps):
        upd = sum(r[4] for r in rec)
        ttt = np.array([r[3] for r in rec])
        return {"vertex_updates_per_s": round(upd / elapsed, 1),
                "ms_per_step": round(elapsed / steps * 1e3, 3),
                "time_to_tol_ms": {"median": round(float(np.median(ttt)), 3),
                                   "p90": round(float(np.percentile(ttt, 90)), 3)},
                "iters_per_bar_step": round(float(np.mean([r[1] for r in rec])), 2),
                "not_ok": sum(1 for r in rec if r[0] != cg.CC_OK)}

    plain = summary(rec_p, el_p, args.steps)
    batched = summary(rec_b, el_b, args.steps)
    # for the batch, every bar's step ends with the batch: time to tolerance = batch step time
    value = batched["vertex_updates_per_s"]

    # dominant kernel of the batched path and its roofline position:
    # algorithmic bytes (flops) = per-mesh model x that mesh's iterations
    S = 8 if prec == cg.FP64 else 4
    per_mesh = [kernel_models([s], S) for s in scenes]
    its_mesh = [0] * len(scenes)
    for k, r in enumerate(rec_k):
        its_mesh[k % len(scenes)] += r[1]
    dom = max(kern_b, key=lambda k: kern_b[k][0])
    ms_tot, launches = kern_b[dom]
    tot_bytes = sum(i * m["bytes"][dom] for i, m in zip(its_mesh, per_mesh))
    tot_flops = sum(i * m["flops"][dom] for i, m in zip(its_mesh, per_mesh))
    secs = ms_tot * 1e-3
    gbs = tot_bytes / secs / 1e9
    tfl = tot_flops / secs / 1e12
    peak_f = FP64_PEAK_TFLOPS if prec == cg.FP64 else FP32_PEAK_TFLOPS
    if tfl / peak_f >= gbs / HBM_PEAK_GBS:
        roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": peak_f, "unit": "TFLOP/s",
                "frac": round(tfl / peak_f, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    roof.update({"kernel": "kb_" + dom, "avg_launch_us": round(ms_tot / max(launches, 1) * 1e3, 2),
                 "launches": launches, "traffic": None,
                 "share_of_kernel_time": round(ms_tot / sum(v[0] for v in kern_b.values()), 3)})

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": batched["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == cg.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "bar21x6x6_Esweep", "bars": len(scenes), "E": list(E_SWEEP),
                   "verts_per_bar": scenes[0].n, "tets_per_bar": scenes[0].m, "basis": "exact",
                   "method": "cc", "sweep": args.sweep, "line_search": True, "tol": TOL,
                   "dt": scenes[0].dt, "precision": args.precision, "path": "batched",
                   "lanes": lanes, "iters_per_graph": args.iters_per_graph},
        "batched": batched,
        "plain_cc": plain,
        "speedup_batched_vs_plain": round(value / plain["vertex_updates_per_s"], 3),
        "autotune_ms": lane_ms,
        "kernel_ms_batched": {k: round(v[0], 3) for k, v in kern_b.items()},
        "batched_uncaptured_ms_per_step": round(el_k / args.steps * 1e3, 3),
        "kernel_ms_plain": {k: round(v[0], 3) for k, v in kern_p.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scenes, args.cpu_budget)
    print(json.dumps(out), flush=True)
    cg.cc_destroy(ctx)


if __name__ == "__main__":
    main()
