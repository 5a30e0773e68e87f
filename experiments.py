#!/usr/bin/env python
"""The paper's two convergence sweeps run on one MI355X (Results, Mesh
Resolution Scaling and Material Stiffness Scaling), iteration counts of
Coordinate Condensation (exact basis), JGS2 (exact basis) and plain
coordinate descent, each as the Jacobi sweep of Algorithm 1.

resolution: the quasistatic stretch of a unit square (left edge held, right
  edge moved +50% in x) at n x n vertices for n = 5 .. 29; no line search;
  rel|grad E| <= 1e-4 or 500 iterations.
stiffness:  one implicit step of a free rod (41 x 2 x 2 vertices, 1 m long)
  whose right end is struck (-0.1 m/s along the rod), E = 1e1 .. 1e6 Pa;
  backtracking line search; rel|grad E| <= 1e-6 or 10,000 iterations.
subspace:   the quasistatic cantilever (21 x 6 x 6 vertices, E = --cantilever-E, clamped at x = 0)
  bent by gravity growing to 1 g over 20 load steps (Results, Subspace
  Quality): CC with the basis fixed at rest, restarted (rebuilt from the
  current configuration every 5 steps) and corotated; Jacobi with line
  search; rel|grad E| <= 1e-6 or 5,000 iterations per step.
warmstart:  the learned warm start evaluated at beam size: the network is
  trained on 50 solver-generated episodes of 21 x 6 x 6 bars (seeds
  1000-1049, 10 steps each), then held-out episodes drawn the same way at
  81 x 21 x 21 (seeds 2000-2004, 30 steps each, exact corotated basis,
  float32 local arithmetic) are stepped with and without the proposal, CC to
  rel|grad E| <= 1e-6: iterations, acceptance and time per step.

The material is the paper's Fixed Corotational model by default (--material
snh for stable neo-Hookean).  A relative termination test replaces the
paper's absolute measures (see the package's design notes).  Prints a
Markdown table and one JSON line per sweep.

    python experiments.py [--sweep resolution|stiffness|subspace|warmstart|all] [--material fcr|snh]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SIZES = (5, 9, 13, 17, 21, 25, 29)
STIFFNESS = (1e1, 1e2, 1e3, 1e4, 1e5, 1e6)


def _solve(cg, ctx, dev, s, mid, method, line_search, max_iters, tol):
    import torch
    x, v = s.initial_state()
    xg = torch.tensor(x, dtype=torch.float64, device=dev)
    vg = torch.tensor(v, dtype=torch.float64, device=dev)
    par = cg.cc_params_default(method=method, sweep=cg.SWEEP_JACOBI, line_search=line_search,
                               max_iters=max_iters, quasistatic=int(s.quasistatic), gravity=s.gravity)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, it, rg = cg.cc_step(ctx, mid, xg, vg, torch.tensor(s.targets(1), device=dev), s.dt, par, tol)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ok = st == cg.CC_OK and np.isfinite(rg)
    return {"iters": int(it), "rel_grad": float(rg), "status": int(st), "ms": round(ms, 2), "converged": bool(ok)}


def _upload(cg, ctx, s, material):
    mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
    cg.cc_mesh_set_material(ctx, mid, cg.MATERIAL_FCR if material == "fcr" else cg.MATERIAL_SNH)
    cg.cc_subspace_build(ctx, mid, 0, s.dt, bool(s.quasistatic))    # exact basis of the step energy
    return mid


def _table(rows, key, label, methods, extra):
    print(f"| {label} | {extra[0]} | CC iterations | JGS2 iterations | CD iterations |")
    print("|---|---|---|---|---|")
    for r in rows:
        cells = []
        for name, _ in methods:
            e = r[name]
            cells.append(str(e["iters"]) if e["converged"] else f">{e['iters']} (r = {e['rel_grad']:.1e})")
        print(f"| {key(r)} | {r[extra[1]]} | " + " | ".join(cells) + " |")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--sweep", choices=("resolution", "stiffness", "subspace", "warmstart", "all"),
                    default="all")
    ap.add_argument("--eval-seeds", type=int, nargs="+", default=[2000, 2001, 2002, 2003, 2004])
    ap.add_argument("--eval-steps", type=int, default=30)
    ap.add_argument("--material", choices=("fcr", "snh"), default="fcr")
    ap.add_argument("--cantilever-E", type=float, default=1e7)
    args = ap.parse_args()

    import torch
    import paper_2510_12053_amd.ccgpu as cg
    from ccscenes import cantilever_bend, rod_impulse, stretch2d

    dev = torch.device("cuda:0")
    ctx = cg.cc_create(0, torch.cuda.Stream(device=dev))
    methods = (("CC", cg.METHOD_CC), ("JGS2", cg.METHOD_JGS2), ("CD", cg.METHOD_CD))

    if args.sweep in ("resolution", "all"):
        tol, cap = 1e-4, 500
        rows = []
        for n in SIZES:
            s = stretch2d(n=n)
            mid = _upload(cg, ctx, s, args.material)
            row = {"n": n, "verts": s.n, "free": int((~s.fixed.astype(bool)).sum())}
            for name, m in methods:
                row[name] = _solve(cg, ctx, dev, s, mid, m, 0, cap, tol)
            rows.append(row)
            print(f"resolution {n}x{n} done", flush=True)
        _table(rows, lambda r: f"{r['n']} x {r['n']}", "n x n", methods, ("free vertices", "free"))
        print(json.dumps({"experiment": "resolution_sweep_stretch2d", "material": args.material, "tol": tol,
                          "max_iters": cap, "line_search": False, "rows": rows}), flush=True)

    if args.sweep in ("stiffness", "all"):
        tol, cap = 1e-6, 10000
        rows = []
        for E in STIFFNESS:
            s = rod_impulse(E=E)
            mid = _upload(cg, ctx, s, args.material)
            row = {"E": E, "verts": s.n}
            for name, m in methods:
                row[name] = _solve(cg, ctx, dev, s, mid, m, 1, cap, tol)
            rows.append(row)
            print(f"stiffness E={E:g} done", flush=True)
        _table(rows, lambda r: f"{r['E']:.0e}", "E (Pa)", methods, ("vertices", "verts"))
        print(json.dumps({"experiment": "stiffness_sweep_rod", "material": args.material, "tol": tol,
                          "max_iters": cap, "line_search": True, "rows": rows}), flush=True)
    if args.sweep in ("subspace", "all"):
        tol, cap, every = 1e-6, 5000, 5
        s = cantilever_bend(E=args.cantilever_E)
        ga = s.meta["gravity_at"]
        variants = (("fixed", 0, False), ("restarted", 0, True), ("corotated", 1, False))
        mids = {name: _upload(cg, ctx, s, args.material) for name, _, _ in variants}
        state = {name: torch.tensor(s.X, dtype=torch.float64, device=dev) for name, _, _ in variants}
        vel = torch.zeros_like(state["fixed"])
        bc = torch.tensor(s.targets(1), device=dev)
        rows = []
        for t in range(1, s.n_steps + 1):
            row = {"step": t, "gravity": float(-ga(t)[1])}
            for name, corot, restart in variants:
                if restart and (t - 1) % every == 0:     # rebuild from the current configuration
                    cg.cc_subspace_build_at(ctx, mids[name], state[name], 0, s.dt, True)
                par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, line_search=1,
                                           max_iters=cap, quasistatic=1, gravity=ga(t), corotate=corot)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, it, rg = cg.cc_step(ctx, mids[name], state[name], vel.clone(), bc, s.dt, par, tol)
                torch.cuda.synchronize()
                row[name] = {"iters": int(it), "rel_grad": float(rg), "status": int(st),
                             "ms": round((time.perf_counter() - t0) * 1e3, 2)}
            rows.append(row)
            tipmask = s.X[:, 0] == s.X[:, 0].max()
            tip = (state["corotated"].cpu().numpy()[tipmask] - s.X[tipmask]).mean(axis=0)
            row["tip_displacement"] = [round(float(c), 4) for c in tip]
            print(f"subspace step {t} done", flush=True)
        print("| load step | gravity (m/s^2) | fixed basis | restarted every 5 | corotated | tip displacement (m) |")
        print("|---|---|---|---|---|---|")
        for r in rows:
            cells = [str(r[n]["iters"]) if r[n]["status"] == cg.CC_OK else f">{r[n]['iters']}"
                     for n, _, _ in variants]
            print(f"| {r['step']} | {r['gravity']:.3f} | " + " | ".join(cells) + f" | {r['tip_displacement']} |")
        print(json.dumps({"experiment": "subspace_quality_cantilever", "material": args.material,
                          "E": args.cantilever_E, "tol": tol,
                          "max_iters": cap, "restart_every": every, "rows": rows}), flush=True)
    if args.sweep in ("warmstart", "all"):
        warm_start_beam(cg, ctx, dev, args.eval_seeds, args.eval_steps)
    cg.cc_destroy(ctx)


WARM_MAX_ITERS = 200     # per step; a step that needs more is reported as not converged


def warm_start_beam(cg, ctx, dev, seeds, steps, tol=1e-6):
    """Held-out evaluation of the learned warm start at 81 x 21 x 21."""
    import torch
    from paper_2510_12053_amd import warmstart as W
    from ccscenes import mlp_init, warm_start_eval_scene, warm_start_train_scene
    train = [warm_start_train_scene(sd) for sd in range(1000, 1050)]
    X, T, _ = W.generate(ctx, train, 10, dev, precision=cg.FP32_MIXED)
    losses, _ = W.train(ctx, X, T, mlp_init(7), epochs=40, batch=4096, lr=2e-3)
    del X, T
    print(f"warmstart: trained, loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    rows = []
    for sd in seeds:
        s = warm_start_eval_scene(sd, n_steps=steps)
        t0 = time.perf_counter()
        mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
        cg.cc_subspace_build(ctx, mid, 0, s.dt, False)
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        row = {"seed": sd, "E": s.E, "gravity": [round(float(g), 3) for g in s.gravity],
               "twist_deg_per_step": round(float(np.rad2deg(s.meta["twist_per_step"])), 3),
               "basis_build_s": round(build, 2)}
        for name, warm in (("plain", 0), ("learned", 1)):
            x, v = s.initial_state()
            xg = torch.tensor(x, dtype=torch.float64, device=dev)
            vg = torch.tensor(v, dtype=torch.float64, device=dev)
            par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, precision=cg.FP32_MIXED,
                                       line_search=1, max_iters=WARM_MAX_ITERS, gravity=s.gravity,
                                       warm_start=warm, corotate=1)
            its, acc, acc_net, ms, bad = [], 0, 0, [], 0
            for t in range(1, steps + 1):
                bc = torch.tensor(s.targets(t), dtype=torch.float64, device=dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, it, rg = cg.cc_step(ctx, mid, xg, vg, bc, s.dt, par, tol)
                torch.cuda.synchronize()
                ms.append((time.perf_counter() - t0) * 1e3)
                its.append(int(it))
                bad += int(st != cg.CC_OK)
                tag = int(cg.cc_step_info(ctx, mid)["warm_accepted"])   # 1 network, 2 correction alone
                acc += int(tag != 0)
                acc_net += int(tag == 1)
                print(f"  seed {sd} {name} step {t}: {it} iterations, {ms[-1]:.1f} ms, status {st}", flush=True)
            row[name] = {"iters_mean": round(float(np.mean(its)), 3), "iters_median": float(np.median(its)),
                         "ms_per_step_median": round(float(np.median(ms)), 2),
                         "ms_per_step_mean": round(float(np.mean(ms)), 2), "not_ok": bad,
                         "accepted": acc, "network_taken": acc_net, "steps": steps, "iters": its}
        rows.append(row)
        print(f"warmstart seed {sd}: E {s.E:.3g}, plain {row['plain']['iters_mean']} it "
              f"{row['plain']['ms_per_step_median']} ms, learned {row['learned']['iters_mean']} it "
              f"{row['learned']['ms_per_step_median']} ms, accepted {row['learned']['accepted']}/{steps} "
              f"(network {row['learned']['network_taken']})",
              flush=True)
    print("| seed | E | plain: iterations (mean) | plain: ms/step (median) | learned: iterations (mean) "
          "| learned: ms/step (median) | proposals taken |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['seed']} | {r['E']:.3g} | {r['plain']['iters_mean']} | {r['plain']['ms_per_step_median']} | "
              f"{r['learned']['iters_mean']} | {r['learned']['ms_per_step_median']} | "
              f"{r['learned']['accepted']}/{steps} ({r['learned']['network_taken']} the network's) |")
    print(json.dumps({"experiment": "warm_start_held_out_beam81x21x21", "tol": tol, "precision": "fp32",
                      "basis": "exact, corotated", "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
