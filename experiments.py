#!/usr/bin/env python
"""The paper's resolution experiment run on one MI355X (Results, Mesh
Resolution Scaling): the quasistatic stretch of a unit square (left edge
held, right edge moved +50% in x) at n x n vertices for n = 5 .. 29, solved
by Coordinate Condensation (exact basis), JGS2 (exact basis) and plain
coordinate descent, each as the Jacobi sweep of Algorithm 1 without line
search, from the same start, to rel|grad E| <= TOL or MAX_ITERS iterations.

Prints a Markdown table and one JSON line.  Stable neo-Hookean material
(E = 1e5, nu = 0.4) and a relative termination test replace the paper's
Fixed Corotational model and its absolute measure, whose threshold the
stretch already nearly meets at the start in these units.

    python experiments.py
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
TOL = 1e-4
MAX_ITERS = 500


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--tol", type=float, default=TOL)
    ap.add_argument("--max-iters", type=int, default=MAX_ITERS)
    args = ap.parse_args()

    import torch
    import paper_2510_12053_amd.ccgpu as cg
    from ccscenes import stretch2d

    dev = torch.device("cuda:0")
    ctx = cg.cc_create(0, torch.cuda.Stream(device=dev))
    methods = (("CC", cg.METHOD_CC), ("JGS2", cg.METHOD_JGS2), ("CD", cg.METHOD_CD))
    rows = []
    for n in SIZES:
        s = stretch2d(n=n)
        mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
        cg.cc_subspace_build(ctx, mid, 0, s.dt, True)          # exact basis of the quasistatic energy
        row = {"n": n, "verts": s.n, "free": int((~s.fixed.astype(bool)).sum())}
        for name, m in methods:
            x, v = s.initial_state()
            xg = torch.tensor(x, dtype=torch.float64, device=dev)
            vg = torch.tensor(v, dtype=torch.float64, device=dev)
            par = cg.cc_params_default(method=m, sweep=cg.SWEEP_JACOBI, line_search=0,
                                       max_iters=args.max_iters, quasistatic=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, rg = cg.cc_step(ctx, mid, xg, vg, torch.tensor(s.targets(1), device=dev), s.dt,
                                    par, args.tol)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            ok = st == cg.CC_OK and np.isfinite(rg)
            row[name] = {"iters": int(it), "rel_grad": float(rg), "status": int(st), "ms": round(ms, 2),
                         "converged": bool(ok)}
        rows.append(row)

    print(f"| n x n | free vertices | CC iterations | JGS2 iterations | CD iterations |")
    print("|---|---|---|---|---|")
    for r in rows:
        cells = []
        for name, _ in methods:
            e = r[name]
            cells.append(str(e["iters"]) if e["converged"] else f">{e['iters']} (r = {e['rel_grad']:.1e})")
        print(f"| {r['n']} x {r['n']} | {r['free']} | " + " | ".join(cells) + " |")
    print(json.dumps({"experiment": "resolution_sweep_stretch2d", "tol": args.tol,
                      "max_iters": args.max_iters, "rows": rows}))
    cg.cc_destroy(ctx)


if __name__ == "__main__":
    main()
