#!/usr/bin/env python
"""HBM traffic of the dominant benchmark kernel from hardware counters.

Run mode (under rocprofv3 --pmc): steps the benchmark workload (four 21x6x6
bars, E = 1e4 .. 1e7, exact bases, batched Jacobi CC, 64 lanes) with one
iteration per step, so that every condensation launch covers all four bars,
then copies a buffer of known size (the calibration kernel).  With
`--workload beam` it steps the 81x21x21 twisted beam instead (R = 1 patch
basis, float32 local arithmetic, 16 lanes), one iteration per step, for the
sparse condensation kernel `kb_prep`.

Trace-summary mode: Markdown table of a `rocprofv3 --kernel-trace --stats`
run of bench.py, with the condensation kernels' average over the last
dispatches (the uncaptured region bench.py times with HIP events) beside the
figure bench.py printed.

Summarize mode: reads the counter CSVs of a FETCH_SIZE run and a WRITE_SIZE
run, scales each counter by the ratio of known to counted bytes of the copy
kernel, and prints a Markdown summary with the per-launch bytes of the
condensation kernels (kb_prep_dm + kb_dm_finish) and the hash of the kernel
source they were measured on.  bench.py reports the traffic only while that
hash matches the current source.

    cd /tmp && export TMPDIR=/tmp          # R: repository root, OUT: an output folder
    timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/ctr_fetch -o run -- python -u $R/bench_counters.py
    timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/ctr_write -o run -- python -u $R/bench_counters.py
    python $R/bench_counters.py --summarize $OUT/ctr_fetch $OUT/ctr_write > $R/profiles/traffic_kb_prep_dm_bar21x6x6_fp64.md
    # the same three commands with `--workload beam` after bench_counters.py -> traffic_kb_prep_beam81x21x21_fp32.md
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 512 * 1024 * 1024      # calibration copy: read and written once each
COPY_REPS = 4
KERNELS = {"bars": ("kb_prep_dm", "kb_dm_finish"),
           "beam": ("kb_prep<", "kb_elem_hess<", "kb_assemble<", "kb_update<", "kb_gradient<",
                    "kb_energy_grad<")}
SOURCE = os.path.join(ROOT, "paper_2510_12053_amd", "csrc", "cc_kernels.hip")


def source_hash():
    with open(SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def run_beam(steps):
    import numpy as np
    import torch
    import paper_2510_12053_amd.ccgpu as cg
    from ccscenes import twist_beam
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = cg.cc_create(0, stream)
    s = twist_beam()
    mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
    cg.cc_subspace_build(ctx, mid, 1, s.dt, False)
    x, v = s.initial_state()
    xs, vs = torch.tensor(x, device=dev), torch.tensor(v, device=dev)
    cg.cc_batch_tuning(ctx, 16, 0)
    par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, precision=cg.FP32_MIXED,
                               line_search=1, max_iters=1)
    for t in range(1, steps + 1):
        cg.cc_step_batch(ctx, [mid], [xs], [vs], [torch.tensor(s.targets(t), device=dev)], s.dt, par,
                         1e-12, gravity=np.zeros((1, 3)))
        torch.cuda.synchronize()
        print(f"step {t} done", flush=True)
    copy_calibration(dev)
    cg.cc_destroy(ctx)


def copy_calibration(dev):
    import torch
    n = COPY_BYTES // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(COPY_REPS):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy done", flush=True)


def run(steps):
    import numpy as np
    import torch
    import paper_2510_12053_amd.ccgpu as cg
    from ccscenes import tet_bar
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = cg.cc_create(0, stream)
    scenes = [tet_bar(E=E) for E in (1e4, 1e5, 1e6, 1e7)]
    mids, xs, vs = [], [], []
    for s in scenes:
        mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
        cg.cc_subspace_build(ctx, mid, 0, s.dt, False)
        mids.append(mid)
        x, v = s.initial_state()
        xs.append(torch.tensor(x, device=dev))
        vs.append(torch.tensor(v, device=dev))
    cg.cc_batch_tuning(ctx, 64, 0)
    par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, line_search=1, max_iters=1)
    grav = np.stack([s.gravity for s in scenes])
    for t in range(1, steps + 1):
        bcs = [torch.tensor(s.targets(t), device=dev) for s in scenes]
        cg.cc_step_batch(ctx, mids, xs, vs, bcs, scenes[0].dt, par, 1e-12, gravity=grav)
        torch.cuda.synchronize()
        print(f"step {t} done", flush=True)
    copy_calibration(dev)
    cg.cc_destroy(ctx)


def _per_dispatch(folder, counter, kernels):
    """{kernel base name: [bytes per dispatch]} from a counter CSV (KiB -> bytes)."""
    out = {}
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    for row in csv.DictReader(open(files[0])):
        if row["Counter_Name"] != counter:
            continue
        name = row["Kernel_Name"]
        key = None
        for k in kernels:
            if k in name:
                key = k
        if key is None and "copy" in name.lower():
            key = "copy"
        if key is None:
            continue
        out.setdefault(key, []).append(float(row["Counter_Value"]) * 1024.0)
    return out


def summarize(fetch_dir, write_dir, workload):
    fe = _per_dispatch(fetch_dir, "FETCH_SIZE", KERNELS[workload])
    wr = _per_dispatch(write_dir, "WRITE_SIZE", KERNELS[workload])
    # the calibration copies are the largest copy dispatches
    cf = sorted(fe.get("copy", []))[-COPY_REPS:]
    cw = sorted(wr.get("copy", []))[-COPY_REPS:]
    sf = COPY_BYTES / (sum(cf) / len(cf))
    sw = COPY_BYTES / (sum(cw) / len(cw))
    if workload == "beam":
        summarize_beam(fe, wr, sf, sw, cf, cw)
        return
    prep_f = fe["kb_prep_dm"]
    fin_f = fe.get("kb_dm_finish", [0.0])
    prep_w = wr["kb_prep_dm"]
    fin_w = wr.get("kb_dm_finish", [0.0])
    mean = lambda v: sum(v) / len(v)
    fetch = (mean(prep_f) + mean(fin_f)) * sf
    write = (mean(prep_w) + mean(fin_w)) * sw
    rec = {"kernel": "kb_prep_dm+kb_dm_finish", "workload": "bar21x6x6_Esweep", "precision": "fp64",
           "meshes_per_launch": 4, "fetch_bytes_per_launch": round(fetch),
           "write_bytes_per_launch": round(write), "fetch_scale": round(sf, 4),
           "write_scale": round(sw, 4), "dispatches": len(prep_f), "source_sha256_16": source_hash()}
    print("# HBM traffic: exact-basis condensation, four 21x6x6 bars, float64\n")
    print("Commands (repo root `$R`, output folder `$OUT`, one MI355X):\n")
    print("```")
    print("cd /tmp && export TMPDIR=/tmp")
    print("timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/ctr_fetch -o run -- python -u $R/bench_counters.py")
    print("timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/ctr_write -o run -- python -u $R/bench_counters.py")
    print("python $R/bench_counters.py --summarize $OUT/ctr_fetch $OUT/ctr_write")
    print("```\n")
    print("Every condensation launch covers all four bars (one iteration per step).  "
          f"Counters are scaled by the calibration copy of {COPY_BYTES >> 20} MiB "
          f"(known bytes / counted bytes): FETCH_SIZE x {sf:.4f}, WRITE_SIZE x {sw:.4f}.\n")
    print("| kernel | dispatches | FETCH_SIZE raw (MB) | WRITE_SIZE raw (MB) |")
    print("|---|---|---|---|")
    print(f"| kb_prep_dm | {len(prep_f)} | {mean(prep_f) / 1e6:.2f} | {mean(prep_w) / 1e6:.3f} |")
    print(f"| kb_dm_finish | {len(fin_f)} | {mean(fin_f) / 1e6:.3f} | {mean(fin_w) / 1e6:.3f} |")
    print(f"| copy (calibration) | {len(cf)} | {mean(cf) / 1e6:.1f} | {mean(cw) / 1e6:.1f} |")
    print(f"\nScaled HBM bytes per launch: fetch {fetch / 1e6:.2f} MB, write {write / 1e6:.3f} MB.\n")
    print("traffic_json: " + json.dumps(rec))


def summarize_beam(fe, wr, sf, sw, cf, cw):
    mean = lambda v: sum(v) / len(v)
    pf, pw = fe["kb_prep<"], wr["kb_prep<"]
    fetch, write = mean(pf) * sf, mean(pw) * sw
    rec = {"kernel": "kb_prep", "workload": "beam81x21x21_twist", "precision": "fp32",
           "meshes_per_launch": 1, "fetch_bytes_per_launch": round(fetch),
           "write_bytes_per_launch": round(write), "fetch_scale": round(sf, 4),
           "write_scale": round(sw, 4), "dispatches": len(pf), "source_sha256_16": source_hash()}
    print("# HBM traffic: sparse condensation, 81x21x21 twisted beam, R = 1 basis, float32\n")
    print("Commands (repo root `$R`, output folder `$OUT`, one MI355X):\n")
    print("```")
    print("cd /tmp && export TMPDIR=/tmp")
    print("timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/ctr_fetch_beam -o run -- python -u $R/bench_counters.py --workload beam")
    print("timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/ctr_write_beam -o run -- python -u $R/bench_counters.py --workload beam")
    print("python $R/bench_counters.py --workload beam --summarize $OUT/ctr_fetch_beam $OUT/ctr_write_beam")
    print("```\n")
    print("One line-searched Jacobi iteration per step, so every `kb_prep` launch covers the whole "
          f"beam.  Counters are scaled by the calibration copy of {COPY_BYTES >> 20} MiB "
          f"(known bytes / counted bytes): FETCH_SIZE x {sf:.4f}, WRITE_SIZE x {sw:.4f}.\n")
    print("| kernel | dispatches | FETCH_SIZE raw (MB) | WRITE_SIZE raw (MB) | scaled fetch + write (MB) |")
    print("|---|---|---|---|---|")
    for k in KERNELS["beam"]:
        if k in fe and k in wr:
            print(f"| {k.rstrip('<')} | {len(fe[k])} | {mean(fe[k]) / 1e6:.2f} | {mean(wr[k]) / 1e6:.3f} | "
                  f"{(mean(fe[k]) * sf + mean(wr[k]) * sw) / 1e6:.2f} |")
    print(f"| copy (calibration) | {len(cf)} | {mean(cf) / 1e6:.1f} | {mean(cw) / 1e6:.1f} | |")
    print(f"\nScaled HBM bytes per launch: fetch {fetch / 1e6:.2f} MB, write {write / 1e6:.3f} MB.\n")
    print("traffic_json: " + json.dumps(rec))


TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -k 10 600 rocprofv3 --kernel-trace --stats "
             "--output-format csv -d $OUT/kt_bench -o run -- python -u $R/bench.py --no-cpu-baseline")


def trace_summary(folder, bench_log):
    stats = glob.glob(os.path.join(folder, "**", "*kernel_stats.csv"), recursive=True)[0]
    trace = glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(stats)))
    disp = list(csv.DictReader(open(trace)))
    b = json.loads([l for l in open(bench_log) if l.startswith("{")][-1])
    ro = b["roofline"]
    print("# Kernel statistics: four 21x6x6 bars (E = 1e4 .. 1e7), float64, plain / batched / "
          "learned+batched CC\n")
    print("Command (repo root `$R`, output folder `$OUT`, one MI355X):\n")
    print("```\n" + TRACE_CMD + "\n```\n")
    print("The profiled process runs the whole bench: warm-start data generation and training, the "
          "timed regions of plain CC (`k_*`), batched and learned+batched CC (`kb_*`, graph replays), "
          "the learned+batched launches once more uncaptured with HIP events, and last the "
          "81x21x21 beam sweep (float32 `kb_*`, sparse `kb_prep`).\n")
    print("| kernel | calls | avg (us) | min (us) | max (us) | share |")
    print("|---|---|---|---|---|---|")
    for r in rows[:24]:
        name = r["Name"][:100].replace("|", "/")
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
              f"{float(r['Percentage']):.2f}% |")

    def last(key, n):
        v = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
             for r in disp if key in r["Kernel_Name"]]
        v = v[-n:]
        return sum(v) / max(len(v), 1)
    n = ro["launches"]
    lp, lf = last("kb_prep_dm", n), last("kb_dm_finish", n)
    print(f"\nDominant kernels of the timed path: `kb_prep_dm` + `kb_dm_finish` (exact-basis "
          f"condensation).  Their last {n} dispatches (the uncaptured learned+batched region) average "
          f"{lp:.1f} + {lf:.1f} = {lp + lf:.1f} us per pair; bench.py's HIP-event average of the "
          f"same launches in this run: {ro['avg_launch_us']} us.\n")
    sel = {k: b[k] for k in ("value", "ms_per_step", "learned_batched", "batched", "plain_cc",
                             "roofline", "corotation", "fixed_corotational") if k in b}
    print("bench.py line of the profiled run (selected fields):\n\n```\n" + json.dumps(sel, indent=1)
          + "\n```")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--workload", choices=("bars", "beam"), default="bars")
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"))
    a = ap.parse_args()
    if a.summarize:
        summarize(*a.summarize, a.workload)
    elif a.trace_summary:
        trace_summary(*a.trace_summary)
    elif a.workload == "beam":
        run_beam(a.steps)
    else:
        run(a.steps)


if __name__ == "__main__":
    main()
