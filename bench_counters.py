#!/usr/bin/env python
"""HBM traffic of the sweep kernels from hardware counters, and the kernel
statistics summary of a profiled bench run.

Run mode (under rocprofv3 --pmc): steps a workload with one Jacobi iteration
per step, so that every launch of the iteration covers the whole workload,
then copies a buffer of known size (the calibration kernel):
  batch64  the 64 seed-drawn bars of the benchmark with their exact bases,
           corotated, float32 local arithmetic (kernel of record:
           kb_prep_band);
  beam     the 81x21x21 twisted beam with its exact, corotated basis,
           float32 local arithmetic.
--dense-rows sets the rows per workgroup of the condensation (the
autotuner's choice in bench.py; 0: the most that fit).

Summarize mode: reads the counter CSVs of a FETCH_SIZE run and a WRITE_SIZE
run, scales each counter by the ratio of known to counted bytes of the copy
kernel, and prints a Markdown summary: for every sweep kernel the scaled
bytes per dispatch beside its algorithmic bytes (bench.kernel_model), and a
`traffic_json` line for the condensation with the hash of the kernel source it
was measured on (bench.py reports the traffic only while that hash matches).
An optional third run of the read-request counters by size adds the fetched
bytes counted request by request, a check of the copy's factor for each
kernel (that factor comes from 128-byte requests, which FETCH_SIZE counts as
64 bytes here).

    cd /tmp && export TMPDIR=/tmp          # R: repository root, OUT: an output folder
    timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/ctr_fetch -o run -- python -u $R/bench_counters.py
    timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/ctr_write -o run -- python -u $R/bench_counters.py
    python $R/bench_counters.py --summarize $OUT/ctr_fetch $OUT/ctr_write > $R/profiles/traffic_kb_prep_band_batch64_fp32.md
    # the same three commands with `--workload beam` -> traffic_kb_prep_band_beam81x21x21_fp32.md

Trace-summary mode: Markdown table of a `rocprofv3 --kernel-trace --stats`
run of bench.py, with the condensation kernels' average over the dispatches
of the uncaptured region bench.py times with HIP events, beside bench.py's
own figure.
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
# counter kernel name fragment -> bench.kernel_model class
KERNELS = {"kb_prep_band<": "cc_prep", "kb_dm_finish<": "cc_prep", "kb_elem_hess<": "elem_hess",
           "kb_assemble<": "assemble", "kb_gradient<": "gradient", "kb_energy_grad<": "energy_grad"}
SOURCE = os.path.join(ROOT, "paper_2510_12053_amd", "csrc", "cc_kernels.hip")


def source_hash():
    with open(SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def scenes_of(workload):
    from ccscenes import batch_bars, twist_beam
    return batch_bars(64) if workload == "batch64" else [twist_beam()]


def run(workload, steps, dense_rows=0):
    import numpy as np
    import torch
    import paper_2510_12053_amd.ccgpu as cg
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    ctx = cg.cc_create(0, stream)
    scenes = scenes_of(workload)
    mids, xs, vs = [], [], []
    for s in scenes:
        mid = cg.cc_mesh_upload(ctx, s.X, s.elems, s.fixed, s.E, s.nu, s.rho)
        cg.cc_subspace_build(ctx, mid, 0, s.dt, False)
        mids.append(mid)
        x, v = s.initial_state()
        xs.append(torch.tensor(x, device=dev))
        vs.append(torch.tensor(v, device=dev))
    print("bases built", flush=True)
    cg.cc_batch_tuning(ctx, 16, 0)
    cg.cc_dense_tuning(ctx, dense_rows, 0)
    par = cg.cc_params_default(method=cg.METHOD_CC, sweep=cg.SWEEP_JACOBI, line_search=1, max_iters=1,
                               precision=cg.FP32_MIXED, corotate=1)
    grav = np.stack([s.gravity for s in scenes])
    for t in range(1, steps + 1):
        bcs = [torch.tensor(s.targets(t), device=dev) for s in scenes]
        cg.cc_step_batch(ctx, mids, xs, vs, bcs, scenes[0].dt, par, 1e-12, gravity=grav)
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


def _per_dispatch(folder, counter, unit=1024.0):
    """{kernel key: [value per dispatch]} from a counter CSV (KiB -> bytes by
    default; unit=1 keeps counts)."""
    out = {}
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    for row in csv.DictReader(open(files[0])):
        if row["Counter_Name"] != counter:
            continue
        name = row["Kernel_Name"]
        key = next((k for k in KERNELS if k in name), None)
        if key is None and "copy" in name.lower():
            key = "copy"
        if key is None:
            continue
        out.setdefault(key, []).append(float(row["Counter_Value"]) * unit)
    return out


REQ_COUNTERS = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum")


def request_bytes(req_dir):
    """{kernel key: (bytes fetched per dispatch counted by request size,
    share of read requests the three sizes account for)} from a pass of
    REQ_COUNTERS; for the copy, its COPY_REPS largest dispatches."""
    c = {n: _per_dispatch(req_dir, n, 1.0) for n in REQ_COUNTERS}
    out = {}
    for k, tot in c["TCC_EA0_RDREQ_sum"].items():
        per = []
        for i in range(len(tot)):
            n32, n64, n128 = (c[n].get(k, [0.0] * len(tot))[i] for n in REQ_COUNTERS[:3])
            per.append((32.0 * n32 + 64.0 * n64 + 128.0 * n128, n32 + n64 + n128, tot[i]))
        if k == "copy":
            per = sorted(per)[-COPY_REPS:]
        byts = sum(p[0] for p in per) / len(per)
        cover = sum(p[1] for p in per) / max(sum(p[2] for p in per), 1.0)
        out[k] = (byts, cover)
    return out


def algorithmic(workload):
    """Algorithmic bytes of one whole-workload launch of every kernel class."""
    from bench import kernel_model
    tot = {}
    for s in scenes_of(workload):
        b, _ = kernel_model(s, 4)
        b = dict(b)
        b["energy_grad"] = b["energy"] + b["gradient"]
        for k, v in b.items():
            tot[k] = tot.get(k, 0) + v
    return tot


def summarize(fetch_dir, write_dir, workload, req_dir=None):
    fe = _per_dispatch(fetch_dir, "FETCH_SIZE")
    rq = request_bytes(req_dir) if req_dir else None
    wr = _per_dispatch(write_dir, "WRITE_SIZE")
    cf = sorted(fe.get("copy", []))[-COPY_REPS:]
    cw = sorted(wr.get("copy", []))[-COPY_REPS:]
    sf = COPY_BYTES / (sum(cf) / len(cf))
    sw = COPY_BYTES / (sum(cw) / len(cw))
    mean = lambda v: sum(v) / len(v)
    # the first dispatches of a class can run before the graph warms up; the
    # iteration launches of every step are alike, so take the mean of all
    alg = algorithmic(workload)
    name = {"batch64": "the 64 seed-drawn bars of the benchmark, exact corotated bases",
            "beam": "the 81x21x21 twisted beam, exact corotated basis"}[workload]
    flag = "" if workload == "batch64" else " --workload beam"
    tag = "batch64" if workload == "batch64" else "beam81x21x21"
    print(f"# HBM traffic of the sweep kernels: {name}, float32 local arithmetic\n")
    print("Commands (repo root `$R`, output folder `$OUT`, one MI355X):\n")
    print("```")
    print("cd /tmp && export TMPDIR=/tmp")
    print(f"timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/ctr_fetch_{tag} -o run -- python -u $R/bench_counters.py{flag}")
    print(f"timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/ctr_write_{tag} -o run -- python -u $R/bench_counters.py{flag}")
    if rq is not None:
        print(f"timeout -s KILL 240 rocprofv3 --pmc {' '.join(REQ_COUNTERS)} --output-format csv "
              f"-d $OUT/ctr_req_{tag} -o run -- python -u $R/bench_counters.py{flag}")
        print(f"python $R/bench_counters.py{flag} --summarize $OUT/ctr_fetch_{tag} $OUT/ctr_write_{tag} "
              f"$OUT/ctr_req_{tag}")
    else:
        print(f"python $R/bench_counters.py{flag} --summarize $OUT/ctr_fetch_{tag} $OUT/ctr_write_{tag}")
    print("```\n")
    print("One line-searched Jacobi iteration per step, so every launch covers the whole workload.  "
          f"Counters are scaled by the calibration copy of {COPY_BYTES >> 20} MiB (known bytes / "
          f"counted bytes): FETCH_SIZE x {sf:.4f}, WRITE_SIZE x {sw:.4f}.  Algorithmic bytes: "
          "`bench.kernel_model` (compulsory bytes of one launch over the workload).\n")
    if rq is not None:
        print("The last two columns count the fetched bytes by read-request size instead "
              "(32 x TCC_EA0_RDREQ_32B + 64 x TCC_EA0_RDREQ_64B + 128 x TCC_EA0_RDREQ_128B, the "
              "three sizes covering the share of TCC_EA0_RDREQ given in brackets) plus the scaled "
              "write bytes. This count needs no calibration: FETCH_SIZE's expression counts a "
              "128-byte request as 64 bytes unless TCC_BUBBLE counts it, and the copy's factor of 2 "
              "shows that it does not here. Where the two fetch columns agree, the kernel's reads are "
              "128-byte requests and the copy's factor applies to it as well.\n")
        print("| kernel | dispatches | fetch (MB) | write (MB) | scaled fetch + write (MB) | algorithmic (MB) "
              "| ratio | fetch by request size (MB) | ratio by request size |")
        print("|---|---|---|---|---|---|---|---|---|")
    else:
        print("| kernel | dispatches | fetch (MB) | write (MB) | scaled fetch + write (MB) | algorithmic (MB) | ratio |")
        print("|---|---|---|---|---|---|---|")
    rows = {}
    for k, cls in KERNELS.items():
        if k not in fe or k not in wr:
            continue
        f, w = mean(fe[k]) * sf, mean(wr[k]) * sw
        rows[k] = (f, w)
        a = alg.get(cls, 0.0) if k != "kb_dm_finish<" else 0.0
        ratio = f"{(f + w) / a:.2f}" if a > 0 else "—"
        line = (f"| {k.rstrip('<')} | {len(fe[k])} | {mean(fe[k]) / 1e6:.2f} | {mean(wr[k]) / 1e6:.3f} | "
                f"{(f + w) / 1e6:.2f} | {a / 1e6 if a else 0:.2f} | {ratio} |")
        if rq is not None:
            rb, cov = rq.get(k, (float("nan"), 0.0))
            rr = f"{(rb + w) / a:.2f}" if a > 0 else "—"
            line += f" {rb / 1e6:.2f} ({cov:.3f}) | {rr} |"
        print(line)
    line = f"| copy (calibration) | {len(cf)} | {mean(cf) / 1e6:.1f} | {mean(cw) / 1e6:.1f} | | | |"
    if rq is not None and "copy" in rq:
        line += f" {rq['copy'][0] / 1e6:.1f} ({rq['copy'][1]:.3f}) | |"
    print(line)
    pf, pw = rows["kb_prep_band<"]
    ff, fw = rows.get("kb_dm_finish<", (0.0, 0.0))
    fetch, write = pf + ff, pw + fw
    print(f"\nCondensation (kb_prep_band + kb_dm_finish): fetch {fetch / 1e6:.1f} MB, write {write / 1e6:.2f} MB "
          f"per launch, against {alg['cc_prep'] / 1e6:.1f} MB algorithmic ({(fetch + write) / alg['cc_prep']:.3f}x).\n")
    rec = {"kernel": "kb_prep_band+kb_dm_finish", "workload": tag, "precision": "fp32",
           "mesh_iters_per_launch": len(scenes_of(workload)), "fetch_bytes_per_launch": round(fetch),
           "write_bytes_per_launch": round(write), "algorithmic_bytes_per_launch": round(alg["cc_prep"]),
           "fetch_scale": round(sf, 4), "write_scale": round(sw, 4),
           "dispatches": len(fe["kb_prep_band<"]), "source_sha256_16": source_hash()}
    print("traffic_json: " + json.dumps(rec))


TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -k 10 900 rocprofv3 --kernel-trace --stats "
             "--output-format csv -d $OUT/kt_bench -o run -- python -u $R/bench.py --no-cpu-baseline")


def trace_summary(folder, bench_log):
    stats = glob.glob(os.path.join(folder, "**", "*kernel_stats.csv"), recursive=True)[0]
    trace = glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(stats)))
    disp = list(csv.DictReader(open(trace)))
    b = json.loads([l for l in open(bench_log) if l.startswith("{")][-1])
    ro = b["roofline"]
    print("# Kernel statistics: bench.py (64-bar batch, exact bases, float32 local arithmetic; "
          "plain / batched / learned+batched CC; beam and float64 bar sections)\n")
    print("Command (repo root `$R`, output folder `$OUT`, one MI355X):\n")
    print("```\n" + TRACE_CMD + "\n```\n")
    print("| kernel | calls | avg (us) | min (us) | max (us) | share |")
    print("|---|---|---|---|---|---|")
    for r in rows[:24]:
        name = r["Name"][:100].replace("|", "/")
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
              f"{float(r['Percentage']):.2f}% |")
    # the profiled (uncaptured) learned+batched region lies between the
    # first two k_profile_mark dispatches (cc_profile_enable marks where a
    # recording starts and stops; the beam's profiled steps come later)
    n = ro["launches"]
    marks = sorted(int(r["Start_Timestamp"]) for r in disp if "k_profile_mark" in r["Kernel_Name"])
    t0, t1 = (marks[0], marks[1]) if len(marks) >= 2 else (0, 1 << 62)

    def window(key):
        return [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                for r in disp if key in r["Kernel_Name"] and t0 < int(r["Start_Timestamp"]) < t1]
    lp, lf = window("kb_prep_band<float"), window("kb_dm_finish<float")
    mp = sum(lp) / max(len(lp), 1)
    mf = sum(lf) / max(len(lf), 1)
    print(f"\nDominant kernels of the timed path: `kb_prep_band` + `kb_dm_finish` (exact-basis "
          f"condensation).  The {len(lp)} dispatches of the uncaptured learned+batched region average "
          f"{mp:.1f} + {mf:.1f} = {mp + mf:.1f} us per pair; bench.py's HIP-event average of the "
          f"same launches in this run: {ro['avg_launch_us']} us.\n")
    # idle time between consecutive batched dispatches on the device: the
    # cost a persistent kernel with grid barriers could remove.  Pairs closer
    # than 50 us belong to one queued stretch of work (graph replays or
    # uncaptured launch sequences); longer gaps are host round trips.
    kb = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in disp
                if "cc::kb_" in r["Kernel_Name"] or "kb_" in r["Kernel_Name"][:40])
    gaps = [(kb[i + 1][0] - kb[i][1]) / 1e3 for i in range(len(kb) - 1)]
    inner = sorted(g for g in gaps if 0 <= g < 50)
    busy = sum((e - a) / 1e3 for a, e, _ in kb)
    if inner:
        med = inner[len(inner) // 2]
        p90 = inner[int(0.9 * (len(inner) - 1))]
        print(f"Gaps between consecutive batched (`kb_*`) dispatches inside queued stretches (< 50 us): "
              f"{len(inner)} pairs, median {med:.2f} us, p90 {p90:.2f} us, total {sum(inner) / 1e3:.1f} ms "
              f"against {busy / 1e3:.1f} ms of `kb_*` kernel time ({100 * sum(inner) / max(busy, 1e-9):.1f}%).\n")
    sel = {k: b[k] for k in ("value", "ms_per_step", "learned_batched", "batched", "plain_cc", "roofline")
           if k in b}
    print("bench.py line of the profiled run (selected fields):\n\n```\n" + json.dumps(sel, indent=1)
          + "\n```")


SQ_PASSES = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_BUSY_CU_CYCLES SQ_INSTS_VALU SQ_INSTS_LDS "
             "SQ_INSTS_VMEM_RD SQ_WAIT_INST_ANY",
             "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_WAIT_INST_LDS SQ_WAIT_ANY SQ_LDS_IDX_ACTIVE "
             "SQ_LDS_BANK_CONFLICT SQ_LDS_ADDR_CONFLICT SQ_INSTS_SALU",
             "TCC_HIT_sum TCC_MISS_sum TCC_EA0_RDREQ_sum TCP_TCC_READ_REQ_sum")


def counters_summary(dirs, workload):
    """Markdown summary of SQ / cache counter passes on the condensation
    kernel: per-dispatch sums over the device, and the ratios the kernel's
    design is judged by."""
    tot, ndisp = {}, {}
    for d in dirs:
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            continue
        for row in csv.DictReader(open(files[0])):
            if "kb_prep_band<" not in row["Kernel_Name"]:
                continue
            c = row["Counter_Name"]
            tot[c] = tot.get(c, 0.0) + float(row["Counter_Value"])
            ndisp.setdefault(c, set()).add(row["Dispatch_Id"])
    per = {c: tot[c] / max(len(ndisp[c]), 1) for c in tot}
    name = {"batch64": "the 64 seed-drawn bars of the benchmark, exact corotated bases",
            "beam": "the 81x21x21 twisted beam, exact corotated basis"}[workload]
    flag = "" if workload == "batch64" else " --workload beam"
    print(f"# Shader and cache counters of kb_prep_band: {name}, float32 local arithmetic\n")
    print("Commands (repo root `$R`, output folder `$OUT`, one MI355X; one pass per counter group):\n")
    print("```")
    print("cd /tmp && export TMPDIR=/tmp")
    for i, grp in enumerate(SQ_PASSES):
        print(f"timeout -s KILL 240 rocprofv3 --pmc {grp} --output-format csv -d $OUT/sq{i} -o run -- "
              f"python -u $R/bench_counters.py{flag}")
    print(f"python $R/bench_counters.py{flag} --counters $OUT/sq0 $OUT/sq1 $OUT/sq2")
    print("```\n")
    print("| counter | per dispatch | dispatches |")
    print("|---|---|---|")
    for c in sorted(per):
        print(f"| {c} | {per[c]:.4g} | {len(ndisp[c])} |")
    g = lambda c: per.get(c, float("nan"))
    print("\nDerived (sums over all shader engines; SQ cycle counters tick once per four cycles "
          "per wave or per CU as their names say):\n")
    print(f"- LDS bank-conflict cycles / LDS active cycles: {g('SQ_LDS_BANK_CONFLICT') / g('SQ_LDS_IDX_ACTIVE'):.3f}")
    print(f"- VALU instructions per busy CU cycle: {g('SQ_INSTS_VALU') / g('SQ_BUSY_CU_CYCLES'):.3f} "
          "(one CU issues at most one wave64 VALU instruction per cycle over its four SIMDs)")
    print(f"- LDS instructions per VALU instruction: {g('SQ_INSTS_LDS') / g('SQ_INSTS_VALU'):.3f}")
    print(f"- wave cycles waiting on any dependency / wave cycles: {g('SQ_WAIT_INST_ANY') / g('SQ_WAVE_CYCLES'):.3f}")
    print(f"- L2 hit rate: {g('TCC_HIT_sum') / (g('TCC_HIT_sum') + g('TCC_MISS_sum')):.3f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--workload", choices=("batch64", "beam"), default="batch64")
    ap.add_argument("--dense-rows", type=int, default=0)
    ap.add_argument("--summarize", nargs="+", metavar="DIR",
                    help="FETCH_DIR WRITE_DIR [REQUEST_SIZE_DIR]")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "BENCH_LOG"))
    ap.add_argument("--counters", nargs="+", metavar="PASS_DIR")
    a = ap.parse_args()
    if a.summarize:
        if len(a.summarize) not in (2, 3):
            ap.error("--summarize takes FETCH_DIR WRITE_DIR [REQUEST_SIZE_DIR]")
        summarize(a.summarize[0], a.summarize[1], a.workload, *a.summarize[2:])
    elif a.trace_summary:
        trace_summary(*a.trace_summary)
    elif a.counters:
        counters_summary(a.counters, a.workload)
    else:
        run(a.workload, a.steps, a.dense_rows)


if __name__ == "__main__":
    main()
