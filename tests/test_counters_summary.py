"""Host logic of the traffic summary (bench_counters.py) on synthetic counter
files: the copy calibration (known bytes over counted bytes), the bytes per
dispatch of each kernel, the read-request-size count, and the hash-stamped
traffic record bench.py reads back.  No GPU: the CSVs are written here in the
layout rocprofv3 writes them."""
import csv
import json
import os

import bench
import bench_counters as BC

MB = 1e6


def _write(folder, rows):
    os.makedirs(os.path.join(folder, "pass"), exist_ok=True)
    path = os.path.join(folder, "pass", "run_counter_collection.csv")
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter,
                        "Counter_Value": value})


PREP = "void cc::kb_prep_band<float, 3, 4, 128>(cc::BatchItem const*, ...)"
FIN = "void cc::kb_dm_finish<float, 3>(cc::BatchItem const*, ...)"
ASM = "void cc::kb_assemble<float, 3>(cc::BatchItem const*, ...)"
COPY = "void at::native::vectorized_elementwise_kernel<copy>(...)"
COPY_KIB = BC.COPY_BYTES / 1024.0


def _fixture(tmp_path):
    # FETCH_SIZE counts half the copy's bytes (a factor of 2 to calibrate);
    # WRITE_SIZE counts them all.  Three dispatches of each sweep kernel.
    fetch, write, req = [], [], []
    for _ in range(3):
        fetch += [(PREP, "FETCH_SIZE", 4000 * MB / 1024), (FIN, "FETCH_SIZE", 10 * MB / 1024),
                  (ASM, "FETCH_SIZE", 200 * MB / 1024)]
        write += [(PREP, "WRITE_SIZE", 12 * MB / 1024), (FIN, "WRITE_SIZE", 12 * MB / 1024),
                  (ASM, "WRITE_SIZE", 100 * MB / 1024)]
        # the condensation's reads as 128-byte requests, the assembly's as 64
        for k, n128, n64 in ((PREP, 8000 * MB / 128, 0), (FIN, 20 * MB / 128, 0), (ASM, 0, 200 * MB / 64)):
            req += [(k, "TCC_EA0_RDREQ_32B_sum", 0), (k, "TCC_EA0_RDREQ_64B_sum", n64),
                    (k, "TCC_EA0_RDREQ_128B_sum", n128), (k, "TCC_EA0_RDREQ_sum", n64 + n128)]
    for _ in range(BC.COPY_REPS):
        fetch.append((COPY, "FETCH_SIZE", COPY_KIB / 2))
        write.append((COPY, "WRITE_SIZE", COPY_KIB))
        n = BC.COPY_BYTES / 128
        req += [(COPY, "TCC_EA0_RDREQ_32B_sum", 0), (COPY, "TCC_EA0_RDREQ_64B_sum", 0),
                (COPY, "TCC_EA0_RDREQ_128B_sum", n), (COPY, "TCC_EA0_RDREQ_sum", n)]
    dirs = [str(tmp_path / d) for d in ("fetch", "write", "req")]
    for d, rows in zip(dirs, (fetch, write, req)):
        _write(d, rows)
    return dirs


def test_request_bytes_and_coverage(tmp_path):
    _, _, req = _fixture(tmp_path)
    rb = BC.request_bytes(req)
    assert abs(rb["kb_prep_band<"][0] - 8000 * MB) <= 1.0 and rb["kb_prep_band<"][1] == 1.0
    assert abs(rb["kb_assemble<"][0] - 200 * MB) <= 1.0
    assert abs(rb["copy"][0] - BC.COPY_BYTES) <= 1.0


def test_summary_scales_by_the_copy_and_stamps_the_source(tmp_path, monkeypatch, capsys):
    fetch, write, req = _fixture(tmp_path)
    monkeypatch.setattr(BC, "algorithmic", lambda workload: {"cc_prep": 7000 * MB, "assemble": 250 * MB,
                                                             "elem_hess": 1.0, "gradient": 1.0,
                                                             "energy_grad": 1.0})
    monkeypatch.setattr(BC, "scenes_of", lambda workload: [None] * 64)
    BC.summarize(fetch, write, "batch64", req)
    out = capsys.readouterr().out
    assert "FETCH_SIZE x 2.0000, WRITE_SIZE x 1.0000" in out
    rec = json.loads(out.split("traffic_json: ")[1].strip())
    # condensation = band kernel + finish: fetch (4000 + 10) MB x 2, write 24 MB
    assert abs(rec["fetch_bytes_per_launch"] - 8020 * MB) <= 2.0
    assert abs(rec["write_bytes_per_launch"] - 24 * MB) <= 2.0
    assert rec["source_sha256_16"] == BC.source_hash()
    assert rec["fetch_scale"] == 2.0 and rec["dispatches"] == 3
    # the assembly row: scaled fetch + write 500 MB against 250 algorithmic,
    # and by request size 300 MB (its 64-byte requests counted in full)
    row = next(l for l in out.splitlines() if l.startswith("| kb_assemble"))
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[4] == "500.00" and cells[6] == "2.00"
    assert cells[7].startswith("200.00") and cells[8] == "1.20"
    # bench.py reads the record back while the hash matches
    path = tmp_path / "traffic.md"
    path.write_text(out)
    got = bench.measured_traffic(str(path))
    assert got is not None and got["fetch_bytes_per_launch"] == rec["fetch_bytes_per_launch"]
    stale = out.replace(BC.source_hash(), "0" * 16)
    path.write_text(stale)
    assert bench.measured_traffic(str(path)) is None


def test_trace_summary_windows_the_profiled_region(tmp_path, capsys):
    """The kernel-trace summary averages the condensation dispatches that lie
    between the first two profile marks only, and measures the idle gaps
    between consecutive batched dispatches."""
    kt = tmp_path / "kt" / "host"
    kt.mkdir(parents=True)
    with open(kt / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage",
                                          "MinNs", "MaxNs", "StdDev"])
        w.writeheader()
        w.writerow({"Name": PREP, "Calls": 5, "TotalDurationNs": 5000, "AverageNs": 1000, "Percentage": 90,
                    "MinNs": 900, "MaxNs": 1100, "StdDev": 10})
    # a prep at t = 0 (before the region), two marks around three prep/finish
    # pairs, and a prep after the region: only the three inside count
    disp = [("cc::kb_prep_band<float, 3, 4, 128>", 0, 5000)]
    disp.append(("cc::k_profile_mark()", 10000, 10001))
    t = 20000
    for dur in (1000, 2000, 3000):
        disp.append(("cc::kb_prep_band<float, 3, 4, 128>", t, t + dur * 1000))
        disp.append(("cc::kb_dm_finish<float, 3>", t + dur * 1000 + 2000, t + dur * 1000 + 12000))
        t += dur * 1000 + 20000
    disp.append(("cc::k_profile_mark()", t, t + 1))
    disp.append(("cc::kb_prep_band<float, 3, 4, 128>", t + 10000, t + 10000 + 9000000))
    with open(kt / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, a, e in disp:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": a, "End_Timestamp": e})
    log = tmp_path / "bench.log"
    log.write_text("[bench] progress\n" + json.dumps({"value": 1.0, "roofline": {"launches": 3,
                                                                               "avg_launch_us": 2010.0}}) + "\n")
    BC.trace_summary(str(tmp_path / "kt"), str(log))
    out = capsys.readouterr().out
    # (1000 + 2000 + 3000) / 3 us of prep, 10 us of finish
    assert "The 3 dispatches of the uncaptured learned+batched region average 2000.0 + 10.0 = 2010.0 us" in out
    assert "HIP-event average of the same launches in this run: 2010.0 us" in out
    # gaps between consecutive kb_ dispatches: 15 us into the region, 2 us
    # prep -> finish three times, 8 us finish -> next prep twice, 18 us out
    assert "(< 50 us): 7 pairs, median 8.00 us" in out
