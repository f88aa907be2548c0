"""Host logic of bench.py that needs no GPU: the HBM-traffic table built from
two rocprofv3 counter files (FETCH_SIZE, then WRITE_SIZE) and the 1 GiB copy
that calibrates them."""
import csv
import json
import sys
from pathlib import Path

sys.path.insert(0, str(Path(__file__).resolve().parents[1]))

import bench  # noqa: E402

CULL = "void seg::(anonymous namespace)::cull_kernel<1, false>(seg::CullJob, unsigned long long*)"
CULL_STATS = "void seg::(anonymous namespace)::cull_kernel<1, true>(seg::CullJob, unsigned long long*)"
# a non-template kernel: its name carries no return type
RESAMPLE = ("seg::(anonymous namespace)::resample_kernel(float const*, long, long const*, long, "
            "float*, unsigned int*)")
COPY = "__amd_rocclr_copyBuffer"


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for d, k, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": counter,
                        "Counter_Value": v})


def test_traffic_table(tmp_path):
    gib_kib = float(1 << 20)
    # the copy's fetch counter reads half its bytes (2 bytes per counted
    # unit), its write counter all of them; a small copy is not the probe
    fetch = [(1, COPY, gib_kib / 2), (2, COPY, 10.0), (3, CULL, 1000.0), (4, CULL, 1200.0),
             (5, CULL_STATS, 9999.0), (6, RESAMPLE, 500.0)]
    write = [(1, COPY, gib_kib), (2, COPY, 10.0), (3, CULL, 40.0), (4, CULL, 60.0),
             (5, CULL_STATS, 9999.0), (6, RESAMPLE, 70.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    bench.write_traffic(str(fp), str(wp), str(out))
    d = json.loads(out.read_text())
    cal = d["calibration"]
    assert cal["dispatches"] == 1
    assert abs(cal["bytes_per_kib_fetch"] - 2.0) < 1e-12
    assert abs(cal["bytes_per_kib_write"] - 1.0) < 1e-12
    # the timed launch (statistics off), averaged over its launches
    c = d["cull_kernel:fp16"]
    assert c["kernel"] == CULL
    assert abs(c["bytes_per_launch"] - (1100.0 * 1024 * 2 + 50.0 * 1024)) < 1e-6
    # found without a return type in its name
    r = d["resample_kernel"]
    assert r["kernel"] == RESAMPLE
    assert abs(r["bytes_per_launch"] - (500.0 * 1024 * 2 + 70.0 * 1024)) < 1e-6
    assert r["source_hash"] == bench.source_hash()
    assert "cull_kernel:bf16" not in d


def test_traffic_request_sizes(tmp_path):
    """The optional third pass: read requests by size add up to read bytes per
    launch, the probe copy's found among the copies by its 1 GiB."""
    gib = float(1 << 30)
    fetch = [(1, COPY, gib / 2048), (2, CULL, 1000.0)]
    write = [(1, COPY, gib / 1024), (2, CULL, 40.0)]
    # (32 B, 64 B, 128 B requests, DRAM 32-byte units) per dispatch
    sizes = {1: (COPY, (0.0, 0.0, gib / 128, gib / 32)), 2: (CULL, (100.0, 50.0, 10.0, 300.0)),
             3: (CULL, (300.0, 150.0, 30.0, 500.0)), 4: (COPY, (4.0, 0.0, 0.0, 4.0))}
    fp, wp, sp, out = (tmp_path / n for n in ("f.csv", "w.csv", "s.csv", "t.json"))
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    with open(sp, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for d, (k, vals) in sizes.items():
            for c, v in zip(bench.SIZE_COUNTERS, vals):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c,
                            "Counter_Value": v})
    bench.write_traffic(str(fp), str(wp), str(out), str(sp))
    d = json.loads(out.read_text())
    rc = d["calibration"]["request_sizes"]
    assert rc["dispatches"] == 1
    assert rc["read_bytes_by_size"] == gib and rc["dram_read_bytes"] == gib
    r = d["cull_kernel:fp16"]["request_sizes"]
    assert r["rdreq_32b"] == 200.0 and r["rdreq_64b"] == 100.0 and r["rdreq_128b"] == 20.0
    assert r["read_bytes_by_size"] == 32.0 * 200 + 64.0 * 100 + 128.0 * 20
    assert r["dram_read_bytes"] == 32.0 * 400


def test_counter_table(tmp_path):
    """Counter passes summarised per kernel: each counter averaged over the
    kernel's dispatches, ratios derived from them, other kernels left out."""
    cull = "void seg::(anonymous namespace)::cull_kernel<1, false, false, false>(seg::CullJob)"
    stats = "void seg::(anonymous namespace)::cull_kernel<1, true, false, false>(seg::CullJob)"
    p1, p2 = tmp_path / "a.csv", tmp_path / "b.csv"
    with open(p1, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for d, v in ((1, 100.0), (2, 300.0)):
            w.writerow({"Dispatch_Id": d, "Kernel_Name": cull, "Counter_Name": "SQ_WAVES",
                        "Counter_Value": 10.0})
            w.writerow({"Dispatch_Id": d, "Kernel_Name": cull, "Counter_Name": "SQ_WAVE_CYCLES",
                        "Counter_Value": v})
            w.writerow({"Dispatch_Id": d, "Kernel_Name": cull, "Counter_Name": "SQ_WAIT_ANY",
                        "Counter_Value": v / 2})
        w.writerow({"Dispatch_Id": 3, "Kernel_Name": stats, "Counter_Name": "SQ_WAVES",
                    "Counter_Value": 99.0})
    with open(p2, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        w.writerow({"Dispatch_Id": 1, "Kernel_Name": cull, "Counter_Name": "SQ_INSTS_MFMA",
                    "Counter_Value": 40.0})
    out = bench.write_counters([str(p1), str(p2)], str(tmp_path / "c.json"))
    c = out["cull_kernel:fp16"]
    assert c["counters"]["SQ_WAVE_CYCLES"] == 200.0
    assert abs(c["derived"]["wait_any_frac"] - 0.5) < 1e-12
    assert abs(c["derived"]["wave_cycles_per_wave"] - 20.0) < 1e-12
    assert abs(c["derived"]["insts_mfma_per_wave"] - 4.0) < 1e-12
    assert set(out) == {"cull_kernel:fp16"}
