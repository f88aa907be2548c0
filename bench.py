#!/usr/bin/env python
"""Benchmark of the segmentation hot path on one MI355X.

One step = one pass of the whole path over one subject resident in HBM:
atlas preparation, the first cut (center test or MFMA prefilter, with its
feature preparation, sort and tile culling), the exact float32 stage on
survivors and the per-fiber argmin / label write.  The workload is the
paper-scale subject: 4,145,000 fibers against 10,000 centroids (100 bundles x
100), 21 points of float32 each, synthetic.

    python bench.py [--steps K] [--warmup W] [--mode bf16|plain|dense|...]

Prints one JSON line.  `value` is pairs/s of the headline mode (N*M per
step); every other compared mode (``mode`` or ``mode:tile``) is reported
under "modes".  The dominant kernel of each mode is timed live with HIP
events recorded by the library right around its launch
(seg_options.profile_events), on the stream the kernel runs on.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fiber-centroid pairs/s and fibers/s at 4.1M x 10k; prefilter vs plain speedup"
PEAK_FP32 = 157.3   # TFLOP/s, MI355X vector FP32 (256 CU x 4 SIMD x 32 lanes x FMA x 2.4 GHz)
PEAK_BF16 = 2500.0  # TFLOP/s dense MFMA
PEAK_FP8 = 5000.0
PEAK_HBM = 8000.0   # GB/s
WORKLOADS = {
    "small-20k-x-800": "20,000 fibers x 800 centroids (40 bundles x 20), 21 pts fp32",
    "exact-1M-x-3600": "1,000,000 fibers x 3,600 centroids (36 bundles x 100), 21 pts fp32",
    "paper-4145k-x-10k": "4,145,000 fibers x 10,000 centroids (100 bundles x 100, 20-80 mm), "
                         "21 pts fp32",
    "large-10M-x-20k": "10,000,000 fibers x 20,000 centroids (200 bundles x 100), 21 pts fp32",
    "clustered-4145k-x-10k": "4,145,000 fibers x 10,000 centroids (100 bundles x 100), 80% of "
                             "the fibers around 5 of the bundles, 21 pts fp32",
}
# kernels whose HBM traffic is summarised: counter-file kernel-name prefix -> key
TRAFFIC_KERNELS = [("seg::(anonymousnamespace)::cull_kernel<0,", "cull_kernel:bf16"),
                   ("seg::(anonymousnamespace)::cull_kernel<1,", "cull_kernel:fp16"),
                   ("seg::prefilter_kernel<0,", "prefilter_kernel:bf16"),
                   ("seg::prefilter_kernel<1,", "prefilter_kernel:fp16"),
                   ("seg::prefilter_kernel<2,", "prefilter_kernel:fp8"),
                   ("seg::plain_kernel<", "plain_kernel"),
                   ("seg::dense_kernel<1, false>", "dense_kernel"),
                   ("seg::(anonymousnamespace)::cull_fiber_kernel<1,", "cull_fiber_kernel:fp16"),
                   ("seg::(anonymousnamespace)::resample_kernel", "resample_kernel")]
KERNEL_SOURCES = ["paper_1912_11494_amd/csrc/seg_device.hpp",
                  "paper_1912_11494_amd/csrc/seg_pf.hpp",
                  "paper_1912_11494_amd/csrc/seg_kernels.hip",
                  "paper_1912_11494_amd/csrc/seg_prefilter.hip",
                  "paper_1912_11494_amd/csrc/seg_cull.hip",
                  "paper_1912_11494_amd/csrc/seg_resample.hip",
                  "paper_1912_11494_amd/csrc/seg_multi.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class Hip:
    """hipEvent_* through ctypes (the library is HIP; so are these events)."""

    def __init__(self):
        self.L = ctypes.CDLL("libamdhip64.so")
        self.L.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.L.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.L.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                               ctypes.c_void_p]
        self.L.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def event(self):
        e = ctypes.c_void_p()
        assert self.L.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def record(self, e, stream):
        assert self.L.hipEventRecord(e, stream) == 0

    def elapsed(self, a, b) -> float:
        ms = ctypes.c_float()
        assert self.L.hipEventSynchronize(b) == 0
        assert self.L.hipEventElapsedTime(ctypes.byref(ms), a, b) == 0
        return float(ms.value)


def source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is absent or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


SIZE_COUNTERS = ["TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum",
                 "TCC_EA0_RDREQ_DRAM_32B_sum"]


def write_traffic(fetch_csv: str, write_csv: str, out_path: str, sizes_csv: str = None) -> None:
    """Summarise two rocprofv3 --pmc runs of this script with --copy-probe
    (FETCH_SIZE, then WRITE_SIZE) into HBM bytes per launch.  The 1 GiB device
    copy in the same runs fixes the byte value of one counted KiB.  A third,
    optional run counts the L2's read requests to memory by size (32, 64 and
    128 bytes) and the DRAM reads in 32-byte units: the read bytes they add
    up to are recorded beside the calibrated figure as a cross-check."""
    import collections
    import csv

    def per_kernel(path, counter):
        acc = collections.defaultdict(list)
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return acc

    def copy_dispatches(path, counter):
        out = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and "copy" in r["Kernel_Name"].lower():
                    out[r["Dispatch_Id"]] = (r["Kernel_Name"], float(r["Counter_Value"]))
        return out

    fe, wr = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    # the probe's copies: the copy dispatches that wrote 1 GiB (the write
    # counter counts KiB), matched by dispatch id in the fetch run (the two
    # runs launch the same sequence)
    gib = float(1 << 30)
    cwr = copy_dispatches(write_csv, "WRITE_SIZE")
    cfe = copy_dispatches(fetch_csv, "FETCH_SIZE")
    probe = [d for d, (_, v) in cwr.items() if abs(v * 1024.0 - gib) < 1e-3 * gib and d in cfe]
    if not probe:
        raise SystemExit("no 1 GiB copy in the counter files: run with --copy-probe")
    fk = sum(cfe[d][1] for d in probe) / len(probe)
    wk = sum(cwr[d][1] for d in probe) / len(probe)
    cf = gib / (fk * 1024.0)
    cw = gib / (wk * 1024.0)
    out = {"calibration": {"kernel": cwr[probe[0]][0], "dispatches": len(probe), "fetch_kib": fk,
                           "write_kib": wk, "bytes_per_kib_fetch": cf, "bytes_per_kib_write": cw,
                           "note": "a 1 GiB device copy (reads 1 GiB, writes 1 GiB) fixes "
                                   "the byte value of one counted KiB"}}
    for prefix, key in TRAFFIC_KERNELS:
        # the launch that bench.py times: statistics off (template flag false)
        ks = [k for k in fe if k.replace(" ", "").removeprefix("void").startswith(
              prefix.replace(" ", "")) and "true" not in k]
        if not ks:
            continue
        k = ks[0]
        f = sum(fe[k]) / len(fe[k])
        w = sum(wr.get(k, [0.0])) / max(1, len(wr.get(k, [0.0])))
        out[key] = {"kernel": k, "fetch_kib": f, "write_kib": w,
                    "bytes_per_launch": f * 1024.0 * cf + w * 1024.0 * cw,
                    "source_hash": source_hash()}
    if sizes_csv:
        sz = {c: per_kernel(sizes_csv, c) for c in SIZE_COUNTERS}

        def sizes_of(vals):
            n32, n64, n128, d32 = (sum(v) / len(v) for v in vals)
            return {"rdreq_32b": n32, "rdreq_64b": n64, "rdreq_128b": n128, "dram_32b": d32,
                    "read_bytes_by_size": 32.0 * n32 + 64.0 * n64 + 128.0 * n128,
                    "dram_read_bytes": 32.0 * d32}

        # the copy: dispatches of the copy kernel whose requests add up to
        # about 1 GiB (the probe's, not torch's small copies)
        cops = [k for k in sz[SIZE_COUNTERS[0]] if "copy" in k.lower()]
        for k in cops:
            per = [32.0 * a + 64.0 * b + 128.0 * c for a, b, c in
                   zip(sz[SIZE_COUNTERS[0]][k], sz[SIZE_COUNTERS[1]][k], sz[SIZE_COUNTERS[2]][k])]
            big = [i for i, v in enumerate(per) if abs(v - gib) < 0.05 * gib]
            if big:
                rs = sizes_of([[sz[c][k][i] for i in big] for c in SIZE_COUNTERS])
                out["calibration"]["request_sizes"] = dict(rs, dispatches=len(big))
                break
        for prefix, key in TRAFFIC_KERNELS:
            if key not in out:
                continue
            k = out[key]["kernel"]
            if all(k in sz[c] for c in SIZE_COUNTERS):
                out[key]["request_sizes"] = sizes_of([sz[c][k] for c in SIZE_COUNTERS])
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    log(f"wrote {out_path}")


# kernels whose counters are summarised: counter-file kernel-name prefix -> key
COUNTER_KERNELS = [("seg::(anonymousnamespace)::cull_kernel<1,false,false,false>", "cull_kernel:fp16"),
                   ("seg::(anonymousnamespace)::cull_fiber_kernel<1,false,false>", "cull_fiber_kernel:fp16"),
                   ("seg::(anonymousnamespace)::rs_scatter_kernel", "rs_scatter_kernel"),
                   ("seg::(anonymousnamespace)::rs_hist_kernel", "rs_hist_kernel"),
                   ("seg::plain_kernel<4,512,false>", "plain_kernel"),
                   ("seg::dense_kernel<1,false>", "dense_kernel"),
                   ("seg::prefilter_kernel<1,16,2,1,false,false>", "prefilter_kernel:fp16"),
                   ("seg::(anonymousnamespace)::resample_kernel", "resample_kernel")]
N_CU = 256


def write_counters(csv_paths, out_path: str) -> dict:
    """Summarise rocprofv3 --pmc counter files (one pass each) per kernel:
    each counter averaged over the kernel's dispatches, and ratios derived
    from them (wait and issue fractions of the wave cycles, instructions per
    wave, matrix-core busy fraction, MFMA FLOPs)."""
    import collections
    import csv

    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    names = {}
    for path in csv_paths:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                k = r["Kernel_Name"].replace(" ", "").removeprefix("void")
                for prefix, key in COUNTER_KERNELS:
                    if k.startswith(prefix.replace(" ", "")):
                        acc[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
                        names[key] = r["Kernel_Name"]
    out = {}
    for key, cs in acc.items():
        c = {n: sum(v) / len(v) for n, v in cs.items()}
        d = {}

        def ratio(name, a, b, scale=1.0):
            if a in c and b in c and c[b] > 0:
                d[name] = scale * c[a] / c[b]

        ratio("wait_any_frac", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES")
        ratio("wait_inst_any_frac", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")
        ratio("active_inst_any_frac", "SQ_ACTIVE_INST_ANY", "SQ_WAVE_CYCLES")
        ratio("active_valu_frac", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES")
        ratio("active_vmem_frac", "SQ_ACTIVE_INST_VMEM", "SQ_WAVE_CYCLES")
        ratio("active_lds_frac", "SQ_ACTIVE_INST_LDS", "SQ_WAVE_CYCLES")
        ratio("wave_cycles_per_wave", "SQ_WAVE_CYCLES", "SQ_WAVES")
        for n in ("VALU", "SALU", "VMEM_RD", "VMEM_WR", "LDS", "SMEM", "MFMA"):
            ratio(f"insts_{n.lower()}_per_wave", f"SQ_INSTS_{n}", "SQ_WAVES")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in c and c.get("GRBM_GUI_ACTIVE", 0) > 0:
            d["mfma_busy_frac"] = c["SQ_VALU_MFMA_BUSY_CYCLES"] / (c["GRBM_GUI_ACTIVE"] * N_CU * 4)
        if "SQ_INSTS_VALU_MFMA_MOPS_F16" in c:
            d["mfma_f16_flop"] = c["SQ_INSTS_VALU_MFMA_MOPS_F16"] * 512
        out[key] = {"kernel": names[key], "dispatches": max(len(v) for v in cs.values()),
                    "counters": c, "derived": d, "source_hash": source_hash()}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    log(f"wrote {out_path}")
    return out


def time_mode(P, hip, f, c, b, t, mode, steps, warmup, tile=0, metric=0):
    import torch

    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    n = f.shape[0]
    out = (torch.empty(n, dtype=torch.int32, device=f.device),
           torch.empty(n, dtype=torch.float32, device=f.device))
    for _ in range(warmup):
        P.segment(f, c, b, t, mode=mode, tile=tile, out=out, metric=metric)
    torch.cuda.synchronize()
    # the steps alone (no events inside: each event recorded between two
    # kernels holds the queue a few microseconds), then the same number of
    # steps again with the library's events around the dominant kernel
    e0, e1 = hip.event(), hip.event()
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    hip.record(e0, sh)
    for k in range(steps):
        P.segment(f, c, b, t, mode=mode, tile=tile, out=out, metric=metric)
    hip.record(e1, sh)
    torch.cuda.synchronize()
    h1 = time.perf_counter()
    total_ms = hip.elapsed(e0, e1)
    pairs = [(hip.event(), hip.event()) for _ in range(steps)]
    arrs = [(ctypes.c_void_p * 2)(a.value, z.value) for a, z in pairs]
    for k in range(steps):
        P.segment(f, c, b, t, mode=mode, tile=tile, out=out, metric=metric,
                  events=ctypes.addressof(arrs[k]))
    torch.cuda.synchronize()
    kern = [hip.elapsed(a, z) for a, z in pairs]
    return {
        "ms_per_step": total_ms / steps,
        "host_ms_per_step": (h1 - h0) * 1e3 / steps,
        "kernel_ms": sum(kern) / steps,
        "kernel_ms_min": min(kern),
        "kernel_ms_max": max(kern),
    }, out


def batch_inputs(workers):
    """Atlases and subjects of the batch workload (drawn before torch starts)."""
    import synth

    wl = "batch-16-subjects-x-2-atlases"
    atl = synth.workload_atlases(wl)
    seed = synth.workload_seed(wl)
    t0 = time.time()
    subs = [synth.make_fibers(atl, sp, seed, subject_idx=i, workers=workers)
            for i, sp in enumerate(synth.workload_subjects(wl))]
    log(f"generated {wl}: {sum(len(f) for f in subs)} fibers in {time.time() - t0:.1f}s")
    return atl, subs


def bench_batch(args, atl, subs, P, hip):
    """The batch workload: 16 subjects (0.3M-4.1M fibers) against two atlases
    (3,600 and 10,000 centroids), one label per (fiber, atlas).  Times the
    batch entry point on its default route (fp16, tile-culled: subjects in
    chunks of at most 2^22 fibers, each chunk's payloads computed once and
    sorted together, then one culled pass per atlas, all in a cached HIP graph),
    its graph-captured flattened launches (bf16 streaming, plain), and one
    call per (subject, atlas) pair, plain and tile-culled; every route's
    labels and distances are compared with the sequential plain calls."""
    import torch

    wl = "batch-16-subjects-x-2-atlases"
    d = torch.device("cuda:0")
    gf = [torch.from_numpy(f).to(d) for f in subs]
    nf = sum(int(f.shape[0]) for f in gf)
    ga = [P.Atlas(torch.from_numpy(a.centroids).to(d), torch.from_numpy(a.bundle_id).to(d),
                  torch.from_numpy(a.thresholds).to(d)) for a in atl]
    pairs = nf * sum(a.n_centroids for a in atl)
    sh = torch.cuda.current_stream().cuda_stream

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = hip.event(), hip.event()
        hip.record(e0, sh)
        for _ in range(steps):
            fn()
        hip.record(e1, sh)
        torch.cuda.synchronize()
        return hip.elapsed(e0, e1) / steps

    def new_outs():
        return [[(torch.empty(f.shape[0], dtype=torch.int32, device=d),
                  torch.empty(f.shape[0], dtype=torch.float32, device=d)) for _ in ga] for f in gf]

    res, outs_of = {}, {}
    steps, warmup = max(1, args.steps // 4), 1
    for mode, tile in (("fp16", 0), ("bf16", 0), ("bf16", 1), ("plain", 0)):
        outs = new_outs()
        ms = timed(lambda: P.segment_batch(ga, gf, mode=mode, tile=tile, outs=outs), steps, warmup)
        key = f"batch {mode}:{tile}"
        res[key] = {"ms": ms, "pairs_per_s": pairs / (ms * 1e-3), "fibers_per_s": nf / (ms * 1e-3)}
        outs_of[key] = outs
        log(f"{key}: {ms:.2f} ms")
    for mode in ("plain", "fp16"):
        outs = new_outs()

        def seq():
            for i, f in enumerate(gf):
                for a, at in enumerate(ga):
                    at.segment(f, mode=mode, out=outs[i][a])

        ms = timed(seq, steps, warmup)
        key = f"sequential {mode}"
        res[key] = {"ms": ms, "pairs_per_s": pairs / (ms * 1e-3), "fibers_per_s": nf / (ms * 1e-3)}
        outs_of[key] = outs
        log(f"{key} (one call per subject and atlas): {ms:.2f} ms")
    ref = outs_of["sequential plain"]

    def ndiff(o, k):
        return int(sum(int((o[i][a][k] != ref[i][a][k]).sum()) for i in range(len(gf))
                       for a in range(len(ga))))

    head = "batch fp16:0"
    for a in ga:
        a.close()
    return {"workload": f"{wl}: {nf:,} fibers, 3,600 + 10,000 centroids", "fibers": nf,
            "pairs": pairs, "headline": head, "ms": res[head]["ms"],
            "fibers_per_s": res[head]["fibers_per_s"], "pairs_per_s": res[head]["pairs_per_s"],
            "vs_sequential_plain": res["sequential plain"]["ms"] / res[head]["ms"],
            "vs_sequential_culled": res["sequential fp16"]["ms"] / res[head]["ms"],
            "steps": steps, "paths": res,
            "label_diffs_vs_sequential_plain": {k: ndiff(o, 0) for k, o in outs_of.items()},
            "dist_diffs_vs_sequential_plain": {k: ndiff(o, 1) for k, o in outs_of.items()}}


def bench_subject(args, wl, at, fib, P, hip, modes_list, tag):
    """One more single-subject workload (the large 10M x 20,000 subject, the
    clustered-density subject): each mode timed against the plain form, with
    survivors per fiber, the fraction of pairs the bound was evaluated on,
    exact-stage drains per wave of 64 sorted rows (the survivor queue drains
    once at the end, and again each time it fills), accepted pairs (a pair a
    prefilter dropped would be missing from its count: false discards =
    plain's accepted pairs minus the mode's) and label / distance differences
    against the plain form.  ``dense`` runs one timed step."""
    import torch

    d = torch.device("cuda:0")
    f = torch.from_numpy(fib).to(d)
    c = torch.from_numpy(at.centroids).to(d)
    b = torch.from_numpy(at.bundle_id).to(d)
    t = torch.from_numpy(at.thresholds).to(d)
    N, M = fib.shape[0], at.n_centroids
    steps, warmup = max(1, args.steps // 4), 1
    modes, outs = {}, {}
    for mode in modes_list:
        ms, wu = (1, 0) if mode == "dense" else (steps, warmup)
        r, out = time_mode(P, hip, f, c, b, t, mode, ms, wu)
        P.segment(f, c, b, t, mode=mode, stats=True)
        st = P.query_stats()
        modes[mode] = {"ms_per_step": r["ms_per_step"], "kernel_ms": r["kernel_ms"],
                       "pairs_per_s": N * M / (r["ms_per_step"] * 1e-3),
                       "fibers_per_s": N / (r["ms_per_step"] * 1e-3),
                       "survivors_per_fiber": st["filter_pass"] / N,
                       "accepted_pairs": st["accepted"],
                       "bound_pairs_frac": st["bound_pairs"] / st["pairs"],
                       "exact_drains_per_wave": st["drains"] / ((N + 63) // 64)}
        outs[mode] = out
        log(f"{tag} {mode}: {r['ms_per_step']:.3f} ms/step, "
            f"{modes[mode]['survivors_per_fiber']:.2f} survivors per fiber")
    ref = outs["plain"]
    for mode, x in modes.items():
        x["label_diffs_vs_plain"] = int((outs[mode][0] != ref[0]).sum().item())
        x["dist_diffs_vs_plain"] = int((outs[mode][1] != ref[1]).sum().item())
        # (the dense form evaluates every pair exactly and counts no stages)
        x["false_discards"] = (None if mode == "dense" else
                               modes["plain"]["accepted_pairs"] - x["accepted_pairs"])
        if mode == "dense":
            x["accepted_pairs"] = None
    foot = footprint(P, f, c, b, t, outs["fp16"])
    del f, c, b, t, outs, ref
    torch.cuda.empty_cache()
    return {"workload": f"{wl}: {WORKLOADS[wl]}", "fibers": N, "centroids": M, "steps": steps,
            "modes": modes, "headline": "fp16", "device_bytes": foot}


def footprint(P, f, c, b, t, out):
    """Device bytes of a call: the caller's inputs and outputs, and the library
    scratch it holds for the current stream after the call."""
    inputs = sum(int(x.numel() * x.element_size()) for x in (f, c, b, t))
    outputs = sum(int(x.numel() * x.element_size()) for x in out)
    scratch = P.scratch_bytes()
    return {"inputs": inputs, "outputs": outputs, "library_scratch": scratch,
            "peak_total": inputs + outputs + scratch,
            "scratch_per_fiber": scratch / max(1, int(f.shape[0]))}


def bench_prepared(P, hip, f, c, b, t, head, args, N, ref_labels):
    """The headline form against a prepared atlas (seg_atlas_create once, then
    one seg_segment_atlas per step): the atlas-side work (its checks, frame,
    centroid order, columns) is done once, as when many subjects meet one
    atlas.  Reported beside the one-shot step, which stays the headline."""
    import torch

    hmode, _, htile = head.partition(":")
    if hmode in ("plain", "dense"):
        return None
    sh = torch.cuda.current_stream().cuda_stream
    n = f.shape[0]
    out = (torch.empty(n, dtype=torch.int32, device=f.device),
           torch.empty(n, dtype=torch.float32, device=f.device))
    atlas = P.Atlas(c, b, t)
    for _ in range(args.warmup):
        atlas.segment(f, mode=hmode, tile=int(htile or 0), out=out)
    torch.cuda.synchronize()
    e0, e1 = hip.event(), hip.event()
    hip.record(e0, sh)
    for _ in range(args.steps):
        atlas.segment(f, mode=hmode, tile=int(htile or 0), out=out)
    hip.record(e1, sh)
    torch.cuda.synchronize()
    ms = hip.elapsed(e0, e1) / args.steps
    diffs = int((out[0].cpu() != ref_labels.cpu()).sum().item())
    atlas.close()
    log(f"prepared atlas on {head}: {ms:.3f} ms/step, {diffs} labels differ from the one-shot call")
    return {"ms_per_step": ms, "pairs_per_s": N * int(c.shape[0]) / (ms * 1e-3), "mode": head,
            "label_diffs_vs_one_shot": diffs}


def bench_multi(P, hip, f, c, b, t, head, args, N, np):
    """Every bundle each fiber passes (CSR rows and bundle counts) on the
    headline form; each call ends by reading the entry count back."""
    import torch

    hmode, _, htile = head.partition(":")
    if hmode not in ("bf16", "fp16", "fp8"):
        return None
    sh = torch.cuda.current_stream().cuda_stream
    atlas = P.Atlas(c, b, t)
    for _ in range(args.warmup):
        out = atlas.segment_multi(f, mode=hmode, tile=int(htile or 0))
    torch.cuda.synchronize()
    e0, e1 = hip.event(), hip.event()
    hip.record(e0, sh)
    for _ in range(args.steps):
        out = atlas.segment_multi(f, mode=hmode, tile=int(htile or 0))
    hip.record(e1, sh)
    torch.cuda.synchronize()
    ms = hip.elapsed(e0, e1) / args.steps
    off = out[0].cpu().numpy()
    per = np.bincount(np.diff(off))
    atlas.close()
    log(f"several labels on {head}: {ms:.3f} ms, {int(off[-1])} entries")
    return {"ms": ms, "mode": head, "entries": int(off[-1]), "pairs_per_s": N * int(c.shape[0]) /
            (ms * 1e-3), "fibers_by_bundle_count": {str(k): int(v) for k, v in enumerate(per)}}


def bench_resample(P, hip, f, at, c, b, t, wl, head, args, N, np):
    """Raw streamlines of the workload's subject (0.2 mm steps, drawn on the
    device) to 21 points: the resampling kernel alone, HIP events on its
    stream, and resampling + segmentation in one library call."""
    import torch

    import synth

    sh = torch.cuda.current_stream().cuda_stream
    pts, off = synth.raw_streamlines_torch(f, synth.workload_seed(wl))
    npts = pts.shape[0]
    out = torch.empty((N, 21, 3), dtype=torch.float32, device=f.device)
    for _ in range(args.warmup):
        P.resample(pts, off, out=out)
    torch.cuda.synchronize()
    evs = [(hip.event(), hip.event()) for _ in range(args.steps)]
    for e0, e1 in evs:
        hip.record(e0, sh)
        P.resample(pts, off, out=out)
        hip.record(e1, sh)
    torch.cuda.synchronize()
    kern = [hip.elapsed(e0, e1) for e0, e1 in evs]
    ms = sum(kern) / len(kern)
    alg_bytes = 12 * npts + 8 * (N + 1) + 4 * 63 * N
    ach = alg_bytes / (ms * 1e-3) / 1e9
    # raw streamlines to labels in one call (resample + the headline mode)
    atlas = P.Atlas(c, b, t)
    hmode, _, htile = head.partition(":")
    lab = (torch.empty(N, dtype=torch.int32, device=f.device),
           torch.empty(N, dtype=torch.float32, device=f.device))
    for _ in range(args.warmup):
        atlas.segment_streamlines(pts, off, mode=hmode, tile=int(htile or 0), fibers=out, out=lab)
    torch.cuda.synchronize()
    e0, e1 = hip.event(), hip.event()
    hip.record(e0, sh)
    for _ in range(args.steps):
        atlas.segment_streamlines(pts, off, mode=hmode, tile=int(htile or 0), fibers=out, out=lab)
    hip.record(e1, sh)
    torch.cuda.synchronize()
    e2e = hip.elapsed(e0, e1) / args.steps
    res = {"ms": ms, "kernel_ms_min": min(kern), "kernel_ms_max": max(kern),
           "streamlines": N, "points": npts, "streamlines_per_s": N / (ms * 1e-3),
           "points_per_s": npts / (ms * 1e-3),
           "roofline": {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM, "unit": "GB/s",
                        "frac": ach / PEAK_HBM, "traffic": traffic_for("resample_kernel"),
                        "kernel": "resample_kernel", "alg_bytes": alg_bytes},
           "resample_plus_segment_ms": e2e, "segment_mode": head}
    log(f"resample: {npts} points in {ms:.3f} ms ({ach:.0f} GB/s algorithmic), "
        f"with segmentation {e2e:.3f} ms")
    if not args.no_cpu:
        import oracle

        # the oracle on every streamline of the subject (about half a second
        # of 16 host threads)
        ns = N
        off_h = off[:ns + 1].cpu().numpy()
        sp = pts[:int(off_h[-1])].cpu().numpy()
        thr = oracle.get().max_threads()
        h0 = time.perf_counter()
        want = oracle.resample_f32(sp, off_h, threads=thr)
        dt = time.perf_counter() - h0
        got = out[:ns].cpu().numpy()
        res["cpu_baseline"] = {"value": ns / dt, "unit": "streamlines/s", "cores": thr,
                               "kind": "oracle",
                               "sample": f"all {ns:,} of {N:,} streamlines "
                                         f"({int(off_h[-1]):,} points), fixed-point arc "
                                         f"length, OpenMP {thr} threads; {dt:.2f} s"}
        res["sample_mismatches_vs_oracle"] = int((~((got == want) | (np.isnan(got) &
                                                   np.isnan(want)))).any(axis=(1, 2)).sum())
    del pts, off
    atlas.close()
    return res


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(fib, at, ref, N, M, args, np):
    """The CPU oracle on the host cores: the paper's progressive discard on
    every fiber with all threads, the same on a sixteenth of the fibers with
    one thread, and the brute-force definition on a 1% fixed-seed sample with
    all threads (each about 10 s of CPU work or less)."""
    import oracle

    O = oracle.get()
    thr = O.max_threads()
    ns = N if args.cpu_sample <= 0 else min(args.cpu_sample, N)
    h0 = time.perf_counter()
    l_cpu, _, _ = O.segment_f32(fib[:ns], at.centroids, at.bundle_id, at.thresholds,
                                mode=oracle.CUT, threads=thr)
    dt = time.perf_counter() - h0
    cpu = {"value": ns * M / dt, "unit": "pairs/s", "cores": thr, "kind": "oracle",
           "sample": f"{'all' if ns == N else 'first'} {ns:,} of {N:,} fibers x all {M:,} "
                     f"centroids, float32, the paper's progressive discard (tests 1-4), "
                     f"OpenMP {thr} threads; {dt:.1f} s",
           "fibers_per_s": ns / dt, "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
           "labels_match_gpu": bool(np.array_equal(l_cpu, ref[0][:ns]))}
    log(f"cpu oracle: {ns} fibers in {dt:.1f}s ({cpu['value']:.3e} pairs/s, {thr} threads)")
    n1 = max(1, ns // 16)
    h0 = time.perf_counter()
    l1, _, _ = O.segment_f32(fib[:n1], at.centroids, at.bundle_id, at.thresholds,
                             mode=oracle.CUT, threads=1)
    dt1 = time.perf_counter() - h0
    cpu["one_thread"] = {"value": n1 * M / dt1, "unit": "pairs/s", "cores": 1,
                         "sample": f"first {n1:,} fibers, progressive discard, 1 thread; "
                                   f"{dt1:.1f} s",
                         "labels_match_gpu": bool(np.array_equal(l1, ref[0][:n1]))}
    log(f"cpu oracle, 1 thread: {n1} fibers in {dt1:.1f}s")
    rng = np.random.default_rng(11494)
    idx = np.sort(rng.choice(N, max(1, N // 100), replace=False))
    h0 = time.perf_counter()
    lb, _, _ = O.segment_f32(fib[idx], at.centroids, at.bundle_id, at.thresholds,
                             mode=oracle.BRUTE, threads=thr)
    dtb = time.perf_counter() - h0
    cpu["brute"] = {"value": len(idx) * M / dtb, "unit": "pairs/s", "cores": thr,
                    "sample": f"{len(idx):,} fibers drawn with seed 11494 (1%), the definition "
                              f"(every point of every pair), {thr} threads; {dtb:.1f} s; "
                              f"all {N:,} fibers would take about {dtb * N / len(idx):.0f} s",
                    "labels_match_gpu": bool(np.array_equal(lb, ref[0][idx]))}
    log(f"cpu oracle, brute force: {len(idx)} fibers in {dtb:.1f}s")
    return cpu


def alg_flops(mode, st, n, m, kfeat=None):
    """Algorithmic FLOPs of the dominant kernel per launch (8 FLOP per point
    distance: 3 sub, 3 mul, 2 add; 2 per multiply-add of the matrix product).
    The tile-culled prefilter evaluates its bound only on `bound_pairs`."""
    if mode == "dense":
        return 328.0 * n * m  # 41 distinct point distances per pair
    exact = 32.0 * st["filter_pass"] + 64.0 * st["test2_pass"] + 224.0 * st["test3_pass"]
    if mode == "plain":
        return 8.0 * n * m + exact
    return 2.0 * kfeat * st["bound_pairs"]  # the exact stage is a kernel of its own


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper-4145k-x-10k", choices=list(WORKLOADS))
    ap.add_argument("--mode", default=None, help="headline mode (default: fastest built)")
    ap.add_argument("--compare", default="plain,dense,bf16,fp16,fp8,bf16_oriented,fp16:1,bf16:1",
                    help="modes to time, `mode` (library tile) or `mode:tile`")
    ap.add_argument("--variants", default="tn,dir,tn+dir",
                    help="metric variants timed on the headline mode (Eq. 3 length "
                         "normalisation `tn`, section 2.4 direction inference `dir`)")
    ap.add_argument("--batch", action="store_true",
                    help="time only the batch workload (16 subjects x 2 atlases)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch workload leg (16 subjects x 2 atlases)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large-subject leg (10M fibers x 20,000 centroids)")
    ap.add_argument("--no-clustered", action="store_true",
                    help="skip the clustered-density leg (80%% of the fibers around 5%% of the "
                         "bundles)")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="processes drawing the synthetic inputs; 1 under a profiler, whose "
                         "preloaded library has initialised the GPU before this script runs")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the several-labels leg (every bundle a fiber passes)")
    ap.add_argument("--no-resample", action="store_true",
                    help="skip the resampling leg (raw streamlines to 21 points)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="fibers of the workload the CPU oracle is timed on (0: all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--traffic-from", nargs="+", metavar="CSV",
                    help="only summarise rocprofv3 counter files (FETCH_SIZE, WRITE_SIZE and, "
                         "optionally, read requests by size) into profiles/traffic.json")
    ap.add_argument("--counters-from", nargs="+", metavar="CSV",
                    help="only summarise rocprofv3 --pmc counter files (one per pass) into "
                         "profiles/counters.json")
    args = ap.parse_args()
    if args.traffic_from:
        if len(args.traffic_from) not in (2, 3):
            raise SystemExit("--traffic-from FETCH_CSV WRITE_CSV [SIZES_CSV]")
        fcsv, wcsv = args.traffic_from[:2]
        write_traffic(fcsv, wcsv, os.path.join(ROOT, "profiles", "traffic.json"),
                      args.traffic_from[2] if len(args.traffic_from) == 3 else None)
        return
    if args.counters_from:
        write_counters(args.counters_from, os.path.join(ROOT, "profiles", "counters.json"))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "this library segments one subject per GPU and has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth

    # every input is drawn before torch starts (the generator forks workers)
    W = max(1, args.gen_workers)
    if args.batch:
        atl, subs = batch_inputs(W)
        import paper_1912_11494_amd as P

        line = bench_batch(args, atl, subs, P, Hip())
        print(json.dumps({"metric": "fiber-centroid pairs/s, batch of 16 subjects x 2 atlases",
                          "value": line["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
                          "steps": line["steps"], "warmup": 1, "ms_per_step": line["ms"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f16+f32", "data": "synthetic",
                          "config": {"workload": line["workload"], "fibers": line["fibers"]},
                          "batch": line}), flush=True)
        return
    wl = args.workload
    at = synth.workload_atlases(wl)[0]
    subj = synth.workload_subjects(wl)[0]
    t0 = time.time()
    fib = synth.make_fibers([at], subj, synth.workload_seed(wl), workers=W)
    log(f"generated {wl}: {fib.shape[0]} fibers x {at.n_centroids} centroids "
        f"in {time.time() - t0:.1f}s")
    large_in = batch_in = clus_in = None
    if wl == "paper-4145k-x-10k" and not args.no_clustered:
        wl_c = "clustered-4145k-x-10k"
        at_c = synth.workload_atlases(wl_c)[0]
        t0 = time.time()
        fib_c = synth.make_fibers([at_c], synth.workload_subjects(wl_c)[0],
                                  synth.workload_seed(wl_c), workers=W)
        log(f"generated {wl_c}: {fib_c.shape[0]} fibers in {time.time() - t0:.1f}s")
        clus_in = (at_c, fib_c)
    if wl == "paper-4145k-x-10k" and not args.no_large:
        wl_l = "large-10M-x-20k"
        at_l = synth.workload_atlases(wl_l)[0]
        t0 = time.time()
        fib_l = synth.make_fibers([at_l], synth.workload_subjects(wl_l)[0],
                                  synth.workload_seed(wl_l), workers=W)
        log(f"generated {wl_l}: {fib_l.shape[0]} fibers in {time.time() - t0:.1f}s")
        large_in = (at_l, fib_l)
    if wl == "paper-4145k-x-10k" and not args.no_batch:
        batch_in = batch_inputs(W)

    import torch

    import paper_1912_11494_amd as P

    hip = Hip()
    d = torch.device("cuda:0")
    f = torch.from_numpy(fib).to(d)
    c = torch.from_numpy(at.centroids).to(d)
    b = torch.from_numpy(at.bundle_id).to(d)
    t = torch.from_numpy(at.thresholds).to(d)
    N, M = fib.shape[0], at.n_centroids

    if args.copy_probe:
        # a copy of known size: reads 1 GiB and writes 1 GiB per launch
        src = torch.empty(1 << 28, dtype=torch.float32, device=d).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    modes = {}
    outs = {}
    for spec in [m for m in args.compare.split(",") if m]:
        mode, _, tile = spec.partition(":")
        tile = int(tile or 0)
        try:
            P.segment(f, c, b, t, mode=mode, tile=tile)
        except P.SegError as e:
            log(f"mode {spec}: not available ({e})")
            continue
        torch.cuda.synchronize()
        r, out = time_mode(P, hip, f, c, b, t, mode, args.steps, args.warmup, tile)
        P.segment(f, c, b, t, mode=mode, tile=tile, stats=True)
        st = P.query_stats()
        r["tile"] = tile
        r["pairs_per_s"] = N * M / (r["ms_per_step"] * 1e-3)
        r["fibers_per_s"] = N / (r["ms_per_step"] * 1e-3)
        r["survivors_per_fiber"] = st["filter_pass"] / N if mode != "dense" else None
        r["accepted_pairs"] = st["accepted"] if mode != "dense" else None
        r["stats"] = st
        modes[spec] = r
        outs[spec] = (out[0].cpu().numpy(), out[1].cpu().numpy())
        r["labelled"] = int((outs[spec][0] >= 0).sum())
        log(f"mode {spec}: {r['ms_per_step']:.3f} ms/step, kernel {r['kernel_ms']:.3f} ms, "
            f"{r['pairs_per_s']:.3e} pairs/s")

    if not modes:
        raise SystemExit("no mode could run")
    ref = outs.get("plain") or next(iter(outs.values()))
    diffs = {m: int((o[0] != ref[0]).sum()) for m, o in outs.items()}
    ddiffs = {m: int((o[1] != ref[1]).sum()) for m, o in outs.items()}

    head = args.mode
    if head is None:
        prod = [m for m in ("bf16", "fp16", "plain") if m in modes]
        head = min(prod, key=lambda m: modes[m]["ms_per_step"])
    r = modes[head]

    def mfma_roofline(spec):
        """The prefilter product of mode `spec`: algorithmic width 15 features
        (symmetric map, 4 point groups) or 2 orders x 63 coordinates (oriented)."""
        mode = spec.split(":")[0]
        x = modes[spec]
        peak = PEAK_FP8 if mode == "fp8" else PEAK_BF16
        kf = {"bf16_oriented": 126}.get(mode, 15)
        ach = alg_flops(mode, x["stats"], N, M, kf) / (x["kernel_ms"] * 1e-3) / 1e12
        culled = x["stats"]["bound_pairs"] < x["stats"]["pairs"]
        kname = "cull_kernel" if culled else "prefilter_kernel"
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": traffic_for(f"{kname}:{mode}"), "kernel": kname,
                "kernel_ms": x["kernel_ms"],
                "bound_pairs_frac": x["stats"]["bound_pairs"] / x["stats"]["pairs"]}

    def cull_roofline(spec):
        """The tile-culled kernel against HBM: per launch, each sorted row's
        permutation entry and payload row (4 + 32 bytes; 4 + 16 + 8 with
        1-byte codes), the record of each fiber with a survivor (252 bytes),
        and the label and distance of each labelled fiber (8 bytes).  The
        centroid records it re-reads are cache-resident (2.5 MB)."""
        mode = spec.split(":")[0]
        x = modes[spec]
        st = x["stats"]
        row = 4 + (28 if mode == "fp8" else 36)
        alg = N * row + st["survivor_rows"] * 252 + x["labelled"] * 8
        ach = alg / (x["kernel_ms"] * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM, "unit": "GB/s",
                "frac": ach / PEAK_HBM, "traffic": traffic_for(f"cull_kernel:{mode}"),
                "kernel": "cull_kernel", "kernel_ms": x["kernel_ms"], "alg_bytes": alg,
                "bound_pairs_frac": st["bound_pairs"] / st["pairs"],
                "mfma": {k: v for k, v in mfma_roofline(spec).items()
                         if k in ("achieved", "peak", "unit", "frac")}}

    if head in ("dense", "plain"):
        ach = alg_flops(head, r["stats"], N, M) / (r["kernel_ms"] * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32, "unit": "TFLOP/s",
                    "frac": ach / PEAK_FP32, "traffic": traffic_for(f"{head}_kernel"),
                    "kernel": f"{head}_kernel", "kernel_ms": r["kernel_ms"]}
        dtype = "f32"
    elif modes[head]["stats"]["bound_pairs"] < modes[head]["stats"]["pairs"]:
        roofline = cull_roofline(head)
        dtype = {"fp8": "fp8+f32", "fp16": "f16+f32"}.get(head.split(":")[0], "bf16+f32")
    else:
        roofline = mfma_roofline(head)
        dtype = {"fp8": "fp8+f32", "fp16": "f16+f32"}.get(head.split(":")[0], "bf16+f32")
    # the compute-bound kernels of the other forms, for reference
    for spec in (f"{head}:1", "fp16:1", "bf16:1"):
        if spec in modes and spec != head:
            roofline["streaming_prefilter"] = dict(mfma_roofline(spec), mode=spec)
            break
    if "dense" in modes:
        dm = modes["dense"]
        a_d = alg_flops("dense", None, N, M) / (dm["kernel_ms"] * 1e-3) / 1e12
        roofline["exact_stage_dense"] = {"achieved": a_d, "peak": PEAK_FP32, "unit": "TFLOP/s",
                                         "frac": a_d / PEAK_FP32, "kernel_ms": dm["kernel_ms"],
                                         "traffic": traffic_for("dense_kernel")}

    # metric variants on the headline form: same path, variant decision in the exact stage
    variants = {}
    hmode, _, htile = head.partition(":")
    for v in [x for x in args.variants.split(",") if x]:
        rv, out = time_mode(P, hip, f, c, b, t, hmode, args.steps, args.warmup, int(htile or 0),
                            metric=v)
        lv, dv = out[0].cpu().numpy(), out[1].cpu().numpy()
        variants[v] = {"ms_per_step": rv["ms_per_step"], "kernel_ms": rv["kernel_ms"],
                       "pairs_per_s": N * M / (rv["ms_per_step"] * 1e-3),
                       "vs_exact_ms": rv["ms_per_step"] / r["ms_per_step"],
                       "labelled": int((lv >= 0).sum()),
                       "label_diffs_vs_exact": int((lv != outs[head][0]).sum())}
        log(f"variant {v} on {head}: {rv['ms_per_step']:.3f} ms/step, "
            f"{variants[v]['label_diffs_vs_exact']} labels differ from Eq. 2")

    # device bytes of the headline: its call again, then the library scratch held
    hmode, _, htile = head.partition(":")
    hout = P.segment(f, c, b, t, mode=hmode, tile=int(htile or 0))
    torch.cuda.synchronize()
    foot = footprint(P, f, c, b, t, hout)
    del hout
    prepared = bench_prepared(P, hip, f, c, b, t, head, args, N, torch.from_numpy(outs[head][0]))
    multi = None if args.no_multi else bench_multi(P, hip, f, c, b, t, head, args, N, np)
    resample = None if args.no_resample else bench_resample(P, hip, f, at, c, b, t, wl, head,
                                                            args, N, np)

    large = batch = clustered = None
    if clus_in is not None:
        clustered = bench_subject(args, "clustered-4145k-x-10k", *clus_in, P, hip,
                                  ("fp16", "plain", "dense"), "clustered")
        del clus_in
    if large_in is not None:
        large = bench_subject(args, "large-10M-x-20k", *large_in, P, hip,
                              ("fp16", "bf16", "fp8", "plain"), "large")
        del large_in
    if batch_in is not None:
        batch = bench_batch(args, *batch_in, P, hip)
        del batch_in

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(fib, at, ref, N, M, args, np)

    plain_ms = modes.get("plain", {}).get("ms_per_step")
    speed = {m: plain_ms / modes[m]["ms_per_step"] for m in modes
             if plain_ms and m not in ("plain", "dense")}
    line = {
        "metric": METRIC,
        "value": r["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{wl}: {WORKLOADS[wl]}", "fibers": N, "centroids": M,
                   "bundles": at.n_bundles, "mode": head},
        "fibers_per_s": r["fibers_per_s"],
        "prefilter_vs_plain_speedup": speed,
        "label_diffs_vs_plain": diffs,
        "dist_diffs_vs_plain": ddiffs,
        "modes": {m: {k: v for k, v in x.items() if k != "stats"} | {"stats": x["stats"]}
                  for m, x in modes.items()},
        "roofline": roofline,
        "variants": variants,
        "prepared_atlas": prepared,
        "multi": multi,
        "resample": resample,
        "device_bytes": foot,
        "large": large,
        "clustered": clustered,
        "batch": batch,
        "cpu_baseline": cpu,
        "source_hash": source_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
