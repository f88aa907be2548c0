"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Labels must match the oracle's float32 decision bit for bit and distances
must match it bit for bit (both take the correctly rounded square root of
the same float32 D); distances are also checked within 1e-5 relative of the
float64 oracle.  Sizes span several fiber tiles and centroid groups with
ragged tails; every mode and kernel configuration must give identical
outputs.
"""
import json
import os
import sys

import numpy as np
import pytest

import inputs
import oracle
import synth
from gpu_common import assert_parity, run, to_gpu

pytestmark = pytest.mark.gpu

PREFILTER_MODES = ["bf16", "fp16", "fp8", "bf16_oriented"]
FILTERED_MODES = ["plain"] + PREFILTER_MODES
ALL_MODES = ["dense"] + FILTERED_MODES


@pytest.fixture(scope="module")
def seg():
    import torch

    assert torch.cuda.is_available(), "GPU tests need the GPU"
    import paper_1912_11494_amd as P

    P.lib()
    return P


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "small_seeded_case.json")
    d = json.load(open(path))
    return (d, np.array(d["fibers"], np.float32).reshape(-1, 21, 3),
            np.array(d["centroids"], np.float32).reshape(-1, 21, 3),
            np.array(d["bundle_id"], np.int32), np.array(d["thresholds"], np.float32))


@pytest.mark.parametrize("mode", ALL_MODES)
def test_golden_case(seg, mode):
    d, fib, cen, bid, thr = _golden()
    log(f"golden mode={mode}")
    lab, dist = run(seg, fib, cen, bid, thr, mode)
    assert lab.tolist() == d["labels_f32"]
    assert np.array_equal(dist, np.array(d["dists_f32"], np.float32))


@pytest.mark.parametrize("mode", ALL_MODES)
@pytest.mark.parametrize("n,nb,per,seed", [(3001, 7, 47, 1), (1000, 40, 20, 2), (257, 3, 5, 3),
                                           (6000, 12, 30, 4)])
def test_synthetic_ragged(seg, mode, n, nb, per, seed):
    fib, at = synth.small_case(n, nb, per, seed=seed)
    log(f"synthetic mode={mode} n={n} m={nb * per} seed={seed}")
    lab, dist = run(seg, fib, at.centroids, at.bundle_id, at.thresholds, mode)
    assert_parity(lab, dist, fib, at.centroids, at.bundle_id, at.thresholds,
                  ctx=f"{mode} n={n} seed={seed}")
    assert (lab >= 0).mean() > 0.3


@pytest.mark.parametrize("mode,tiles", [("dense", [1, 2]), ("plain", [1, 2, 4]),
                                        ("bf16", [1, 2, 3, 4, 5, 6, 7]),
                                        ("fp16", [1, 2, 4, 6]), ("fp8", [1, 2, 4, 6]),
                                        ("bf16_oriented", [1, 2])])
def test_tiles_identical(seg, mode, tiles):
    fib, at = synth.small_case(5000, 10, 31, seed=9)
    outs = []
    for t in tiles:
        log(f"tile mode={mode} tile={t}")
        outs.append(run(seg, fib, at.centroids, at.bundle_id, at.thresholds, mode, tile=t))
    for lab, dist in outs[1:]:
        assert np.array_equal(lab, outs[0][0]) and np.array_equal(dist, outs[0][1])
    assert_parity(*outs[0], fib, at.centroids, at.bundle_id, at.thresholds, ctx=mode)


def _adversarial(seed=5):
    """Near-threshold, reversed, exact-copy and tied pairs."""
    rng = np.random.default_rng(seed)
    spec = synth.AtlasSpec(9, 8, 20.0, 120.0, 5.0, 9.0)
    at = synth.make_atlas(spec, seed)
    cen, bid, thr = at.centroids, at.bundle_id, at.thresholds
    fibs = []
    for k in range(600):
        c = int(rng.integers(len(cen)))
        t = rng.normal(size=3)
        r = float(thr[bid[c]]) * (1.0 + [-1e-6, 0.0, 1e-6, -1e-3, 1e-3, 0.5][k % 6])
        t *= r / np.linalg.norm(t)
        f = (cen[c].astype(np.float64) + t).astype(np.float32)
        if k % 2:
            f = f[::-1].copy()
        fibs.append(f)
    fibs.append(cen[3].copy())             # D = 0
    fibs.append(cen[4][::-1].copy())       # D = 0 through the inverse order
    fib = np.stack(fibs)
    # duplicate centroids with other bundle ids: ties must keep the lower index
    cen2 = np.concatenate([cen, cen[:10]])
    bid2 = np.concatenate([bid, (bid[:10] + 1) % spec.n_bundles]).astype(np.int32)
    return fib, cen2, bid2, thr


@pytest.mark.parametrize("mode", ALL_MODES)
def test_adversarial(seg, mode):
    fib, cen, bid, thr = _adversarial()
    log(f"adversarial mode={mode}")
    lab, dist = run(seg, fib, cen, bid, thr, mode)
    assert_parity(lab, dist, fib, cen, bid, thr, ctx=f"adversarial {mode}", check_f64=False)
    assert dist[-1] == 0 and dist[-2] == 0


@pytest.mark.parametrize("mode", ALL_MODES)
def test_special_thresholds(seg, mode):
    fib, at = synth.small_case(700, 5, 9, seed=12)
    cen, bid = at.centroids, at.bundle_id
    # T = +inf: a nearest-centroid classifier; mixed with T < 0 and T = -0.0
    thr = np.array([np.inf, -1.0, 7.0, -0.0, np.inf], np.float32)
    log(f"special thresholds mode={mode}")
    lab, dist = run(seg, fib, cen, bid, thr, mode)
    assert_parity(lab, dist, fib, cen, bid, thr, ctx=f"special {mode}", check_f64=False)
    assert not np.isin(lab, [1]).any()
    lab, dist = run(seg, fib, cen, bid, np.full(5, -3.0, np.float32), mode)
    assert (lab == -1).all() and np.isinf(dist).all()


@pytest.mark.parametrize("mode,tile", [(m, 0) for m in ALL_MODES] +
                         [(m, 1) for m in ("bf16", "fp16", "fp8")])
def test_infinite_coordinates_unvalidated(seg, mode, tile):
    """Without validation an infinite coordinate is an ordinary float32 value:
    its point distances are +inf, so the pair is accepted by a bundle with
    T = +inf (D = +inf <= T2) and by no other.  Fibers carry infinities in x,
    centroids in y (no inf - inf).  Every cut must keep these pairs; a bf16
    code of an infinite feature would make the matrix product NaN."""
    fib, at = synth.small_case(600, 5, 9, seed=23)
    fib = fib.copy()
    cen = at.centroids.copy()
    thr = at.thresholds.copy()
    # bundle 3 (centroids 27-35) always matches, and each of its centroids has
    # an infinite coordinate: it is the label of every fiber without a finite
    # match, at distance +inf
    thr[3] = np.inf
    cen[27:36:2, 7, 1] = np.inf
    cen[28:36:2, 10, 1] = -np.inf
    fib[5, 3, 0] = np.inf
    fib[77, 10, 0] = -np.inf
    fib[400, 0, 0] = np.inf
    fib[401, 20, 0] = np.inf
    log(f"infinite coordinates mode={mode} tile={tile}")
    lab, dist = run(seg, fib, cen, at.bundle_id, thr, mode, tile)
    assert_parity(lab, dist, fib, cen, at.bundle_id, thr, ctx=f"inf {mode}:{tile}",
                  check_f64=False)
    assert (lab[[5, 77, 400, 401]] == 3).all() and np.isinf(dist[[5, 77, 400, 401]]).all()
    assert (lab >= 0).all() and np.isinf(dist).sum() > 100


@pytest.mark.parametrize("mode", ALL_MODES)
def test_empty_and_single(seg, mode):
    import torch

    fib, at = synth.small_case(130, 3, 4, seed=13)
    cen, bid, thr = at.centroids, at.bundle_id, at.thresholds
    log(f"empty/single mode={mode}")
    # M = 0
    lab, dist = run(seg, fib, cen[:0], bid[:0], thr, mode)
    assert (lab == -1).all() and np.isinf(dist).all()
    # N = 0
    f, c, b, t = to_gpu(fib[:0], cen, bid, thr)
    l0, d0 = seg.segment(f, c, b, t, mode=mode)
    assert l0.numel() == 0
    # one fiber, one centroid
    lab, dist = run(seg, fib[:1], cen[:1], bid[:1] * 0, thr[:1], mode)
    assert_parity(lab, dist, fib[:1], cen[:1], bid[:1] * 0, thr[:1], ctx="1x1", check_f64=False)
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", PREFILTER_MODES)
def test_every_tile_hits(seg, mode):
    """Thresholds far above every distance: every pair survives the first cut,
    so each wave has a hit in every centroid tile (9,000 centroids: 282 tiles,
    more than a wave records during the centroid loop) and the survivor queue
    fills and drains many times.  The result is the nearest centroid."""
    fib, at = synth.small_case(300, 90, 100, seed=21)
    thr = np.full(at.n_bundles, 1000.0, np.float32)
    log(f"every tile hits mode={mode} m={at.n_centroids}")
    lab, dist = run(seg, fib, at.centroids, at.bundle_id, thr, mode)
    assert_parity(lab, dist, fib, at.centroids, at.bundle_id, thr, ctx=f"all-hit {mode}")
    assert (lab >= 0).all()


def test_validation_errors(seg):
    import torch

    fib, at = synth.small_case(100, 3, 4, seed=14)
    bid = at.bundle_id.copy()
    bid[5] = 3  # out of range for 3 bundles
    f, c, b, t = to_gpu(fib, at.centroids, bid, at.thresholds)
    with pytest.raises(seg.SegError) as e:
        seg.segment(f, c, b, t, validate=True)
    assert e.value.code == -2
    # without validation the bad centroid simply never matches
    lab, dist = seg.segment(f, c, b, t, validate=False)
    torch.cuda.synchronize()
    bid_ok = at.bundle_id.copy()
    thr_ext = np.concatenate([at.thresholds, np.array([-1.0], np.float32)])
    bid_ok[5] = 3
    l32, d32, _ = oracle.segment_f32(fib, at.centroids, bid_ok, thr_ext)
    assert np.array_equal(lab.cpu().numpy(), l32)
    bad = fib.copy()
    bad[7, 3, 1] = np.nan
    f2, c2, b2, t2 = to_gpu(bad, at.centroids, at.bundle_id, at.thresholds)
    with pytest.raises(seg.SegError) as e:
        seg.segment(f2, c2, b2, t2, validate=True)
    assert e.value.code == -3
    with pytest.raises(ValueError):
        seg.segment(f.cpu(), c, b, t)


@pytest.mark.parametrize("mode", FILTERED_MODES)
@pytest.mark.parametrize("case", ["synthetic", "adversarial"])
def test_filter_keeps_accepted_pairs(seg, mode, case):
    """Zero false discards: every pair the oracle accepts survives the first cut."""
    if case == "synthetic":
        fib, at = synth.small_case(2000, 6, 20, seed=15)
        cen, bid, thr = at.centroids, at.bundle_id, at.thresholds
    else:
        fib, cen, bid, thr = _adversarial()
    acc = oracle.accepted_pairs_f32(fib, cen, bid, thr)
    f, c, b, t = to_gpu(fib, cen, bid, thr)
    log(f"filter pairs mode={mode} case={case}")
    pairs = seg.filter_pairs(f, c, b, t, mode=mode, capacity=1 << 22)
    pairs = pairs.cpu().numpy().astype(np.int64)
    surv = set(map(tuple, pairs.tolist()))
    missing = [p for p in map(tuple, acc.tolist()) if p not in surv]
    assert not missing, f"{mode} dropped {len(missing)} accepted pairs, e.g. {missing[:3]}"
    assert len(acc) > (1000 if case == "synthetic" else 250)
    frac = len(pairs) / (len(fib) * len(cen))
    log(f"  survivors {len(pairs)} ({frac:.2e} of pairs), accepted {len(acc)}")
    if mode != "fp8":
        assert frac < 0.05, f"{mode} cut keeps {frac:.2%} of pairs"


def test_stats_and_determinism(seg):
    import torch

    fib, at = synth.small_case(4000, 8, 25, seed=16)
    f, c, b, t = to_gpu(fib, at.centroids, at.bundle_id, at.thresholds)
    lab, dist = seg.segment(f, c, b, t, mode="plain", stats=True)
    st = seg.query_stats()
    assert st["pairs"] == 4000 * 200
    assert st["accepted"] >= int((lab >= 0).sum().item())
    assert st["filter_pass"] >= st["test2_pass"] >= st["test3_pass"] >= st["accepted"]
    for _ in range(3):
        l2, d2 = seg.segment(f, c, b, t, mode="plain")
        torch.cuda.synchronize()
        assert torch.equal(l2, lab) and torch.equal(d2, dist)


@pytest.mark.workloads("small-20k-x-800", "exact-1M-x-3600", "paper-4145k-x-10k", "large-10M-x-20k",
                       "clustered-4145k-x-10k")
@pytest.mark.parametrize("wl", ["small-20k-x-800", "exact-1M-x-3600", "paper-4145k-x-10k",
                                "large-10M-x-20k", "clustered-4145k-x-10k"])
def test_full_size_sampled(seg, wl):
    """Full-size workload in the launch configuration the benchmark times;
    the oracle recomputes a fixed sample of fibers one by one.  The clustered
    subject packs 80% of its fibers around 5 of the 100 bundles, so its
    sorted waves hold many survivors (the exact stage drains its queue many
    times per wave)."""
    import torch

    at = synth.workload_atlases(wl)[0]
    subj = synth.workload_subjects(wl)[0]
    fib = inputs.fibers(wl)
    f, c, b, t = to_gpu(fib, at.centroids, at.bundle_id, at.thresholds)
    rng = np.random.default_rng(len(wl))
    idx = np.sort(rng.choice(subj.n_fibers, 3000, replace=False))
    idx = np.concatenate([idx, np.arange(subj.n_fibers - 200, subj.n_fibers)])
    o32 = oracle.segment_f32(fib[idx], at.centroids, at.bundle_id, at.thresholds, mode=oracle.CUT)
    for mode in ALL_MODES:
        if mode == "dense" and wl.split("-")[0] in ("paper", "large", "clustered"):
            continue  # 0.2-0.8 s of GPU time; covered by the smaller cases
        log(f"full size {wl} mode {mode}")
        lab, dist = seg.segment(f, c, b, t, mode=mode)
        torch.cuda.synchronize()
        lab = lab.cpu().numpy()
        dist = dist.cpu().numpy()
        assert_parity(lab[idx], dist[idx], fib[idx], at.centroids, at.bundle_id, at.thresholds,
                      ctx=f"{wl} {mode}", o32=o32)
        # any-size properties: labels in range, dists finite iff labelled, within threshold
        assert ((lab >= -1) & (lab < at.n_bundles)).all()
        assert (np.isfinite(dist) == (lab >= 0)).all()
        ok = lab >= 0
        assert (dist[ok] <= at.thresholds[lab[ok]] * (1 + 1e-6)).all()
