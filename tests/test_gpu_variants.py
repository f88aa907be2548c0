"""GPU parity of the metric variants through the C ABI: length normalisation
(Eq. 3) and direction inference (section 2.4), alone and together, in every
mode and kernel form, against the float32 oracle's variant decision, labels
and distances bit for bit."""
import sys

import numpy as np
import pytest

import inputs
import oracle
import synth
from gpu_common import to_gpu

pytestmark = pytest.mark.gpu

METRICS = {"tn": oracle.TN, "dir": oracle.DIR, "tn+dir": oracle.TN | oracle.DIR}
FORMS = [("dense", 0), ("plain", 0), ("bf16", 0), ("fp16", 0), ("fp8", 0), ("fp16", 1),
         ("bf16_oriented", 0)]


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


def _run(seg, fib, cen, bid, thr, mode, tile, metric):
    import torch

    f, c, b, t = to_gpu(fib, cen, bid, thr)
    lab, dist = seg.segment(f, c, b, t, mode=mode, tile=tile, metric=metric)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), dist.cpu().numpy()


def _assert_same(lab, dist, want, ctx):
    l32, d32 = want[0], want[1]
    bad = np.nonzero(lab != l32)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} label differences, first {bad[:5]}"
    same = (dist == d32) | (np.isinf(dist) & np.isinf(d32))
    assert same.all(), f"{ctx}: {int((~same).sum())} distance differences"


@pytest.mark.parametrize("metric", sorted(METRICS))
@pytest.mark.parametrize("mode,tile", FORMS)
def test_variant_ragged(seg, metric, mode, tile):
    fib, at = synth.small_case(5000, 12, 30, seed=41, thr_lo=4.0, thr_hi=7.0)
    want = oracle.segment_ext_f32(fib, at.centroids, at.bundle_id, at.thresholds,
                                  METRICS[metric])
    log(f"variant {metric} mode={mode} tile={tile}")
    lab, dist = _run(seg, fib, at.centroids, at.bundle_id, at.thresholds, mode, tile, metric)
    _assert_same(lab, dist, want, f"{metric} {mode}:{tile}")
    assert (lab >= 0).mean() > 0.2


def test_variants_change_results(seg):
    """Length normalisation is not the plain metric: on this set it changes
    some labels or distances, as the oracle says.  (Direction inference
    changes nothing here: the fibers are noisy copies of open curves, whose end
    points pick the same order as Eq. 2; see test_direction_closed_form.)"""
    fib, at = synth.small_case(5000, 12, 30, seed=41, thr_lo=4.0, thr_hi=7.0)
    base = oracle.segment_f32(fib, at.centroids, at.bundle_id, at.thresholds)
    for metric in ("tn", "tn+dir"):
        flags = METRICS[metric]
        want = oracle.segment_ext_f32(fib, at.centroids, at.bundle_id, at.thresholds, flags)
        assert (want[0] != base[0]).any() or (want[1] != base[1]).any(), metric
        lab, dist = _run(seg, fib, at.centroids, at.bundle_id, at.thresholds, "fp16", 0, metric)
        _assert_same(lab, dist, want, f"{metric} fp16")


@pytest.mark.parametrize("mode", ["dense", "plain", "fp16", "bf16_oriented"])
def test_length_norm_closed_form(seg, mode):
    """Collinear centered lines of lengths 40 (fiber) and 20 (centroid):
    d_ME = 10, TN = 1.25; kept at T = 11.5 with distance 11.25, dropped at T = 11."""
    a = np.zeros((21, 3), np.float32)
    a[:, 0] = (np.arange(21) - 10) * 2.0
    b = np.zeros((21, 3), np.float32)
    b[:, 0] = (np.arange(21) - 10) * 1.0
    a += np.float32(50.0)
    b += np.float32(50.0)
    fib = np.stack([a, a[::-1].copy()])
    cen = b[None]
    bid = np.zeros(1, np.int32)
    lab, dist = _run(seg, fib, cen, bid, np.array([11.5], np.float32), mode, 0, "tn")
    assert (lab == 0).all() and (dist == np.float32(11.25)).all()
    lab, dist = _run(seg, fib, cen, bid, np.array([11.0], np.float32), mode, 0, "tn")
    assert (lab == -1).all()
    lab, dist = _run(seg, fib, cen, bid, np.array([11.0], np.float32), mode, 0, 0)
    assert (lab == 0).all() and (dist == np.float32(10.0)).all()


@pytest.mark.parametrize("mode,tile", FORMS)
def test_direction_closed_form(seg, mode, tile):
    """A 300-degree arc centroid and a fiber with its end points but its
    interior reversed: the end points choose the direct order, whose largest
    distance is the diameter 2R; Eq. 2 takes the inverse order (distance R)."""
    R = 20.0
    th = np.deg2rad(np.arange(21) * 15.0)
    b = np.zeros((21, 3))
    b[:, 0] = 100.0 + R * np.cos(th)
    b[:, 1] = 100.0 + R * np.sin(th)
    b[:, 2] = 100.0
    b = b.astype(np.float32)
    a = b.copy()
    a[1:20] = b[19:0:-1]
    fib, cen, bid = a[None], b[None], np.zeros(1, np.int32)
    for T in (25.0, 45.0):
        thr = np.array([T], np.float32)
        for metric in ("dir", 0):
            flags = METRICS[metric] if metric else 0
            want = oracle.segment_ext_f32(fib, cen, bid, thr, flags)
            lab, dist = _run(seg, fib, cen, bid, thr, mode, tile, metric)
            _assert_same(lab, dist, want, f"arc T={T} {metric} {mode}:{tile}")
        plain = oracle.segment_ext_f32(fib, cen, bid, thr, 0)
        dirv = oracle.segment_ext_f32(fib, cen, bid, thr, oracle.DIR)
        assert plain[0][0] == 0 and (dirv[0][0] == -1 if T < 2 * R else dirv[1][0] > plain[1][0])


@pytest.mark.parametrize("metric", sorted(METRICS))
def test_variant_batch(seg, metric):
    import torch

    long_ = synth.make_atlas(synth.AtlasSpec(6, 9, 80.0, 200.0, 6.0, 12.0), 501)
    short = synth.make_atlas(synth.AtlasSpec(11, 10, 20.0, 80.0, 5.0, 8.0), 502)
    atl = [long_, short]
    d = torch.device("cuda:0")
    ga = [seg.Atlas(torch.from_numpy(a.centroids).to(d), torch.from_numpy(a.bundle_id).to(d),
                    torch.from_numpy(a.thresholds).to(d)) for a in atl]
    subs = [synth.make_fibers(atl, synth.SubjectSpec(n, 2.0, (0.2, 0.2)), 43, subject_idx=i)
            for i, n in enumerate([700, 1300])]
    gf = [torch.from_numpy(f).to(d) for f in subs]
    for mode, tile in (("plain", 0), ("bf16", 1), ("bf16", 0)):
        log(f"variant batch {metric} mode={mode} tile={tile}")
        outs = seg.segment_batch(ga, gf, mode=mode, tile=tile, metric=metric)
        torch.cuda.synchronize()
        for i, f in enumerate(subs):
            for a, at in enumerate(atl):
                want = oracle.segment_ext_f32(f, at.centroids, at.bundle_id, at.thresholds,
                                              METRICS[metric])
                _assert_same(outs[i][a][0].cpu().numpy(), outs[i][a][1].cpu().numpy(), want,
                             f"batch {metric} {mode} {i} {a}")


def test_unknown_metric_rejected(seg):
    fib, at = synth.small_case(100, 3, 4, seed=14)
    f, c, b, t = to_gpu(fib, at.centroids, at.bundle_id, at.thresholds)
    with pytest.raises(seg.SegError) as e:
        seg.segment(f, c, b, t, metric=4)
    assert e.value.code == -1


@pytest.mark.workloads("paper-4145k-x-10k")
def test_variants_full_size_sampled(seg):
    """Paper-scale subject (4.1M x 10k) in the benchmark's launch configuration
    for each variant; the oracle recomputes a fixed sample of fibers."""
    import torch

    wl = "paper-4145k-x-10k"
    at = synth.workload_atlases(wl)[0]
    subj = synth.workload_subjects(wl)[0]
    fib = inputs.fibers(wl)
    f, c, b, t = to_gpu(fib, at.centroids, at.bundle_id, at.thresholds)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(subj.n_fibers, 1500, replace=False))
    idx = np.concatenate([idx, np.arange(subj.n_fibers - 100, subj.n_fibers)])
    for metric, flags in METRICS.items():
        want = oracle.segment_ext_f32(fib[idx], at.centroids, at.bundle_id, at.thresholds, flags)
        for mode in ("plain", "fp16", "bf16"):
            log(f"variants full size {metric} mode {mode}")
            lab, dist = seg.segment(f, c, b, t, mode=mode, metric=metric)
            torch.cuda.synchronize()
            lab, dist = lab.cpu().numpy(), dist.cpu().numpy()
            _assert_same(lab[idx], dist[idx], want, f"full {metric} {mode}")
            ok = lab >= 0
            assert ((lab >= -1) & (lab < at.n_bundles)).all()
            assert (np.isfinite(dist) == ok).all()
            assert (dist[ok] <= at.thresholds[lab[ok]]).all()
