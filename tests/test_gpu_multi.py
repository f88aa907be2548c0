"""GPU parity of several labels per fiber (the previous version's
classification, section 2.4) through the C ABI: CSR offsets, bundles,
distances and bundle counts equal the float32 oracle's bit for bit."""
import sys

import numpy as np
import pytest

import inputs
import oracle
import pins
import synth
from gpu_common import to_gpu

pytestmark = pytest.mark.gpu

MODES = ["bf16", "fp16", "fp8"]
METRICS = {0: 0, "tn": oracle.TN, "dir": oracle.DIR}


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


def _atlas(seg, cen, bid, thr):
    _, c, b, t = to_gpu(cen[:1], cen, bid, thr)
    return seg.Atlas(c, b, t)


def _multi(seg, fib, cen, bid, thr, mode, metric=0, max_per_fiber=8, capacity=None, tile=0):
    import torch

    atlas = _atlas(seg, cen, bid, thr)
    f = torch.from_numpy(np.ascontiguousarray(fib, np.float32)).to("cuda:0")
    out = atlas.segment_multi(f, max_per_fiber=max_per_fiber, capacity=capacity, mode=mode,
                              metric=metric, tile=tile)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in out]


def _same(got, want, ctx):
    names = ("offsets", "bundles", "dists", "bundle_counts")
    for name, g, w in zip(names, got, want):
        assert g.shape == w.shape, f"{ctx}: {name} shape {g.shape} vs {w.shape}"
        bad = np.nonzero(g != w)[0]
        assert bad.size == 0, f"{ctx}: {name} differs at {bad[:5]}"


@pytest.mark.parametrize("metric", sorted(METRICS, key=str))
@pytest.mark.parametrize("mode", MODES)
def test_multi_overlapping(seg, mode, metric):
    """Bundles that share shapes: many fibers are in two or three bundles."""
    fib, cen, bid, thr = pins._overlapping_set(np.random.default_rng(31), n=5000, nb=12, per=10)
    want = oracle.segment_multi_f32(fib, cen, bid, thr, METRICS[metric])
    log(f"multi overlapping mode={mode} metric={metric}")
    got = _multi(seg, fib, cen, bid, thr, mode, metric)
    _same(got, want, f"overlapping {mode} {metric}")
    if metric == 0:
        assert (np.diff(want[0]) >= 2).sum() > 500


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,nb,per,seed", [(3001, 7, 47, 1), (257, 3, 5, 3), (20000, 40, 20, 31)])
def test_multi_ragged(seg, mode, n, nb, per, seed):
    fib, at = synth.small_case(n, nb, per, seed=seed)
    want = oracle.segment_multi_f32(fib, at.centroids, at.bundle_id, at.thresholds)
    log(f"multi ragged mode={mode} n={n}")
    _same(_multi(seg, fib, at.centroids, at.bundle_id, at.thresholds, mode), want,
          f"ragged {mode} n={n}")


def test_multi_matches_single_label(seg):
    """The closest-bundle label of the single-label path is the member of
    smallest distance, with the same distance."""
    import torch

    fib, cen, bid, thr = pins._overlapping_set(np.random.default_rng(32), n=8000, nb=10, per=8)
    off, bun, dst, cnt = _multi(seg, fib, cen, bid, thr, "fp16")
    f, c, b, t = to_gpu(fib, cen, bid, thr)
    lab, dist = seg.segment(f, c, b, t, mode="fp16")
    torch.cuda.synchronize()
    lab, dist = lab.cpu().numpy(), dist.cpu().numpy()
    assert np.array_equal(cnt, np.bincount(bun, minlength=len(thr)))
    for i in range(len(fib)):
        bb, dd = bun[off[i]:off[i + 1]], dst[off[i]:off[i + 1]]
        if lab[i] < 0:
            assert bb.size == 0
        else:
            assert lab[i] in bb and dd.min() == dist[i]


def test_multi_capacity_and_slots(seg):
    import torch

    fib, cen, bid, thr = pins._overlapping_set(np.random.default_rng(33), n=2000, nb=8, per=6)
    want = oracle.segment_multi_f32(fib, cen, bid, thr)
    total = int(want[0][-1])
    log("multi capacity")
    # too small a capacity: SEG_ECAPACITY; the binding's retry gets it right
    with pytest.raises(seg.SegError) as e:
        _multi(seg, fib, cen, bid, thr, "bf16", capacity=total - 1)
    assert e.value.code == -9
    _same(_multi(seg, fib, cen, bid, thr, "bf16", capacity=total), want, "exact capacity")
    _same(_multi(seg, fib, cen, bid, thr, "bf16", capacity=None), want, "retry")
    # fewer slots than some fiber's bundles: SEG_ERANGE
    most = int(np.diff(want[0]).max())
    assert most >= 2
    with pytest.raises(seg.SegError) as e:
        _multi(seg, fib, cen, bid, thr, "bf16", max_per_fiber=most - 1)
    assert e.value.code == -6
    _same(_multi(seg, fib, cen, bid, thr, "bf16", max_per_fiber=most), want, "tight slots")
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", MODES)
def test_multi_all_bundles(seg, mode):
    """Infinite thresholds: every fiber in every bundle (16 bundles, 16 slots);
    every tile passes and every pair survives, so each wave drains its queue
    many times."""
    fib, at = synth.small_case(600, 16, 30, seed=34)
    thr = np.full(16, np.inf, np.float32)
    want = oracle.segment_multi_f32(fib, at.centroids, at.bundle_id, thr)
    log(f"multi all bundles mode={mode}")
    got = _multi(seg, fib, at.centroids, at.bundle_id, thr, mode, max_per_fiber=16)
    _same(got, want, f"all bundles {mode}")
    assert (np.diff(got[0]) == 16).all()


def test_multi_edges(seg):
    import torch

    fib, cen, bid, thr = pins._overlapping_set(np.random.default_rng(35), n=100, nb=4, per=3)
    log("multi edges")
    # no fibers
    off, bun, dst, cnt = _multi(seg, fib[:0], cen, bid, thr, "fp16")
    assert off.tolist() == [0] and bun.size == 0 and cnt.tolist() == [0, 0, 0, 0]
    # negative thresholds: nobody is a member
    off, bun, dst, cnt = _multi(seg, fib, cen, bid, np.full(4, -1.0, np.float32), "fp16")
    assert off[-1] == 0 and cnt.sum() == 0
    # an empty bundle in the middle
    b2 = bid.copy()
    b2[b2 == 1] = 3
    want = oracle.segment_multi_f32(fib, cen, b2, thr)
    _same(_multi(seg, fib, cen, b2, thr, "fp16"), want, "empty bundle")
    # a mode without the culled form is rejected, and so is a streaming tile
    atlas = _atlas(seg, cen, bid, thr)
    f = torch.from_numpy(fib).to("cuda:0")
    for kw in (dict(mode="plain"), dict(mode="dense"), dict(mode="fp16", tile=1)):
        with pytest.raises(seg.SegError) as e:
            atlas.segment_multi(f, **kw)
        assert e.value.code == -7


def test_multi_validation(seg):
    import torch

    fib, cen, bid, thr = pins._overlapping_set(np.random.default_rng(37), n=200, nb=4, per=3)
    atlas = _atlas(seg, cen, bid, thr)
    bad = fib.copy()
    bad[17, 3, 2] = np.inf
    log("multi validation")
    with pytest.raises(seg.SegError) as e:
        atlas.segment_multi(torch.from_numpy(bad).to("cuda:0"), mode="fp16", validate=True)
    assert e.value.code == -3
    # a valid call afterwards is unaffected
    want = oracle.segment_multi_f32(fib, cen, bid, thr)
    _same(_multi(seg, fib, cen, bid, thr, "fp16"), want, "after a rejected call")


@pytest.mark.workloads("paper-4145k-x-10k")
def test_multi_full_size_sampled(seg):
    """Paper-scale subject in the benchmark's configuration; the oracle
    recomputes the rows of a fixed sample of fibers."""
    import torch

    wl = "paper-4145k-x-10k"
    at = synth.workload_atlases(wl)[0]
    subj = synth.workload_subjects(wl)[0]
    fib = inputs.fibers(wl)
    atlas = _atlas(seg, at.centroids, at.bundle_id, at.thresholds)
    f = torch.from_numpy(fib).to("cuda:0")
    off, bun, dst, cnt = [x.cpu().numpy() for x in atlas.segment_multi(f, mode="fp16")]
    n = len(fib)
    rng = np.random.default_rng(36)
    idx = np.concatenate([np.sort(rng.choice(n, 1500, replace=False)), np.arange(n - 50, n)])
    w_off, w_bun, w_dst, _ = oracle.segment_multi_f32(fib[idx], at.centroids, at.bundle_id,
                                                      at.thresholds)
    for k, i in enumerate(idx):
        assert np.array_equal(bun[off[i]:off[i + 1]], w_bun[w_off[k]:w_off[k + 1]]), i
        assert np.array_equal(dst[off[i]:off[i + 1]], w_dst[w_off[k]:w_off[k + 1]]), i
    assert np.array_equal(cnt, np.bincount(bun, minlength=at.n_bundles))
    assert (np.diff(off) >= 0).all() and off[0] == 0 and off[-1] == len(bun)
