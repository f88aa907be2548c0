"""GPU parity of seg_segment_noalloc, the entry point that allocates nothing
(its scratch is a fixed device array), against seg_segment through the C ABI
and against the float32 oracle: labels and distances bit for bit, on two
calls in a row with the second one smaller, in the dense and plain modes,
with statistics and with validation."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_parity, to_gpu

pytestmark = pytest.mark.gpu


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


def _both(seg, fib, at, mode, **kw):
    """(noalloc labels, dists), (seg_segment labels, dists) as numpy arrays."""
    import torch

    f, c, b, t = to_gpu(fib, at.centroids, at.bundle_id, at.thresholds)
    n = fib.shape[0]
    # outputs filled with garbage first: the call must write every entry
    out = (torch.full((n,), 12345, dtype=torch.int32, device=f.device),
           torch.full((n,), -7.0, dtype=torch.float32, device=f.device))
    seg.segment_noalloc(f, c, b, t, out=out, mode=mode, **kw)
    ref = seg.segment(f, c, b, t, mode=mode, **kw)
    torch.cuda.synchronize()
    return ((out[0].cpu().numpy(), out[1].cpu().numpy()),
            (ref[0].cpu().numpy(), ref[1].cpu().numpy()))


@pytest.mark.parametrize("mode", ["plain", "dense"])
def test_noalloc_two_calls_second_smaller(seg, mode):
    # first call: a larger subject and atlas; second: smaller both ways, so
    # stale centroid records past the second atlas stay in the array
    cases = [(synth.small_case(6001, 30, 41, seed=71), 6001),
             (synth.small_case(1303, 7, 13, seed=72), 1303)]
    for (fib, at), n in cases:
        log(f"noalloc mode={mode} n={n} m={at.n_centroids}")
        (lab, dist), (rl, rd) = _both(seg, fib, at, mode)
        assert np.array_equal(lab, rl) and np.array_equal(dist, rd), f"{mode}: differs from seg_segment"
        assert_parity(lab, dist, fib, at.centroids, at.bundle_id, at.thresholds,
                      ctx=f"noalloc {mode} n={n}", check_f64=False)


def test_noalloc_stats_and_validation(seg):
    import torch

    fib, at = synth.small_case(2500, 12, 25, seed=73)
    log("noalloc stats + validate")
    (lab, dist), (rl, rd) = _both(seg, fib, at, "plain", stats=True, validate=True)
    assert np.array_equal(lab, rl) and np.array_equal(dist, rd)
    f, c, b, t = to_gpu(fib, at.centroids, at.bundle_id, at.thresholds)
    out = (torch.empty(len(fib), dtype=torch.int32, device=f.device),
           torch.empty(len(fib), dtype=torch.float32, device=f.device))
    seg.segment_noalloc(f, c, b, t, out=out, mode="plain", stats=True)
    s1 = seg.query_stats()
    seg.segment(f, c, b, t, mode="plain", stats=True)
    s2 = seg.query_stats()
    assert s1 == s2
    assert s1["accepted"] == len(oracle.accepted_pairs_f32(fib, at.centroids, at.bundle_id,
                                                           at.thresholds))
    # validation reports a bad bundle id from the fixed array's flag word
    bad = at.bundle_id.copy()
    bad[3] = at.n_bundles
    f, c, b, t = to_gpu(fib, at.centroids, bad, at.thresholds)
    with pytest.raises(seg.SegError) as e:
        seg.segment_noalloc(f, c, b, t, out=out, mode="plain", validate=True)
    assert e.value.code == -2
    torch.cuda.synchronize()


def test_noalloc_largest_atlas_and_empty(seg):
    import torch

    M = seg.NOALLOC_MAX_CENTROIDS
    fib, at = synth.small_case(700, M // 128, 128, seed=74)
    assert at.n_centroids == M
    log(f"noalloc largest atlas m={M}")
    (lab, dist), (rl, rd) = _both(seg, fib, at, "plain")
    assert np.array_equal(lab, rl) and np.array_equal(dist, rd)
    assert_parity(lab, dist, fib, at.centroids, at.bundle_id, at.thresholds, ctx="noalloc max M",
                  check_f64=False)
    f, c, b, t = to_gpu(fib, at.centroids, at.bundle_id, at.thresholds)
    out = (torch.zeros(len(fib), dtype=torch.int32, device=f.device),
           torch.zeros(len(fib), dtype=torch.float32, device=f.device))
    seg.segment_noalloc(f, c[:0], b[:0], t, out=out, mode="dense")
    torch.cuda.synchronize()
    assert (out[0].cpu().numpy() == -1).all() and np.isinf(out[1].cpu().numpy()).all()
    with pytest.raises(seg.SegError) as e:
        seg.segment_noalloc(f, torch.cat([c, c[:1]]), torch.cat([b, b[:1]]), t, out=out)
    assert e.value.code == -6
