"""The oracle reproduces the stored seeded cases (guards the oracle against drift)."""
import json
import os

import numpy as np

import oracle

PATH = os.path.join(os.path.dirname(__file__), "golden", "small_seeded_case.json")


def load():
    with open(PATH) as fh:
        d = json.load(fh)
    fib = np.array(d["fibers"], np.float32).reshape(-1, 21, 3)
    cen = np.array(d["centroids"], np.float32).reshape(-1, 21, 3)
    return d, fib, cen, np.array(d["bundle_id"], np.int32), np.array(d["thresholds"], np.float32)


def test_golden_oracle(O):
    d, fib, cen, bid, thr = load()
    for mode in (oracle.BRUTE, oracle.CUT):
        lab, dist, best = O.segment_f32(fib, cen, bid, thr, mode=mode)
        assert lab.tolist() == d["labels_f32"] and best.tolist() == d["best_f32"]
        assert np.array_equal(dist, np.array(d["dists_f32"], np.float32))
    l64, d64, _ = O.segment_f64(fib, cen, bid, thr)
    assert l64.tolist() == d["labels_f64"]
    assert np.array_equal(d64, np.array(d["dists_f64"]))
    assert 20 <= (lab >= 0).sum() < len(lab)


PATH_RS = os.path.join(os.path.dirname(__file__), "golden", "small_resample_case.json")


def load_resample():
    with open(PATH_RS) as fh:
        d = json.load(fh)
    return (np.array(d["points"], np.float32).reshape(-1, 3), np.array(d["offsets"], np.int64),
            np.array(d["resampled"], np.float32).reshape(-1, 21, 3))


def test_golden_resample(O):
    pts, off, want = load_resample()
    assert np.array_equal(O.resample_f32(pts, off), want)
    assert len(off) == 11 and np.diff(off).min() == 1
