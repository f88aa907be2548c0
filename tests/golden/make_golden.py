"""Write the small seeded golden cases: inputs from ``synth``, outputs from ``oracle``.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_seeded_case.json")
OUT_RS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_resample_case.json")


def main():
    fib, at = synth.small_case(70, 6, 4, seed=20191224, thr_lo=6.0, thr_hi=10.0, sigma=2.0,
                               matched=0.6)
    lab, dist, best = oracle.segment_f32(fib, at.centroids, at.bundle_id, at.thresholds,
                                         mode=oracle.BRUTE)
    l64, d64, b64 = oracle.segment_f64(fib, at.centroids, at.bundle_id, at.thresholds)
    doc = {
        "about": "70 fibers x 24 centroids (6 bundles x 4), seeded synthetic; expected "
                 "outputs written by the CPU oracle (float32 decision, float64 distances). "
                 "Definition: Eq. 1-2, threshold rule of section 2.3, closest bundle of "
                 "section 2.4 / Algorithm 1.",
        "fibers": [float(x) for x in fib.ravel()],
        "centroids": [float(x) for x in at.centroids.ravel()],
        "bundle_id": [int(x) for x in at.bundle_id],
        "thresholds": [float(x) for x in at.thresholds],
        "labels_f32": [int(x) for x in lab],
        "dists_f32": [float(x) for x in dist],
        "best_f32": [int(x) for x in best],
        "labels_f64": [int(x) for x in l64],
        "dists_f64": [float(x) for x in d64],
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh)
    print(OUT, int((lab >= 0).sum()), "labelled")

    # raw streamlines around 8 of those fibers (1 mm steps), plus a single
    # point and a two-point streamline
    rng = np.random.default_rng(20191225)
    pts, off = synth.raw_streamlines(fib[:8], rng, step=1.0, jitter=0.02, dup=0.3)
    pts = np.concatenate([pts, fib[12, :1], fib[13, [0, 20]]])
    off = np.concatenate([off, [off[-1] + 1, off[-1] + 3]])
    rs = oracle.resample_f32(pts, off)
    doc = {
        "about": "10 raw streamlines (8 densified fibers of the seeded case with 1 mm "
                 "steps and repeated points, one single point, one two-point line); "
                 "expected 21-point resampling written by the CPU oracle (float32, points "
                 "equidistant in arc length, section 2.3).",
        "points": [float(x) for x in pts.ravel()],
        "offsets": [int(x) for x in off],
        "resampled": [float(x) for x in rs.ravel()],
    }
    with open(OUT_RS, "w") as fh:
        json.dump(doc, fh)
    print(OUT_RS, len(off) - 1, "streamlines,", pts.shape[0], "points")


if __name__ == "__main__":
    main()
