"""The seeded input generator: reproducible and shaped like the workloads."""
import numpy as np

import synth
from synth import fibers as F


def test_reproducible_and_chunk_addressable():
    fib1, at1 = synth.small_case(3000, 6, 5, seed=77)
    fib2, at2 = synth.small_case(3000, 6, 5, seed=77)
    assert np.array_equal(fib1, fib2) and np.array_equal(at1.centroids, at2.centroids)
    subj = synth.SubjectSpec(F.CHUNK + 500, 2.0, (0.3,))
    whole = synth.make_fibers([at1], subj, 5)
    part = synth.make_fibers([at1], subj, 5, start=F.CHUNK - 100, count=300)
    assert np.array_equal(part, whole[F.CHUNK - 100:F.CHUNK + 200])


def test_centroid_shapes():
    spec = synth.AtlasSpec(10, 30, 20.0, 80.0, 5.0, 8.0)
    at = synth.make_atlas(spec, 3)
    c = at.centroids.astype(np.float64)
    assert at.centroids.dtype == np.float32 and c.shape == (300, 21, 3)
    assert (c >= -1e-4).all() and (c <= F.BOX + 1e-4).all()
    chord = np.linalg.norm(np.diff(c, axis=1), axis=2)
    assert (chord.max(1) <= 1.25 * chord.min(1) * (1 + 1e-5)).all()
    length = chord.sum(1)
    assert length.min() > 20.0 * 0.95 and length.max() < 80.0 * 1.0001
    assert np.array_equal(at.bundle_id, np.arange(300) // 30)
    assert ((at.thresholds >= 5.0) & (at.thresholds <= 8.0)).all()


def test_config_shapes():
    for name, (m, b) in {"small-20k-x-800": (800, 40), "exact-1M-x-3600": (3600, 36),
                         "paper-4145k-x-10k": (10000, 100),
                         "large-10M-x-20k": (20000, 200)}.items():
        spec = synth.WORKLOADS[name]["atlases"][0]
        assert spec.n_centroids == m and spec.n_bundles == b
    assert synth.workload_subjects("paper-4145k-x-10k")[0].n_fibers == 4_145_000
    s5 = synth.workload_subjects("batch-16-subjects-x-2-atlases")
    assert len(s5) == 16 and all(300_000 <= s.n_fibers <= 4_100_000 for s in s5)
    assert [a.n_centroids for a in synth.WORKLOADS["batch-16-subjects-x-2-atlases"]["atlases"]] == [3600, 10000]


def test_matched_fraction():
    spec = synth.AtlasSpec(4, 5, 20.0, 80.0, 5.0, 8.0)
    at = synth.make_atlas(spec, 9)
    subj = synth.SubjectSpec(2000, 0.0, (0.5,))
    fib = synth.make_fibers([at], subj, 9)
    # with sigma = 0 a matched fiber is an exact copy of a centroid, maybe reversed
    cen = at.centroids.reshape(20, -1)
    fwd = (fib.reshape(2000, 1, -1) == cen[None]).all(2).any(1)
    rev = (fib[:, ::-1].reshape(2000, 1, -1) == cen[None]).all(2).any(1)
    assert (fwd | rev).sum() == 1000
    assert 400 < rev.sum() < 600


def test_centroids_equal_chords_by_construction():
    at = synth.make_atlas(synth.AtlasSpec(5, 40, 20.0, 80.0, 5.0, 8.0), 4)
    c = at.centroids.astype(np.float64)
    chord = np.linalg.norm(np.diff(c, axis=1), axis=2)
    assert (chord.max(1) / chord.min(1) < 1 + 1e-4).all()
    u = np.diff(c, axis=1) / chord[..., None]
    turn = np.degrees(np.arccos(np.clip((u[:, 1:] * u[:, :-1]).sum(2), -1, 1)))
    assert turn.max() <= 40.0 + 1e-2


def test_raw_streamlines_shape():
    fib, _ = synth.small_case(300, 3, 5, seed=8, len_lo=20.0, len_hi=80.0)
    rng = np.random.default_rng(3)
    pts, off = synth.raw_streamlines(fib, rng, step=0.2, jitter=0.0, dup=0.5)
    assert pts.dtype == np.float32 and off.dtype == np.int64 and off[0] == 0
    assert off[-1] == pts.shape[0] and len(off) == 301
    for i in range(0, 300, 37):
        p = pts[off[i]:off[i + 1]].astype(np.float64)
        assert np.array_equal(p[0], fib[i, 0]) and np.array_equal(p[-1], fib[i, 20])
        step = np.linalg.norm(np.diff(p, axis=0), axis=1)
        assert np.median(step) < 0.3 and step.max() < 0.5
    # about half the streamlines repeat one point (a zero-length step)
    zero = [(np.linalg.norm(np.diff(pts[off[i]:off[i + 1]], axis=0), axis=1) == 0).any()
            for i in range(300)]
    assert 100 < sum(zero) < 200
    again, off2 = synth.raw_streamlines(fib, np.random.default_rng(3), step=0.2, jitter=0.0,
                                        dup=0.5)
    assert np.array_equal(again, pts) and np.array_equal(off2, off)


def test_no_fork_after_gpu_init(monkeypatch):
    """Once torch has initialised the GPU, the generator draws every chunk in
    this process (a forked worker would inherit the device state); the output
    is the same as with the pool."""
    import multiprocessing

    import torch

    at = synth.make_atlas(synth.AtlasSpec(4, 5, 20.0, 80.0, 5.0, 8.0), 3)
    subj = synth.SubjectSpec(3 * F.CHUNK // 2, 2.0, (0.3,))
    want = synth.make_fibers([at], subj, 8, workers=1)
    assert not synth.gpu_in_use()

    def no_pool(*a, **k):
        raise AssertionError("a worker pool was started after GPU initialisation")

    monkeypatch.setattr(torch.cuda, "is_initialized", lambda: True)
    monkeypatch.setattr(multiprocessing.context.ForkContext, "Pool", no_pool, raising=False)
    monkeypatch.setattr(multiprocessing.context.BaseContext, "Pool", no_pool)
    assert synth.gpu_in_use()
    got = synth.make_fibers([at], subj, 8, workers=4)
    assert np.array_equal(got, want)
