"""GPU parity of resampling raw streamlines to 21 points equidistant in arc
length (the step before the comparison, section 2.3) through the C ABI:
every output coordinate equals the float32 oracle's bit for bit, and
resample-then-segment equals the oracle's resample-then-segment."""
import sys

import numpy as np
import pytest

import inputs
import oracle
import pins
import synth
from gpu_common import to_gpu

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


def _gpu_resample(seg, pts, off, validate=False):
    import torch

    d = torch.device("cuda:0")
    out = seg.resample(torch.from_numpy(np.ascontiguousarray(pts, np.float32)).to(d),
                       torch.from_numpy(np.ascontiguousarray(off, np.int64)).to(d),
                       validate=validate)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _same(a, b, ctx):
    same = (a == b) | (np.isnan(a) & np.isnan(b))
    bad = np.nonzero(~same.all(axis=(1, 2)))[0]
    assert bad.size == 0, f"{ctx}: {bad.size} streamlines differ, first {bad[:5]}"


def _corner_lines():
    """The four hand-worked corners of the fixed-point reading: a rounding
    tie, saturated lengths, a sum a float32 running total would lose, a
    floored target (expected points in test_resample_edges)."""
    u = 2.0**-24
    c = np.zeros((4098, 3))
    c[1:, 0] = 4096.0
    c[2:, 1] = np.arange(1, 4097) * 2.0**-12
    return [np.array([[0.0, 0, 0], [4096.0, 0, 0], [2.0**-13, 0, 0], [8192.0, 0, 0]]),
            np.array([[0.0, 0, 0], [20000.0, 0, 0], [60000.0, 0, 0]]), c,
            np.array([[0.0, 0, 0], [10 * u, 0, 0], [19 * u, 0, 0]])]


def _edge_lines():
    """Single points, two points, zero-length lines, the fixed-point corners,
    repeated points, a 5,000-point line (longer than a wave's LDS slice)."""
    rng = np.random.default_rng(5)
    lines = [np.array([[5.0, 6.0, 7.0]]), np.array([[1.0, 2.0, 3.0], [4.0, 8.0, 12.0]]),
             np.repeat(np.array([[9.0, 9.0, 9.0]]), 50, 0)] + _corner_lines()
    c = pins._raw_curve(rng, 300, 60.0, (50.0, 60.0, 70.0))
    lines.append(np.repeat(c, rng.integers(1, 4, len(c)), axis=0))
    lines.append(pins._raw_curve(rng, 5000, 180.0, (10.0, 20.0, 10.0)))
    lines.append(pins._raw_curve(rng, 3, 0.001, (90.0, 90.0, 90.0)))
    return lines


def test_golden_resample(seg):
    from test_golden import load_resample

    pts, off, want = load_resample()
    log("resample golden")
    _same(_gpu_resample(seg, pts, off), want, "golden")


@pytest.mark.parametrize("n,step,seed", [(1, 0.2, 1), (255, 0.2, 2), (257, 0.5, 3),
                                         (3001, 0.2, 4), (20000, 0.2, 5)])
def test_resample_ragged(seg, n, step, seed):
    fib, _ = synth.small_case(n, 7, 9, seed=seed, len_lo=20.0, len_hi=200.0)
    pts, off = synth.raw_streamlines(fib, np.random.default_rng(seed), step=step, dup=0.2)
    log(f"resample ragged n={n} points={pts.shape[0]}")
    got = _gpu_resample(seg, pts, off)
    _same(got, oracle.resample_f32(pts, off), f"ragged n={n}")
    assert np.isfinite(got).all()


def test_resample_edges(seg):
    lines = _edge_lines()
    pts, off = pins._csr(lines)
    log(f"resample edges {len(lines)} lines")
    got = _gpu_resample(seg, pts, off)
    _same(got, oracle.resample_f32(pts, off), "edges")
    f32 = np.float32
    assert np.array_equal(got[3][10], np.zeros(3, f32))
    assert np.array_equal(got[4][10], np.array([20000.0, 0, 0], f32))
    assert np.array_equal(got[4][5], np.array([10000.0, 0, 0], f32))
    assert np.array_equal(got[5][10], np.array([2048.5, 0, 0], f32))
    assert np.array_equal(got[6][10], np.array([9 * 2.0**-24, 0, 0], f32))


def test_resample_interleaved_edges(seg):
    """Edge lines scattered between ordinary ones, so one wave holds lanes of
    very different lengths."""
    fib, _ = synth.small_case(500, 4, 5, seed=9)
    pts0, off0 = synth.raw_streamlines(fib, np.random.default_rng(9))
    lines = [pts0[off0[i]:off0[i + 1]] for i in range(500)]
    edges = _edge_lines()
    for i, e in enumerate(edges):
        lines.insert(37 * i + 5, e)
    pts, off = pins._csr(lines)
    log("resample interleaved edges")
    _same(_gpu_resample(seg, pts, off), oracle.resample_f32(pts, off), "interleaved")


def test_resample_single_points(seg):
    """3,000 streamlines of one point each, and a set mixing one- and
    two-point streamlines."""
    rng = np.random.default_rng(15)
    pts = rng.uniform(0, 100, (3000, 3)).astype(np.float32)
    off = np.arange(3001, dtype=np.int64)
    log("resample single points")
    got = _gpu_resample(seg, pts, off)
    assert np.array_equal(got, np.repeat(pts[:, None, :], 21, axis=1))
    k = rng.integers(1, 3, 2000)
    off2 = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
    pts2 = rng.uniform(0, 100, (int(off2[-1]), 3)).astype(np.float32)
    _same(_gpu_resample(seg, pts2, off2), oracle.resample_f32(pts2, off2), "one and two points")


def test_segment_streamlines_validation(seg):
    import torch

    fib, at = synth.small_case(300, 3, 4, seed=16)
    pts, off = synth.raw_streamlines(fib, np.random.default_rng(16))
    d = torch.device("cuda:0")
    _, c, b, t = to_gpu(fib[:1], at.centroids, at.bundle_id, at.thresholds)
    atlas = seg.Atlas(c, b, t)
    bad = off.copy()
    bad[10] = bad[9]
    log("segment streamlines validation")
    with pytest.raises(seg.SegError) as e:
        atlas.segment_streamlines(torch.from_numpy(pts).to(d), torch.from_numpy(bad).to(d),
                                  mode="fp16", validate=True)
    assert e.value.code == -8
    nanpts = pts.copy()
    nanpts[5, 1] = np.nan
    with pytest.raises(seg.SegError) as e:
        atlas.segment_streamlines(torch.from_numpy(nanpts).to(d), torch.from_numpy(off).to(d),
                                  mode="fp16", validate=True)
    assert e.value.code == -3


def test_resample_long_lines(seg):
    """Streamlines of 500 to 3,000 points: those of more than 640 segments
    take the one-lane path, the others the wave path; and segment counts
    around a chunk of 64, a round of four chunks and the slice of 640."""
    rng = np.random.default_rng(13)
    sizes = [int(x) for x in rng.integers(500, 3000, 300)]
    sizes += [2, 3, 63, 64, 65, 66, 127, 128, 129, 256, 257, 258, 512, 513, 639, 640, 641, 642,
              643, 1025, 2049]
    lines = [pins._raw_curve(rng, k, rng.uniform(100, 250), rng.uniform([20, 20, 20], [60, 60, 60]))
             for k in sizes]
    pts, off = pins._csr(lines)
    log(f"resample long lines: {pts.shape[0]} points")
    _same(_gpu_resample(seg, pts, off), oracle.resample_f32(pts, off), "long lines")


def test_resample_overlap_after_bad(seg):
    """Decreasing offsets: streamline 3 is invalid and streamline 4 re-reads
    points of streamline 2; each valid one still equals the oracle on its own
    points."""
    fib, _ = synth.small_case(70, 2, 3, seed=14)
    pts, off = synth.raw_streamlines(fib, np.random.default_rng(14))
    bad = off.copy()
    bad[4] = off[2] + 3  # streamline 3 = [off[3], off[2] + 3): decreasing
    log("resample overlap after a bad streamline")
    got = _gpu_resample(seg, pts, bad)
    assert np.isnan(got[3]).all()
    for i in range(70):
        if i == 3:
            continue
        want = oracle.resample_f32(pts[bad[i]:bad[i + 1]], np.array([0, bad[i + 1] - bad[i]]))
        assert np.array_equal(got[i], want[0]), i


def test_resample_bad_offsets(seg):
    import torch

    fib, _ = synth.small_case(40, 2, 3, seed=10)
    pts, off = synth.raw_streamlines(fib, np.random.default_rng(10))
    want = oracle.resample_f32(pts, off)
    bad = off.copy()
    bad[7] = bad[6]            # streamline 6 is empty
    bad[20] = pts.shape[0] + 5  # streamline 19 ends past the points, 20 starts there
    log("resample bad offsets")
    got = _gpu_resample(seg, pts, bad)
    for i in (6, 19, 20):
        assert np.isnan(got[i]).all(), i
    ok = [i for i in range(40) if i not in (6, 7, 19, 20)]  # 7 now spans 6 and 7
    assert np.array_equal(got[ok], want[ok])
    with pytest.raises(seg.SegError) as e:
        _gpu_resample(seg, pts, bad, validate=True)
    assert e.value.code == -8
    # more than 2^24 points in one streamline: NaN, and SEG_EOFFSETS on validation
    d = torch.device("cuda:0")
    gbig = torch.zeros((2**24 + 2, 3), dtype=torch.float32, device=d)
    for o2 in ([0, 2**24 + 1], [0, 1, 2**24 + 2]):
        got2 = seg.resample(gbig, torch.tensor(o2, dtype=torch.int64, device=d)).cpu().numpy()
        assert np.isnan(got2[-1]).all()
        if len(o2) == 3:
            assert np.array_equal(got2[0], np.zeros((21, 3), np.float32))
        with pytest.raises(seg.SegError) as e:
            seg.resample(gbig, torch.tensor(o2, dtype=torch.int64, device=d), validate=True)
        assert e.value.code == -8
    del gbig
    # valid offsets pass validation
    _same(_gpu_resample(seg, pts, off, validate=True), want, "validated")
    empty = seg.resample(torch.zeros((0, 3), dtype=torch.float32, device=d),
                         torch.zeros(1, dtype=torch.int64, device=d))
    assert empty.shape == (0, 21, 3)


@pytest.mark.parametrize("mode,metric", [("plain", 0), ("fp16", 0), ("bf16", 0), ("fp16", "tn"),
                                         ("dense", "dir")])
def test_segment_streamlines(seg, mode, metric):
    """Raw streamlines to labels in one call equals the oracle's resampling
    followed by the oracle's segmentation."""
    import torch

    fib, at = synth.small_case(6000, 12, 25, seed=11, len_lo=20.0, len_hi=120.0)
    pts, off = synth.raw_streamlines(fib, np.random.default_rng(11), dup=0.05)
    rs = oracle.resample_f32(pts, off)
    flags = {0: 0, "tn": oracle.TN, "dir": oracle.DIR}[metric]
    want = oracle.segment_ext_f32(rs, at.centroids, at.bundle_id, at.thresholds, flags)
    d = torch.device("cuda:0")
    _, c, b, t = to_gpu(fib[:1], at.centroids, at.bundle_id, at.thresholds)
    atlas = seg.Atlas(c, b, t)
    log(f"segment streamlines mode={mode} metric={metric}")
    lab, dist, fibers = atlas.segment_streamlines(torch.from_numpy(pts).to(d),
                                                  torch.from_numpy(off).to(d), mode=mode,
                                                  metric=metric, validate=True)
    torch.cuda.synchronize()
    assert np.array_equal(fibers.cpu().numpy(), rs)
    lab, dist = lab.cpu().numpy(), dist.cpu().numpy()
    assert np.array_equal(lab, want[0])
    assert np.array_equal(dist, want[1])
    assert (lab >= 0).mean() > 0.3


@pytest.mark.workloads("paper-4145k-x-10k")
def test_resample_full_size_sampled(seg):
    """Paper-scale subject as raw streamlines (4,145,000 streamlines, about 10^9
    points at 0.2 mm steps) in the benchmark's launch configuration; the
    oracle recomputes a fixed sample of streamlines."""
    import torch

    wl = "paper-4145k-x-10k"
    at = synth.workload_atlases(wl)[0]
    subj = synth.workload_subjects(wl)[0]
    fib = inputs.fibers(wl)
    d = torch.device("cuda:0")
    f = torch.from_numpy(fib).to(d)
    pts, off = synth.raw_streamlines_torch(f, synth.workload_seed(wl))
    del f
    log(f"resample full size: {pts.shape[0]} points")
    out = seg.resample(pts, off)
    torch.cuda.synchronize()
    n = fib.shape[0]
    rng = np.random.default_rng(12)
    idx = np.concatenate([np.sort(rng.choice(n, 2000, replace=False)), np.arange(n - 50, n)])
    off_h = off.cpu().numpy()
    lines = [pts[int(off_h[i]):int(off_h[i + 1])].cpu().numpy() for i in idx]
    sp, so = pins._csr(lines)
    want = oracle.resample_f32(sp, so)
    got = out[torch.from_numpy(idx).to(d)].cpu().numpy()
    _same(got, want, "full size sample")
    assert torch.isfinite(out).all().item()
