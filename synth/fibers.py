"""Seeded generator of atlases and subject fiber sets.

Shapes follow the paper's workloads: every fiber and centroid is a polyline of
21 points with 3 float32 coordinates in millimetres (paper, section 2.2 and
section 2.3: fibers are resampled to 21 equidistant points).  The real data
(tractography of the ARCHI database and the LNAO-SWM79 / 62-bundle atlases,
section 2.1-2.2) is not available, so these curves stand in for it.

Recipe (one reading of the workload text, fixed here once):

* A centroid is a cubic Bezier curve.  Its target length L is uniform in
  [len_lo, len_hi].  The control points P1..P3 are P0 plus offsets uniform in a
  cube of side 0.6 L.  The curve is sampled at ``_SAMPLES`` parameter values
  and scaled about P0 so that the sampled polyline has arc length L.  It is
  then resampled to 21 points equidistant in arc length; a shape whose
  resampled chord spacing varies by more than 25% (a cusp) is redrawn.  P0 is
  drawn uniformly
  among the positions that keep the whole curve inside the 180 x 220 x 180 mm
  box; a shape that cannot fit is redrawn.
* Centroids are stored bundle-major: centroid c belongs to bundle
  c // per_bundle.
* Bundle thresholds are uniform in [thr_lo, thr_hi] (mm).
* A matched fiber copies a uniformly drawn centroid and adds a smooth
  displacement: four Gaussian knots N(0, sigma^2 I3) placed at t = 0, 1/3,
  2/3, 1 and linearly interpolated to the 21 points (point i sits at
  t = i / 20).  Its point order is reversed with probability 1/2.
* An unmatched fiber is an independent curve from the centroid generator.
* Fibers are generated in chunks of ``CHUNK`` with an independent random
  stream per chunk, so any fiber range can be generated without the rest.

Nothing here evaluates a fiber-to-centroid distance.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

N_POINTS = 21
BOX = np.array([180.0, 220.0, 180.0])
CHUNK = 65536
_SAMPLES = 48


@dataclass(frozen=True)
class AtlasSpec:
    n_bundles: int
    per_bundle: int
    len_lo: float
    len_hi: float
    thr_lo: float
    thr_hi: float

    @property
    def n_centroids(self) -> int:
        return self.n_bundles * self.per_bundle


@dataclass(frozen=True)
class SubjectSpec:
    n_fibers: int
    sigma: float
    # fraction of fibers copied from each atlas (one entry per atlas)
    matched: Sequence[float]


@dataclass
class Atlas:
    centroids: np.ndarray  # float32 [M, 21, 3]
    bundle_id: np.ndarray  # int32 [M]
    thresholds: np.ndarray  # float32 [B]
    spec: Optional[AtlasSpec] = None

    @property
    def n_centroids(self) -> int:
        return int(self.centroids.shape[0])

    @property
    def n_bundles(self) -> int:
        return int(self.thresholds.shape[0])


_LONG = dict(len_lo=20.0, len_hi=200.0)
_SHORT = dict(len_lo=20.0, len_hi=80.0)

# The five workloads, named by what they are: a small case the oracle runs in
# full, a plain exact-path case, the paper-scale subject (4,145,000 fibers,
# section 3), a large probabilistic-like subject and a batch of uneven subjects
# against two atlases.  Each carries its own seed.
WORKLOADS = {
    "small-20k-x-800": dict(
        seed=12494,
        atlases=[AtlasSpec(40, 20, thr_lo=6.0, thr_hi=10.0, **_LONG)],
        subjects=[SubjectSpec(20_000, 2.0, (0.6,))],
    ),
    "exact-1M-x-3600": dict(
        seed=13494,
        atlases=[AtlasSpec(36, 100, thr_lo=6.0, thr_hi=12.0, **_LONG)],
        subjects=[SubjectSpec(1_000_000, 3.0, (0.5,))],
    ),
    "paper-4145k-x-10k": dict(
        seed=14494,
        atlases=[AtlasSpec(100, 100, thr_lo=5.0, thr_hi=8.0, **_SHORT)],
        subjects=[SubjectSpec(4_145_000, 2.0, (0.3,))],
    ),
    "large-10M-x-20k": dict(
        seed=15494,
        atlases=[AtlasSpec(200, 100, thr_lo=5.0, thr_hi=8.0, **_SHORT)],
        subjects=[SubjectSpec(10_000_000, 2.0, (0.3,))],
    ),
    "batch-16-subjects-x-2-atlases": dict(
        seed=16494,
        atlases=[
            AtlasSpec(36, 100, len_lo=80.0, len_hi=200.0, thr_lo=6.0, thr_hi=12.0),
            AtlasSpec(100, 100, thr_lo=5.0, thr_hi=8.0, **_SHORT),
        ],
        subjects=None,  # drawn: 16 subjects, sizes uniform in [0.3M, 4.1M]
        n_subjects=16,
        size_lo=300_000,
        size_hi=4_100_000,
        sigma=2.0,
        matched=(0.15, 0.15),
    ),
}


def workload_seed(name: str) -> int:
    return WORKLOADS[name]["seed"]


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _bernstein(samples: int) -> np.ndarray:
    t = np.linspace(0.0, 1.0, samples)
    return np.stack([(1 - t) ** 3, 3 * t * (1 - t) ** 2, 3 * t**2 * (1 - t), t**3], 0)


def _resample_equidistant(poly: np.ndarray, n_out: int) -> np.ndarray:
    """Points equidistant in arc length along each polyline (float64)."""
    n, s, _ = poly.shape
    seg = np.sqrt((np.diff(poly, axis=1) ** 2).sum(2))  # [n, s-1]
    cum = np.concatenate([np.zeros((n, 1)), np.cumsum(seg, 1)], 1)  # [n, s]
    total = cum[:, -1]
    tgt = np.linspace(0.0, 1.0, n_out)[None, :] * total[:, None]  # [n, n_out]
    stride = float(total.max()) * 2.0 + 1.0
    off = np.arange(n, dtype=np.float64)[:, None] * stride
    j = np.searchsorted((cum + off).ravel(), (tgt + off).ravel(), side="right") - 1
    j = j.reshape(n, n_out) - np.arange(n)[:, None] * s
    j = np.clip(j, 0, s - 2)
    rows = np.arange(n)[:, None]
    c0 = cum[rows, j]
    seglen = seg[rows, j]
    w = np.where(seglen > 0, (tgt - c0) / np.where(seglen > 0, seglen, 1.0), 0.0)
    w = np.clip(w, 0.0, 1.0)[..., None]
    out = poly[rows, j] * (1 - w) + poly[rows, j + 1] * w
    out[:, 0] = poly[:, 0]
    out[:, -1] = poly[:, -1]
    return out


def bezier_curves(rng: np.random.Generator, n: int, len_lo: float, len_hi: float,
                  box: np.ndarray = BOX, samples: int = _SAMPLES) -> np.ndarray:
    """``n`` random cubic Bezier curves resampled to 21 points, float64 [n,21,3]."""
    out = np.empty((n, N_POINTS, 3))
    todo = np.arange(n)
    bern = _bernstein(samples)  # [4, S]
    while todo.size:
        k = todo.size
        length = rng.uniform(len_lo, len_hi, k)
        side = 0.6 * length
        ctrl = np.zeros((k, 4, 3))
        ctrl[:, 1:, :] = rng.uniform(-0.5, 0.5, (k, 3, 3)) * side[:, None, None]
        poly = (ctrl.transpose(0, 2, 1).reshape(-1, 4) @ bern).reshape(k, 3, samples)
        poly = poly.transpose(0, 2, 1)  # [k, S, 3], P0 at the origin
        arc = np.sqrt((np.diff(poly, axis=1) ** 2).sum(2)).sum(1)
        ok = arc > 1e-6 * length
        scale = np.where(ok, length / np.where(ok, arc, 1.0), 0.0)
        poly *= scale[:, None, None]
        lo = poly.min(1)
        hi = poly.max(1)
        fits = ok & np.all(hi - lo <= box[None, :], axis=1)
        pts = _resample_equidistant(poly[fits], N_POINTS)
        # streamlines are smooth: a shape with a cusp (chord spacing of the
        # resampled points varying by more than 25%) is redrawn
        chord = np.sqrt((np.diff(pts, axis=1) ** 2).sum(2))
        smooth = chord.max(1) <= 1.25 * chord.min(1)
        idx = np.nonzero(fits)[0]
        fits[idx[~smooth]] = False
        pts = pts[smooth]
        p0 = lo[fits] * -1.0 + rng.uniform(0.0, 1.0, (int(fits.sum()), 3)) * (
            box[None, :] - (hi[fits] - lo[fits]))
        out[todo[fits]] = pts + p0[:, None, :]
        todo = todo[~fits]
    return out


def make_atlas(spec: AtlasSpec, seed: int) -> Atlas:
    rng = _rng(seed, 0)
    cen = bezier_curves(rng, spec.n_centroids, spec.len_lo, spec.len_hi)
    bid = (np.arange(spec.n_centroids) // spec.per_bundle).astype(np.int32)
    thr = rng.uniform(spec.thr_lo, spec.thr_hi, spec.n_bundles).astype(np.float32)
    return Atlas(cen.astype(np.float32), bid, thr, spec)


def _fiber_chunk(atlases: Sequence[Atlas], matched: Sequence[float], sigma: float,
                 n: int, rng: np.random.Generator) -> np.ndarray:
    counts = [int(round(f * n)) for f in matched]
    n_match = sum(counts)
    if n_match > n:
        raise ValueError("matched fractions exceed 1")
    parts = []
    for atlas, cnt in zip(atlases, counts):
        if cnt == 0:
            continue
        pick = rng.integers(0, atlas.n_centroids, cnt)
        base = atlas.centroids[pick].astype(np.float64)
        knots = rng.normal(0.0, sigma, (cnt, 4, 3))
        t = np.arange(N_POINTS) / (N_POINTS - 1)
        seg = np.minimum((t * 3).astype(int), 2)
        w = (t * 3 - seg)[None, :, None]
        disp = knots[:, seg, :] * (1 - w) + knots[:, seg + 1, :] * w
        f = base + disp
        flip = rng.random(cnt) < 0.5
        f[flip] = f[flip, ::-1, :]
        parts.append(f)
    n_free = n - n_match
    if n_free:
        # each unmatched fiber takes the length range of a uniformly chosen atlas
        which = rng.integers(0, len(atlases), n_free)
        free = np.empty((n_free, N_POINTS, 3))
        for a, atlas in enumerate(atlases):
            sel = np.nonzero(which == a)[0]
            if sel.size:
                spec = atlas.spec
                lo, hi = (spec.len_lo, spec.len_hi) if spec else (20.0, 200.0)
                free[sel] = bezier_curves(rng, sel.size, lo, hi)
        parts.append(free)
    allf = np.concatenate(parts, 0) if parts else np.empty((0, N_POINTS, 3))
    allf = allf[rng.permutation(n)]
    return allf.astype(np.float32)


def _chunk_job(args):
    atlases, subject, seed, subject_idx, c = args
    lo = c * CHUNK
    n = min(CHUNK, subject.n_fibers - lo)
    return _fiber_chunk(atlases, subject.matched, subject.sigma, n,
                        _rng(seed, 1, subject_idx, c))


def make_fibers(atlases: Sequence[Atlas], subject: SubjectSpec, seed: int,
                subject_idx: int = 0, start: int = 0, count: Optional[int] = None,
                workers: int = 1) -> np.ndarray:
    """Fibers [start, start+count) of a subject, float32 [count, 21, 3].

    ``workers`` > 1 draws the chunks in a pool of forked processes (same
    output); call it before the process has touched the GPU.
    """
    if count is None:
        count = subject.n_fibers - start
    if start < 0 or count < 0 or start + count > subject.n_fibers:
        raise ValueError("fiber range outside the subject")
    out = np.empty((count, N_POINTS, 3), np.float32)
    c0, c1 = start // CHUNK, (start + count + CHUNK - 1) // CHUNK
    jobs = [(atlases, subject, seed, subject_idx, c) for c in range(c0, c1)]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp

        # close + join (not terminate): the workers end on their own, with no
        # signal, which matters when a profiler has hooked the process
        pool = mp.get_context("fork").Pool(min(workers, len(jobs)))
        try:
            chunks = pool.map(_chunk_job, jobs, chunksize=1)
        finally:
            pool.close()
            pool.join()
    else:
        chunks = map(_chunk_job, jobs)
    for c, chunk in zip(range(c0, c1), chunks):
        lo = c * CHUNK
        n = chunk.shape[0]
        a = max(start, lo)
        b = min(start + count, lo + n)
        out[a - start:b - start] = chunk[a - lo:b - lo]
    return out


def workload_atlases(name: str) -> List[Atlas]:
    seed = workload_seed(name)
    return [make_atlas(spec, seed * 10 + i) for i, spec in enumerate(WORKLOADS[name]["atlases"])]


def workload_subjects(name: str) -> List[SubjectSpec]:
    c = WORKLOADS[name]
    if c["subjects"] is not None:
        return list(c["subjects"])
    rng = _rng(workload_seed(name), 2)
    sizes = rng.integers(c["size_lo"], c["size_hi"] + 1, c["n_subjects"])
    return [SubjectSpec(int(s), c["sigma"], tuple(c["matched"])) for s in sizes]


def small_case(n_fibers: int, n_bundles: int, per_bundle: int, seed: int,
               len_lo: float = 20.0, len_hi: float = 200.0, thr_lo: float = 6.0,
               thr_hi: float = 10.0, sigma: float = 2.0, matched: float = 0.6):
    """A small atlas + subject with the workload's structure, for tests."""
    spec = AtlasSpec(n_bundles, per_bundle, len_lo, len_hi, thr_lo, thr_hi)
    atlas = make_atlas(spec, seed)
    subj = SubjectSpec(n_fibers, sigma, (matched,))
    fibers = make_fibers([atlas], subj, seed)
    return fibers, atlas
