"""Seeded generator of atlases and subject fiber sets.

Shapes follow the paper's workloads: every fiber and centroid is a polyline of
21 points with 3 float32 coordinates in millimetres (paper, section 2.2 and
section 2.3: fibers are resampled to 21 equidistant points).  The real data
(tractography of the ARCHI database and the LNAO-SWM79 / 62-bundle atlases,
section 2.1-2.2) is not available, so these curves stand in for it.

Recipe (one reading of the workload text, fixed here once):

* A centroid follows the direction of a random cubic Bezier curve.  Its
  length L is uniform in [len_lo, len_hi].  The control points P1..P3 are P0
  plus offsets uniform in a cube of side 0.6 L.  Point i+1 is point i plus
  L / 20 times the unit tangent of the Bezier curve at parameter
  (i + 1/2) / 20, so the 21 points are equally spaced along the polyline by
  construction (no resampling).  A shape that turns by more than 40 degrees
  between two consecutive chords (near a cusp) is redrawn.  P0 is drawn
  uniformly among the positions that keep the whole curve inside the
  180 x 220 x 180 mm box; a shape that cannot fit is redrawn.
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
* A raw streamline (the tractography output before resampling) is a 21-point
  fiber densified by its parameter: m = max(1, round(|p1 - p0| / step)) points
  per chord, 20 m + 1 in all, placed by linear interpolation at parameter
  j / m, interior points moved by N(0, jitter^2 I3); with probability ``dup``
  one interior point is repeated (a zero-length step).  The step defaults to
  the paper's 0.2 mm tractography step.

Nothing here evaluates a fiber-to-centroid distance.
"""
from __future__ import annotations

import sys
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

N_POINTS = 21
BOX = np.array([180.0, 220.0, 180.0])
CHUNK = 65536
_MAX_TURN_DEG = 40.0


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
    # clustered density: (fiber fraction, bundle fraction): that fraction of
    # the fibers are copies of centroids of the first round(bundle fraction x
    # bundles) bundles of the first atlas; `matched` applies to the rest
    hot: Optional[Tuple[float, float]] = None


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
    # the paper-scale atlas and subject size with 80% of the fibers packed
    # around 5% of the bundles (dense regions, as near the cortex)
    "clustered-4145k-x-10k": dict(
        seed=17494,
        atlases=[AtlasSpec(100, 100, thr_lo=5.0, thr_hi=8.0, **_SHORT)],
        subjects=[SubjectSpec(4_145_000, 2.0, (0.3,), hot=(0.8, 0.05))],
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


def bezier_curves(rng: np.random.Generator, n: int, len_lo: float, len_hi: float,
                  box: np.ndarray = BOX) -> np.ndarray:
    """``n`` random smooth curves of 21 equally spaced points, float64 [n,21,3]."""
    out = np.empty((n, N_POINTS, 3))
    todo = np.arange(n)
    t = (np.arange(N_POINTS - 1) + 0.5) / (N_POINTS - 1)
    dbasis = np.stack([(1 - t) ** 2, 2 * t * (1 - t), t**2], 0)  # [3, 20]
    cos_max = np.cos(np.deg2rad(_MAX_TURN_DEG))
    while todo.size:
        k = todo.size
        length = rng.uniform(len_lo, len_hi, k)
        side = 0.6 * length
        ctrl = np.zeros((k, 4, 3))
        ctrl[:, 1:, :] = rng.uniform(-0.5, 0.5, (k, 3, 3)) * side[:, None, None]
        diff = ctrl[:, 1:, :] - ctrl[:, :-1, :]  # [k, 3, 3]
        tan = np.einsum("kjc,jt->ktc", diff, dbasis)  # [k, 20, 3], Bezier tangent / 3
        speed = np.sqrt((tan**2).sum(2))
        ok = speed.min(1) > 1e-6 * length
        u = tan / np.where(speed > 0, speed, 1.0)[..., None]
        turn = (u[:, 1:] * u[:, :-1]).sum(2).min(1)
        ok &= turn >= cos_max
        pts = np.zeros((k, N_POINTS, 3))
        pts[:, 1:] = np.cumsum(u * (length / (N_POINTS - 1))[:, None, None], 1)
        lo = pts.min(1)
        hi = pts.max(1)
        fits = ok & np.all(hi - lo <= box[None, :], axis=1)
        p0 = lo[fits] * -1.0 + rng.uniform(0.0, 1.0, (int(fits.sum()), 3)) * (
            box[None, :] - (hi[fits] - lo[fits]))
        out[todo[fits]] = pts[fits] + p0[:, None, :]
        todo = todo[~fits]
    return out


def raw_streamlines(fibers: np.ndarray, rng: np.random.Generator, step: float = 0.2,
                    jitter: float = 0.02, dup: float = 0.01):
    """Raw streamlines drawn around 21-point fibers (see the recipe above):
    (points float32 [P, 3], offsets int64 [n + 1])."""
    f = np.asarray(fibers, np.float64)
    n = f.shape[0]
    chord = np.sqrt(((f[:, 1] - f[:, 0]) ** 2).sum(1)) if n else np.zeros(0)
    m = np.maximum(1, np.rint(chord / step)).astype(np.int64)
    base_k = (N_POINTS - 1) * m + 1
    extra = (rng.random(n) < dup) & (base_k > 2)
    dpos = np.minimum(rng.integers(1, np.maximum(base_k - 1, 2)), base_k - 2)
    k = base_k + extra
    off = np.zeros(n + 1, np.int64)
    np.cumsum(k, out=off[1:])
    fid = np.repeat(np.arange(n), k)
    j = np.arange(off[-1]) - off[fid]
    j = j - (extra[fid] & (j > dpos[fid]))  # the repeated point reuses index dpos
    u = j / m[fid]
    i0 = np.minimum(np.floor(u).astype(np.int64), N_POINTS - 2)
    w = (u - i0)[:, None]
    pts = f[fid, i0] * (1 - w) + f[fid, i0 + 1] * w
    noise = rng.normal(0.0, jitter, (off[-1], 3))
    # the same displacement for a point and its repeat; none on the end points
    interior = (j > 0) & (j < base_k[fid] - 1)
    pts[interior] += noise[(off[fid] + j)[interior]]
    return pts.astype(np.float32), off


def raw_streamlines_torch(fibers, seed: int, step: float = 0.2, jitter: float = 0.02,
                          dup: float = 0.01, chunk: int = 1 << 19):
    """The raw-streamline recipe drawn with torch on the fibers' device (for
    paper-scale subjects, ~10^9 points): (points float32 [P, 3], offsets int64
    [n + 1]).  Same recipe as ``raw_streamlines``, a different random stream."""
    import torch

    dev = fibers.device
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    n = fibers.shape[0]
    f = fibers.to(torch.float32)
    chord = (f[:, 1] - f[:, 0]).double().pow(2).sum(1).sqrt()
    m = torch.clamp(torch.round(chord / step), min=1).long()
    base_k = (N_POINTS - 1) * m + 1
    extra = (torch.rand(n, generator=g, device=dev) < dup).long()
    dpos = 1 + (torch.rand(n, generator=g, device=dev, dtype=torch.float64)
                * (base_k - 2).double()).long()
    dpos = torch.minimum(dpos, base_k - 2)
    k = base_k + extra
    off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(k, 0, out=off[1:])
    total = int(off[-1].item())
    pts = torch.empty((total, 3), dtype=torch.float32, device=dev)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        p0, p1 = int(off[c0].item()), int(off[c1].item())
        kk = k[c0:c1]
        fid = torch.repeat_interleave(torch.arange(c0, c1, device=dev), kk, output_size=p1 - p0)
        j = torch.arange(p0, p1, device=dev) - off[fid]
        j = j - ((extra[fid] == 1) & (j > dpos[fid])).long()
        u = j.double() / m[fid].double()
        i0 = torch.clamp(torch.floor(u).long(), max=N_POINTS - 2)
        w = (u - i0.double()).float()[:, None]
        a = f[fid, i0]
        b = f[fid, i0 + 1]
        q = a * (1 - w) + b * w
        noise = torch.randn((p1 - p0, 3), generator=g, device=dev) * jitter
        # a repeated point takes the displacement of the point it repeats
        src = j + off[fid] - p0
        interior = (j > 0) & (j < base_k[fid] - 1)
        q = torch.where(interior[:, None], q + noise[src], q)
        pts[p0:p1] = q
    return pts, off


def make_atlas(spec: AtlasSpec, seed: int) -> Atlas:
    rng = _rng(seed, 0)
    cen = bezier_curves(rng, spec.n_centroids, spec.len_lo, spec.len_hi)
    bid = (np.arange(spec.n_centroids) // spec.per_bundle).astype(np.int32)
    thr = rng.uniform(spec.thr_lo, spec.thr_hi, spec.n_bundles).astype(np.float32)
    return Atlas(cen.astype(np.float32), bid, thr, spec)


def _fiber_chunk(atlases: Sequence[Atlas], matched: Sequence[float], sigma: float,
                 n: int, rng: np.random.Generator, hot=None) -> np.ndarray:
    n_all = n
    hot_part = None
    if hot is not None:
        # copies of the hot bundles' centroids (ids are bundle-major)
        n_hot = int(round(hot[0] * n))
        at0 = atlases[0]
        per = at0.spec.per_bundle if at0.spec else int(np.bincount(at0.bundle_id).max())
        nb_hot = max(1, int(round(hot[1] * (int(at0.bundle_id.max()) + 1))))
        hot_part = _copies(at0, rng.integers(0, nb_hot * per, n_hot), sigma, rng)
        n -= n_hot
    counts = [int(round(f * n)) for f in matched]
    n_match = sum(counts)
    if n_match > n:
        raise ValueError("matched fractions exceed 1")
    parts = [] if hot_part is None else [hot_part]
    for atlas, cnt in zip(atlases, counts):
        if cnt == 0:
            continue
        pick = rng.integers(0, atlas.n_centroids, cnt)
        parts.append(_copies(atlas, pick, sigma, rng))
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
    allf = allf[rng.permutation(n_all)]
    return allf.astype(np.float32)


def _copies(atlas: Atlas, pick: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Copies of centroids ``pick`` with a smooth displacement (4 knots of
    N(0, sigma) per axis, linear between them), half of them reversed."""
    cnt = pick.size
    base = atlas.centroids[pick].astype(np.float64)
    knots = rng.normal(0.0, sigma, (cnt, 4, 3))
    t = np.arange(N_POINTS) / (N_POINTS - 1)
    seg = np.minimum((t * 3).astype(int), 2)
    w = (t * 3 - seg)[None, :, None]
    disp = knots[:, seg, :] * (1 - w) + knots[:, seg + 1, :] * w
    f = base + disp
    flip = rng.random(cnt) < 0.5
    f[flip] = f[flip, ::-1, :]
    return f


def _chunk_job(args):
    atlases, subject, seed, subject_idx, c = args
    lo = c * CHUNK
    n = min(CHUNK, subject.n_fibers - lo)
    return _fiber_chunk(atlases, subject.matched, subject.sigma, n,
                        _rng(seed, 1, subject_idx, c), subject.hot)


def gpu_in_use() -> bool:
    """Whether this process has already initialised the GPU through torch.

    A forked worker would inherit that device state, so the fiber generator
    then draws its chunks in this process instead (same output)."""
    torch = sys.modules.get("torch")
    if torch is None:
        return False
    try:
        return bool(torch.cuda.is_initialized())
    except Exception:  # a torch without the cuda module: nothing initialised
        return False


def make_fibers(atlases: Sequence[Atlas], subject: SubjectSpec, seed: int,
                subject_idx: int = 0, start: int = 0, count: Optional[int] = None,
                workers: int = 1) -> np.ndarray:
    """Fibers [start, start+count) of a subject, float32 [count, 21, 3].

    ``workers`` > 1 draws the chunks in a pool of forked processes (same
    output), unless the process has initialised the GPU (``gpu_in_use``):
    then every chunk is drawn here, one after another.  A process whose GPU
    was initialised by something other than torch (a profiler's preloaded
    library) must pass ``workers=1`` itself.
    """
    if workers > 1 and gpu_in_use():
        workers = 1
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
