"""Pins of the CPU oracle to facts the paper and the mathematics fix.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with a fact that does not come from the oracle itself:
closed forms of d_ME (Eq. 2) on constructed curves, exact integer cases,
symmetry / reversal invariants, the special cases that reduce to a plain
nearest-neighbour argmin, an exact rational model of the float32 expression,
and an independent NumPy float64 brute force.  ``test_oracle_mutants`` runs
the same pins against deliberately broken builds of the oracle to show that
each plausible mistake is caught by at least one of them.
"""
from __future__ import annotations

import math

import numpy as np

import exact_fp32 as X
from oracle import BRUTE, CUT
from oracle import np_fp64

F32 = np.float32


def _smooth_curve(rng, length=60.0, start=(90.0, 110.0, 90.0)):
    """A gently bent curve of 21 points (no two points close to each other)."""
    t = np.linspace(0, 1, 21)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    v = rng.normal(size=3)
    v -= v.dot(u) * u
    v /= np.linalg.norm(v)
    pts = np.asarray(start)[None, :] + length * t[:, None] * u[None, :] \
        + 0.15 * length * np.sin(np.pi * t)[:, None] * v[None, :]
    return pts.astype(F32)


def _random_set(rng, n, m, nb, near=0.5):
    """Fibers near centroids plus free fibers; thresholds U(6, 10)."""
    cen = np.stack([_smooth_curve(rng, rng.uniform(20, 120),
                                  rng.uniform([20, 20, 20], [160, 200, 160])) for _ in range(m)])
    bid = (np.arange(m) * nb // max(m, 1)).astype(np.int32)
    thr = rng.uniform(6, 10, nb).astype(F32)
    fib = []
    for i in range(n):
        if rng.random() < near and m:
            c = cen[rng.integers(m)].astype(np.float64)
            f = c + rng.normal(0, 2.0, 3)[None, :] + rng.normal(0, 0.7, (21, 3))
            if rng.random() < 0.5:
                f = f[::-1]
        else:
            f = _smooth_curve(rng, rng.uniform(20, 120), rng.uniform([20, 20, 20], [160, 200, 160]))
        fib.append(f.astype(F32))
    return np.stack(fib), cen, bid, thr


# --------------------------------------------------------------------------
def pin_expression_rounding(O, n_pairs=60, seed=1):
    """Float32 d_ME^2 equals an exact rational model of the written expression."""
    rng = np.random.default_rng(seed)
    for k in range(n_pairs):
        scale = [1e-3, 1.0, 100.0, 1e4][k % 4]
        a = (rng.normal(0, scale, (21, 3)) + 100.0 * (k % 2)).astype(F32)
        b = (a + rng.normal(0, scale, (21, 3))).astype(F32)
        md, mi = O.pair_f32(a, b)
        emd, emi = X.pair(a, b)
        assert F32(md) == X.to_f32(emd) and F32(mi) == X.to_f32(emi), (k, md, float(emd), mi,
                                                                        float(emi))
    # subnormal differences must not be flushed to zero
    a = np.zeros((21, 3), F32)
    b = np.zeros((21, 3), F32)
    b[3, 0] = F32(1e-20)  # the square, 1e-40, is a binary32 subnormal
    md, mi = O.pair_f32(a, b)
    want = float(X.to_f32(X.pair(a, b)[0]))
    assert want > 0 and md == want, (md, want)


def pin_straight_translation(O, seed=2):
    """Straight fiber a, centroid a + t (or reversed a + t): d_ME = |t| exactly in R."""
    rng = np.random.default_rng(seed)
    for k in range(20):
        # the second half sits at the origin, where float32 differences of
        # the stored points are not exact (float64 must not round them)
        p = rng.uniform(40, 140, 3) if k < 10 else rng.uniform(-0.5, 0.5, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        s = rng.uniform(1.0, 4.0) if k < 10 else rng.uniform(0.01, 0.05)
        a = (p[None, :] + (np.arange(21) - 10)[:, None] * s * u[None, :]).astype(F32)
        t = rng.normal(0, 3.0, 3)
        for rev in (False, True):
            b = ((a[::-1] if rev else a).astype(np.float64) + t).astype(F32)
            # exact |t|^2 of the stored float32 points (direct order for b = a+t)
            diff = (a.astype(np.float64) - (b[::-1] if rev else b).astype(np.float64))
            want = float((diff ** 2).sum(1).max())
            md, mi = O.pair_f64(a, b)
            got = min(md, mi)
            assert abs(got - want) <= 1e-12 * want, (k, rev, got, want)
            md32, mi32 = O.pair_f32(a, b)
            assert abs(min(md32, mi32) - want) <= 1e-6 * want
            # the flipped order of a straight fiber is the worse one
            assert (mi if not rev else md) >= want * (1 - 1e-12)
            assert abs(math.sqrt(want) - np.linalg.norm(t)) < 1e-3


def pin_integer_exact(O):
    """Integer coordinates make every step exact: d = 13 for t = (3, 4, 12)."""
    a = np.stack([np.arange(21) * 2.0, np.full(21, 50.0), np.full(21, 60.0)], 1).astype(F32)
    b = (a + np.array([3.0, 4.0, 12.0])).astype(F32)
    md, mi = O.pair_f32(a, b)
    assert md == 169.0 and mi > 169.0
    bid = np.zeros(1, np.int32)
    lab, dist, best = O.segment_f32(a[None], b[None], bid, np.array([13.0], F32), mode=BRUTE)
    assert lab[0] == 0 and dist[0] == 13.0 and best[0] == 0
    # "under the threshold" is inclusive; one ulp below rejects
    lab, dist, _ = O.segment_f32(a[None], b[None], bid,
                                 np.array([np.nextafter(F32(13), F32(0))], F32), mode=BRUTE)
    assert lab[0] == -1 and dist[0] == np.inf
    for mode in (BRUTE, CUT):
        lab, dist, _ = O.segment_f32(a[None], b[None], bid, np.array([13.0], F32), mode=mode)
        assert lab[0] == 0 and dist[0] == 13.0
    lab, dist, _ = O.segment_f64(a[None], b[None], bid, np.array([13.0], F32))
    assert lab[0] == 0 and dist[0] == 13.0
    lab, dist, _ = O.segment_f64(a[None], b[None], bid,
                                 np.array([np.nextafter(F32(13), F32(0))], F32))
    assert lab[0] == -1 and dist[0] == np.inf


def pin_single_point(O, seed=3):
    """Moving one point of a copy by delta gives d_ME = |delta| (its order is direct)."""
    rng = np.random.default_rng(seed)
    for j in (0, 3, 10, 17, 20):
        a = _smooth_curve(rng)
        delta = np.array([0.0, 0.0, 0.0])
        delta[j % 3] = 2.0 + j / 10.0  # exactly representable sums on this grid
        b = a.astype(np.float64).copy()
        b[j] += delta
        b = b.astype(F32)
        want = float(((a[j].astype(np.float64) - b[j].astype(np.float64)) ** 2).sum())
        md, mi = O.pair_f64(a, b)
        assert md == want and mi > want, (j, md, mi, want)
        md32, mi32 = O.pair_f32(a, b)
        assert abs(min(md32, mi32) - want) <= 1e-6 * want
        # the same with the centroid stored in inverse order
        md, mi = O.pair_f64(a, b[::-1])
        assert mi == want and md > want


def pin_arcs(O):
    """Concentric arcs, radii R and R + r, same angles: d_ME = r."""
    R, r = 40.0, 5.0
    th = np.linspace(0.0, 1.2, 21)
    c = np.array([90.0, 110.0, 90.0])
    a = np.stack([c[0] + R * np.cos(th), c[1] + R * np.sin(th), np.full(21, c[2])], 1).astype(F32)
    b = np.stack([c[0] + (R + r) * np.cos(th), c[1] + (R + r) * np.sin(th),
                  np.full(21, c[2])], 1).astype(F32)
    md, mi = O.pair_f64(a, b)
    assert abs(math.sqrt(min(md, mi)) - r) < 1e-4, (md, mi)
    assert mi > md
    lab, dist, _ = O.segment_f64(a[None], b[None], np.zeros(1, np.int32), np.array([5.01], F32))
    assert lab[0] == 0 and abs(dist[0] - r) < 1e-4


def pin_invariants(O, seed=4):
    """Symmetry, reversal and self-distance hold bit for bit in float32."""
    rng = np.random.default_rng(seed)
    for k in range(40):
        a = _smooth_curve(rng, rng.uniform(20, 100))
        b = (a + rng.normal(0, 3, (21, 3))).astype(F32) if k % 2 else \
            _smooth_curve(rng, rng.uniform(20, 100))
        d_ab = min(O.pair_f32(a, b))
        assert d_ab == min(O.pair_f32(b, a))
        assert d_ab == min(O.pair_f32(a[::-1], b)) == min(O.pair_f32(a, b[::-1]))
        assert O.pair_f32(a, a) == (0.0, O.pair_f32(a, a)[1]) and min(O.pair_f32(a, a[::-1])) == 0
        # D is at least every single point distance of the better order, and
        # at least the center distance (which both orders share)
        md, mi = O.pair_f32(a, b)
        dc = float(X.to_f32(X.d2(a[10], b[10])))
        assert md >= dc and mi >= dc
        assert md == max(float(X.to_f32(X.d2(a[i], b[i]))) for i in range(21))


def pin_set_invariants(O, seed=5):
    """Fiber reversal and permutation leave the per-fiber outputs unchanged."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _random_set(rng, 60, 25, 7)
    lab, dist, best = O.segment_f32(fib, cen, bid, thr, mode=BRUTE)
    assert (lab >= 0).sum() >= 10, "the set should contain matches"
    lab2, dist2, best2 = O.segment_f32(fib[:, ::-1], cen, bid, thr, mode=BRUTE)
    assert np.array_equal(lab, lab2) and np.array_equal(dist, dist2)
    perm = rng.permutation(len(fib))
    lab3, dist3, _ = O.segment_f32(fib[perm], cen, bid, thr, mode=BRUTE)
    assert np.array_equal(lab3, lab[perm]) and np.array_equal(dist3, dist[perm])


def pin_ties_and_order(O, seed=6):
    """Closest centroid wins over the first found; equal distance keeps the lower index."""
    rng = np.random.default_rng(seed)
    a = _smooth_curve(rng)
    far = (a.astype(np.float64) + [0.0, 0.0, 4.0]).astype(F32)
    near = (a.astype(np.float64) + [0.0, 3.0, 0.0]).astype(F32)
    cen = np.stack([far, near])
    bid = np.array([0, 1], np.int32)
    thr = np.array([10.0, 10.0], F32)
    for mode in (BRUTE, CUT):
        lab, dist, best = O.segment_f32(a[None], cen, bid, thr, mode=mode)
        assert lab[0] == 1 and best[0] == 1 and abs(dist[0] - 3.0) < 1e-5
    # duplicate centroid with a higher index (other bundle) never wins
    cen = np.stack([near, far, near])
    bid = np.array([2, 0, 1], np.int32)
    thr = np.array([10.0, 10.0, 10.0], F32)
    for mode in (BRUTE, CUT):
        lab, dist, best = O.segment_f32(a[None], cen, bid, thr, mode=mode)
        assert lab[0] == 2 and best[0] == 0


def pin_threshold_per_bundle(O, seed=7):
    """The threshold is the one of the centroid's own bundle; labels are bundle ids."""
    rng = np.random.default_rng(seed)
    a = _smooth_curve(rng)
    c0 = (a.astype(np.float64) + [5.0, 0.0, 0.0]).astype(F32)   # d = 5
    c1 = (a.astype(np.float64) + [0.0, 7.0, 0.0]).astype(F32)   # d = 7
    cen = np.stack([c0, c1, c1, c1])
    bid = np.array([1, 0, 0, 0], np.int32)  # centroid 0 is bundle 1
    thr = np.array([8.0, 4.0], F32)          # bundle 1 rejects d = 5, bundle 0 accepts 7
    for mode in (BRUTE, CUT):
        lab, dist, best = O.segment_f32(a[None], cen, bid, thr, mode=mode)
        assert lab[0] == 0 and best[0] == 1 and abs(dist[0] - 7.0) < 1e-5, (lab, best, dist)
    lab, dist, best = O.segment_f64(a[None], cen, bid, thr)
    assert lab[0] == 0 and best[0] == 1


def pin_special_cases(O, seed=8):
    """Infinite thresholds reduce to a nearest-centroid argmin; negative ones never match."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _random_set(rng, 40, 15, 5, near=0.3)
    inf = np.full(5, np.inf, F32)
    d = np_fp64.dme_matrix(fib, cen)
    lab, dist, best = O.segment_f32(fib, cen, bid, inf, mode=BRUTE)
    srt = np.sort(d, 1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-4 * srt[:, 0]
    assert clear.sum() > 30
    assert np.array_equal(best[clear], np.argmin(d, 1)[clear])
    assert np.array_equal(lab[clear], bid[np.argmin(d, 1)][clear])
    lab, dist, best = O.segment_f32(fib, cen, bid, np.full(5, -1.0, F32), mode=CUT)
    assert (lab == -1).all() and np.isinf(dist).all() and (best == -1).all()
    lab, dist, best = O.segment_f32(fib, cen[:0], bid[:0], thr, mode=CUT)
    assert (lab == -1).all() and np.isinf(dist).all()
    lab, dist, best = O.segment_f32(fib[:0], cen, bid, thr)
    assert lab.shape == (0,)
    # a single centroid: label iff d_ME <= T
    for i in range(10):
        lab, dist, _ = O.segment_f64(fib[i:i + 1], cen[:1], bid[:1] * 0, np.array([8.0], F32))
        assert (lab[0] == 0) == (d[i, 0] <= 8.0)


def pin_cut_equals_brute(O, seed=9):
    """The paper's progressive discard reaches exactly the brute-force result."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _random_set(rng, 150, 40, 9, near=0.7)
    # near-threshold pairs: a copy translated by exactly the threshold
    extra = []
    for k in range(30):
        c = rng.integers(len(cen))
        t = rng.normal(size=3)
        t *= float(thr[bid[c]]) / np.linalg.norm(t) * (1 + (k % 3 - 1) * 1e-7)
        f = (cen[c].astype(np.float64) + t).astype(F32)
        extra.append(f[::-1] if k % 2 else f)
    fib = np.concatenate([fib, np.stack(extra)])
    a = O.segment_f32(fib, cen, bid, thr, mode=BRUTE)
    b = O.segment_f32(fib, cen, bid, thr, mode=CUT)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert (a[0] >= 0).sum() > 60


def pin_f64_vs_numpy(O, seed=10):
    """C float64 loops agree with the vectorised NumPy float64 brute force.

    The set is shifted to straddle the origin, where float32 differences of
    the inputs are not exact, so the float64 oracle must not round them.
    """
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _random_set(rng, 120, 30, 6, near=0.6)
    shift = np.array([90.0, 110.0, 90.0])
    fib = (fib.astype(np.float64) - shift).astype(F32)
    cen = (cen.astype(np.float64) - shift).astype(F32)
    lab, dist, best = O.segment_f64(fib, cen, bid, thr)
    nl, nd, nb = np_fp64.segment(fib, cen, bid, thr)
    d = np_fp64.dme_matrix(fib, cen)
    t = thr.astype(np.float64)[bid]
    margin = np.abs(d - t[None, :]).min(1) > 1e-9
    assert np.array_equal(lab[margin], nl[margin])
    ok = lab >= 0
    assert np.allclose(dist[ok & margin], nd[ok & margin], rtol=1e-12, atol=0)
    assert (ok & margin).sum() > 40


def pin_f32_vs_f64(O, seed=11):
    """The float32 decision agrees with float64 away from the boundary and ties."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _random_set(rng, 120, 30, 6, near=0.6)
    l32, d32, b32 = O.segment_f32(fib, cen, bid, thr, mode=BRUTE)
    l64, d64, b64 = O.segment_f64(fib, cen, bid, thr)
    d = np_fp64.dme_matrix(fib, cen)
    t = thr.astype(np.float64)[bid]
    dm = np.where(d <= t[None, :], d, np.inf)
    srt = np.sort(dm, 1)
    with np.errstate(invalid="ignore"):
        tie = (srt[:, 1] - srt[:, 0]) <= 1e-4
    clear = (np.abs(d - t[None, :]).min(1) > 1e-4) & ~tie
    assert clear.sum() > 60
    assert np.array_equal(l32[clear], l64[clear])
    ok = clear & (l64 >= 0)
    assert np.allclose(d32[ok].astype(np.float64), d64[ok], rtol=1e-6, atol=0)


ALL_PINS = [
    pin_expression_rounding,
    pin_straight_translation,
    pin_integer_exact,
    pin_single_point,
    pin_arcs,
    pin_invariants,
    pin_set_invariants,
    pin_ties_and_order,
    pin_threshold_per_bundle,
    pin_special_cases,
    pin_cut_equals_brute,
    pin_f64_vs_numpy,
    pin_f32_vs_f64,
]
