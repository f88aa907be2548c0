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

import functools
import math

import numpy as np

import exact_fp32 as X
from oracle import BRUTE, CUT, DIR, TN
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


# ------------------------------------------------------------ metric variants
def _line(length, n=21):
    """Straight polyline along x, centered at the origin, spacing length / 20."""
    p = np.zeros((n, 3), F32)
    p[:, 0] = (np.arange(n) - 10) * (length / 20.0)
    return p


def pin_tn_closed_form(O):
    """Collinear centered lines of lengths L and L' (spacings exact in float):
    d_ME = |L - L'| / 2, TN = (|L - L'| / max + 1)^2 - 1, metric = d_ME + TN."""
    for L, Lc, dme, tn in [(40.0, 20.0, 10.0, 1.25), (40.0, 30.0, 5.0, 0.5625),
                           (40.0, 10.0, 15.0, 2.0625), (20.0, 40.0, 10.0, 1.25)]:
        a, b = _line(L), _line(Lc)
        assert O.arc_length_f32(a) == L and O.arc_length_f32(b) == Lc
        assert O.tn_f32(L, Lc) == tn
        bid = np.zeros(1, np.int32)
        for fib in (a, a[::-1].copy()):
            for T, ok in [(dme + tn + 0.25, True), (dme + tn - 0.25, False)]:
                for mode in (BRUTE, CUT):
                    lab, dist, _ = O.segment_ext_f32(fib[None], b[None], bid,
                                                     np.array([T], F32), TN, mode=mode)
                    if ok:
                        assert lab[0] == 0 and dist[0] == dme + tn
                    else:
                        assert lab[0] == -1 and np.isinf(dist[0])
                # without the length term the pair is accepted at d_ME
                lab, dist, _ = O.segment_ext_f32(fib[None], b[None], bid,
                                                 np.array([dme + tn - 0.25], F32), 0)
                assert lab[0] == 0 and dist[0] == dme


def pin_tn_properties(O, seed=12):
    """TN is symmetric, zero for equal lengths, in [0, 3]; the length-normalised
    labels are a subset of the plain ones with no smaller distance; integer
    translates (identical lengths) keep their plain result."""
    rng = np.random.default_rng(seed)
    for _ in range(200):
        ls, lc = (rng.uniform(1, 200, 2)).astype(F32)
        t = O.tn_f32(float(ls), float(lc))
        assert t == O.tn_f32(float(lc), float(ls))
        assert 0.0 <= t <= 3.0
        assert O.tn_f32(float(ls), float(ls)) == 0.0
    assert O.tn_f32(0.0, 0.0) == 0.0
    fib, cen, bid, thr = _random_set(rng, 150, 25, 5, near=0.7)
    l0, d0, _ = O.segment_f32(fib, cen, bid, thr, mode=BRUTE)
    l1, d1, _ = O.segment_ext_f32(fib, cen, bid, thr, TN, mode=BRUTE)
    lab = l1 >= 0
    assert (l0[lab] >= 0).all() and (d1[lab] >= d0[lab]).all()
    assert lab.sum() > 20
    # integer curves and integer translations: equal lengths, TN = 0 for the source
    cen_i = np.round(cen[:6] / 4.0).astype(F32) * 4.0
    shift = rng.integers(-2, 3, (6, 3)).astype(F32)
    fib_i = cen_i + shift[:, None, :]
    bid_i = np.arange(6, dtype=np.int32)
    thr_i = np.full(6, 5.0, F32)
    l0, d0, b0 = O.segment_f32(fib_i, cen_i, bid_i, thr_i, mode=BRUTE)
    l1, d1, b1 = O.segment_ext_f32(fib_i, cen_i, bid_i, thr_i, TN, mode=BRUTE)
    same = b0 == np.arange(6)
    assert same.sum() >= 4
    assert np.array_equal(l1[same], l0[same]) and np.array_equal(d1[same], d0[same])


def pin_variants_cut_equals_brute(O, seed=13):
    """Each variant reaches the same result by the paper's progressive discard
    as by its brute-force definition; no flags is the plain decision."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _random_set(rng, 200, 40, 8, near=0.6)
    base = O.segment_f32(fib, cen, bid, thr, mode=BRUTE)
    e0 = O.segment_ext_f32(fib, cen, bid, thr, 0, mode=CUT)
    assert all(np.array_equal(x, y) for x, y in zip(base, e0))
    for flags in (TN, DIR, TN | DIR):
        a = O.segment_ext_f32(fib, cen, bid, thr, flags, mode=BRUTE)
        b = O.segment_ext_f32(fib, cen, bid, thr, flags, mode=CUT)
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), flags


def _arc(radius, span_deg, center=(100.0, 100.0, 100.0), n=21, start_deg=0.0):
    th = np.deg2rad(start_deg + np.arange(n) * span_deg / (n - 1))
    p = np.zeros((n, 3))
    p[:, 0] = center[0] + radius * np.cos(th)
    p[:, 1] = center[1] + radius * np.sin(th)
    p[:, 2] = center[2]
    return p.astype(F32)


def pin_dir_closed_form(O):
    """A 300-degree arc b and the fiber a with b's end points but its interior in
    the inverse order: the end points choose the direct order, whose largest
    distance is the widest interior chord (the diameter, 2R), while Eq. 2 takes
    the inverse order, whose largest distance is the end-point chord (R)."""
    R = 20.0
    b = _arc(R, 300.0)
    a = b.copy()
    a[1:20] = b[19:0:-1]
    bid = np.zeros(1, np.int32)
    pa, pb = a.astype(np.float64), b.astype(np.float64)
    d_dir = max(((pa[i] - pb[i]) ** 2).sum() for i in range(21))
    d_inv = max(((pa[i] - pb[20 - i]) ** 2).sum() for i in range(21))
    assert abs(math.sqrt(d_dir) - 2 * R) < 1e-3 and abs(math.sqrt(d_inv) - R) < 1e-3
    for T in (25.0, 45.0):
        thr = np.array([T], F32)
        for mode in (BRUTE, CUT):
            le, de, _ = O.segment_ext_f32(a[None], b[None], bid, thr, 0, mode=mode)
            ld, dd, _ = O.segment_ext_f32(a[None], b[None], bid, thr, DIR, mode=mode)
            assert le[0] == 0 and abs(de[0] - math.sqrt(d_inv)) <= 1e-5 * R
            if T < 2 * R:
                assert ld[0] == -1 and np.isinf(dd[0])
            else:
                assert ld[0] == 0 and abs(dd[0] - math.sqrt(d_dir)) <= 1e-5 * 2 * R


def pin_dir_tie_direct(O):
    """A closed loop centroid (b_0 = b_20) ties the end-point test of any fiber;
    the tie takes the direct order."""
    b = _arc(15.0, 360.0)
    b[20] = b[0]
    a = b.copy()
    a[1:20] = b[19:0:-1]  # interior in the inverse order: direct order is far off
    a += F32(0.5)
    bid = np.zeros(1, np.int32)
    thr = np.array([100.0], F32)
    pa, pb = a.astype(np.float64), b.astype(np.float64)
    d_dir = max(((pa[i] - pb[i]) ** 2).sum() for i in range(21))
    d_inv = max(((pa[i] - pb[20 - i]) ** 2).sum() for i in range(21))
    assert d_dir > 4 * d_inv
    for mode in (BRUTE, CUT):
        ld, dd, _ = O.segment_ext_f32(a[None], b[None], bid, thr, DIR, mode=mode)
        assert ld[0] == 0 and abs(dd[0] - math.sqrt(d_dir)) <= 1e-5 * math.sqrt(d_dir)


def pin_dir_consistent_copies(O, seed=14):
    """Noisy copies (either order) of well-separated open curves: the end points
    pick the order Eq. 2 takes, so direction inference changes nothing."""
    rng = np.random.default_rng(seed)
    cen = np.stack([_smooth_curve(rng, rng.uniform(60, 120),
                                  rng.uniform([20, 20, 20], [120, 160, 120])) for _ in range(12)])
    bid = np.arange(12, dtype=np.int32)
    thr = np.full(12, 3.0, F32)
    fib = []
    for i in range(120):
        f = cen[i % 12].astype(np.float64) + rng.normal(0, 0.3, (21, 3))
        fib.append((f[::-1] if i % 2 else f).astype(F32))
    fib = np.stack(fib)
    e = O.segment_ext_f32(fib, cen, bid, thr, 0, mode=BRUTE)
    d = O.segment_ext_f32(fib, cen, bid, thr, DIR, mode=BRUTE)
    assert (e[0] >= 0).mean() > 0.9
    assert all(np.array_equal(x, y) for x, y in zip(e, d))


# ---------------------------------------------------------------- resampling

def _csr(lines):
    """Stack polylines into (points [P, 3] float32, offsets [n + 1] int64)."""
    off = np.zeros(len(lines) + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in lines])
    pts = np.concatenate([np.asarray(x, F32).reshape(-1, 3) for x in lines]) if lines else \
        np.zeros((0, 3), F32)
    return pts, off


def _raw_curve(rng, npts, length, start):
    """A smooth bent curve sampled at ``npts`` random, unevenly spaced parameters."""
    t = np.sort(rng.uniform(0, 1, npts))
    t[0], t[-1] = 0.0, 1.0
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    v = rng.normal(size=3)
    v -= v.dot(u) * u
    v /= np.linalg.norm(v)
    pts = np.asarray(start)[None, :] + length * t[:, None] * u[None, :] \
        + 0.2 * length * np.sin(np.pi * t)[:, None] * v[None, :]
    return pts.astype(F32)


def _interp_f64(p):
    """21 points equidistant in arc length by np.interp over the float64
    cumulative length (a library routine, not the oracle's loop)."""
    q = p.astype(np.float64)
    cum = np.concatenate([[0.0], np.cumsum(np.sqrt((np.diff(q, axis=0) ** 2).sum(1)))])
    t = np.linspace(0.0, cum[-1], 21)
    return np.stack([np.interp(t, cum, q[:, c]) for c in range(3)], 1)


def pin_resample_closed_forms(O):
    """Straight lines with exact spacings: 41 points j (1.5, 2, 0) give k (3, 4, 0);
    two points give p0 + k/20 (p1 - p0); 21 unit steps give the input back; one
    point or a zero-length line gives 21 copies; end points are copied."""
    base = np.array([64.0, 32.0, 16.0])
    line = base + np.arange(41)[:, None] * np.array([1.5, 2.0, 0.0])
    two = np.array([[10.0, 20.0, 30.0], [30.0, 60.0, 90.0]])
    steps = [np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, -1.0])]
    walk = np.zeros((21, 3))
    walk[0] = base
    for i in range(1, 21):
        walk[i] = walk[i - 1] + steps[i % 3]
    single = np.array([[5.0, 6.0, 7.0]])
    still = np.repeat(np.array([[1.0, 2.0, 3.0]]), 7, 0)
    out = O.resample_f32(*_csr([line, two, walk, single, still]))
    k = np.arange(21)[:, None]
    assert np.array_equal(out[0], (base + k * np.array([3.0, 4.0, 0.0])).astype(F32))
    want2 = two[0] + k / 20.0 * (two[1] - two[0])
    assert np.abs(out[1] - want2).max() <= 4 * 2.0**-24 * 90.0
    assert np.array_equal(out[1][[0, 20]], two.astype(F32))
    assert np.array_equal(out[2], walk.astype(F32))
    assert np.array_equal(out[3], np.repeat(single, 21, 0).astype(F32))
    assert np.array_equal(out[4], np.repeat(still[:1], 21, 0).astype(F32))


def pin_resample_uneven_line(O, seed=15):
    """A straight line with uneven spacing (coordinates on a 1/64 grid, so the
    arc length sums are exact): point k sits at arc length k L / 20, not at
    an index fraction."""
    rng = np.random.default_rng(seed)
    for _ in range(5):
        x = np.unique(np.round(rng.uniform(0, 40, 30) * 64) / 64)
        x = np.concatenate([[0.0], x[(x > 0) & (x < 40)], [40.0]])
        p = np.zeros((x.size, 3))
        p[:, 0] = 50.0 + x
        p[:, 1] = 70.0
        p[:, 2] = 90.0
        out = O.resample_f32(*_csr([p]))[0]
        want = 50.0 + 2.0 * np.arange(21)
        assert np.abs(out[:, 0] - want).max() <= 2.0**-24 * 90.0 * 2
        assert (out[:, 1] == 70.0).all() and (out[:, 2] == 90.0).all()


def pin_resample_vs_interp(O, seed=16):
    """Smooth curves sampled unevenly (2 to 600 points) agree with np.interp over
    the float64 arc length within the float32 error of P sequential sums."""
    rng = np.random.default_rng(seed)
    lines = [_raw_curve(rng, int(rng.integers(2, 600)), rng.uniform(5, 200),
                        rng.uniform([20, 20, 20], [150, 190, 150])) for _ in range(60)]
    out = O.resample_f32(*_csr(lines))
    for p, o in zip(lines, out):
        want = _interp_f64(p)
        L = float(np.sqrt((np.diff(p.astype(np.float64), axis=0) ** 2).sum(1)).sum())
        tol = 2.0 * (len(p) + 4) * 2.0**-24 * L + 1e-5
        assert np.abs(o - want).max() <= tol, (len(p), np.abs(o - want).max(), tol)
        assert np.array_equal(o[[0, 20]], p[[0, -1]])


@functools.lru_cache(maxsize=1)
def _long_line():
    """2^24 + 1 points 0.25 mm apart along x (exact in float32)."""
    big = np.zeros((2**24 + 1, 3), F32)
    big[:, 0] = np.arange(2**24 + 1, dtype=F32) * F32(0.25)
    big.setflags(write=False)
    return big


def pin_resample_invariants(O, seed=17):
    """Repeating points (zero-length steps) changes nothing, bit for bit; a set
    gives each streamline's own result; reversal gives the reversed points
    within the float32 error; bad offsets are rejected."""
    rng = np.random.default_rng(seed)
    lines = [_raw_curve(rng, int(rng.integers(3, 300)), rng.uniform(10, 150),
                        rng.uniform([20, 20, 20], [150, 190, 150])) for _ in range(20)]
    whole = O.resample_f32(*_csr(lines))
    for i, p in enumerate(lines):
        assert np.array_equal(O.resample_f32(*_csr([p]))[0], whole[i])
        rep = np.repeat(p, rng.integers(1, 3, len(p)), axis=0)
        assert np.array_equal(O.resample_f32(*_csr([rep]))[0], whole[i])
        rev = O.resample_f32(*_csr([p[::-1]]))[0]
        L = float(np.sqrt((np.diff(p.astype(np.float64), axis=0) ** 2).sum(1)).sum())
        assert np.abs(rev[::-1] - whole[i]).max() <= 4.0 * (len(p) + 4) * 2.0**-24 * L + 1e-5
    pts, off = _csr(lines[:3])
    for bad in ([0, 5, 5, off[3]], [0, 5, 3, off[3]], [0, 5, 9, off[3] + 1], [-1, 5, 9, off[3]]):
        try:
            O.resample_f32(pts, np.array(bad, np.int64))
        except ValueError:
            continue
        raise AssertionError(f"offsets {bad} accepted")
    # at most 2^24 points per streamline: the exact sum stays below 2^62
    big = _long_line()
    one = O.resample_f32(big[:2**24], np.array([0, 2**24], np.int64))[0]
    assert one[10, 0] == F32(0.25 * (2**24 - 1) / 2) and one[20, 0] == big[2**24 - 1, 0]
    try:
        O.resample_f32(big, np.array([0, 2**24 + 1], np.int64))
    except ValueError:
        pass
    else:
        raise AssertionError("a streamline of 2^24 + 1 points accepted")


def pin_resample_rounding_corners(O):
    """Corners of the fixed-point reading, worked by hand (lengths in units of
    u = 2^-24 mm).
    (a) A tie.  Along x: 0, 4096, 2^-13, 8192.  fl(2^-13 - 4096) = -4096 (a
        tie, to even) and fl(8192 - 2^-13) = 8192, so the lengths are 2^36,
        2^36, 2^37 u, L = 2^38 and t_10 = 2^37 = S_2: the first segment
        reaching t_10 is the second, at w = 1, and fma(1, -4096, 4096) puts
        point 10 at x = 0, not at the third input point (x = 2^-13).
    (b) Saturation.  Along x: 0, 20000, 60000: both lengths are at least 2^14
        mm and count 2^38 u each, L = 2^39; t_10 = S_1 is the end of the first
        segment (x = 20000) and t_5 its middle (x = 10000).  Unsaturated
        lengths would put them at 30000 and 15000.
    (c) Exact sums.  (0,0,0), (4096,0,0), then 4096 steps of 2^-12 mm along y:
        L = 2^36 + 2^24 u (4097 mm) exactly, t_10 = L / 2, w = 1/2 + 2^-13, so
        point 10 is (2048.5, 0, 0).  A float32 running sum stays at 4096
        (4096 + 2^-12 is a tie, to even) and would give 2048.
    (d) Floored targets.  Along x: 0, 10 u, 19 u: L = 19 u, t_10 = floor(9.5)
        = 9 on the first segment at w = fl(9/10), so point 10 is at 9 u (fl(fl(0.9)
        * 10) = 9); a rounded target (10) would give 10 u."""
    u = 2.0**-24
    a = np.array([[0.0, 0, 0], [4096.0, 0, 0], [2.0**-13, 0, 0], [8192.0, 0, 0]])
    b = np.array([[0.0, 0, 0], [20000.0, 0, 0], [60000.0, 0, 0]])
    c = np.zeros((4098, 3))
    c[1:, 0] = 4096.0
    c[2:, 1] = np.arange(1, 4097) * 2.0**-12
    d = np.array([[0.0, 0, 0], [10 * u, 0, 0], [19 * u, 0, 0]])
    out = O.resample_f32(*_csr([a, b, c, d]))
    assert np.array_equal(out[0][10], np.array([0.0, 0.0, 0.0], F32)), out[0][10]
    assert np.array_equal(out[1][10], np.array([20000.0, 0.0, 0.0], F32)), out[1][10]
    assert np.array_equal(out[1][5], np.array([10000.0, 0.0, 0.0], F32)), out[1][5]
    assert np.array_equal(out[2][10], np.array([2048.5, 0.0, 0.0], F32)), out[2][10]
    assert np.array_equal(out[2][20], np.array([4096.0, 1.0, 0.0], F32)), out[2][20]
    assert np.array_equal(out[3][10], np.array([9 * u, 0.0, 0.0], F32)), out[3][10]


# ---------------------------------------------------------------- several labels

def _overlapping_set(rng, n=300, nb=6, per=4):
    """Bundles that share shapes: each base curve has shifted copies (0.5 to 3
    mm) in two or three bundles, so many fibers pass several bundles."""
    base = [_smooth_curve(rng, rng.uniform(30, 90), rng.uniform([30, 30, 30], [120, 150, 120]))
            for _ in range(per * 2)]
    cen, bid = [], []
    for b in range(nb):
        for k in range(per):
            c = base[(b * per // 2 + k) % len(base)].astype(np.float64)
            cen.append((c + rng.uniform(-3, 3, 3)[None, :]).astype(F32))
            bid.append(b)
    cen = np.stack(cen)
    bid = np.array(bid, np.int32)
    fib = np.stack([(base[rng.integers(len(base))].astype(np.float64)
                     + rng.normal(0, 0.7, (21, 3)))[::(1 if rng.random() < 0.5 else -1)]
                    .astype(F32) for _ in range(n)])
    thr = rng.uniform(3.0, 6.0, nb).astype(F32)
    return fib, cen, bid, thr


def _rows(off, bun, dst):
    return [(bun[off[f]:off[f + 1]], dst[off[f]:off[f + 1]]) for f in range(len(off) - 1)]


def pin_multi_closed_form(O):
    """Translated copies of a straight fiber (d_ME = |t|, exact): bundle 0 holds
    copies at 3 and 1.5 mm (T = 2), bundle 1 at 1 and 2 mm (T = 2.5), bundle 2
    at 5 mm (T = 4), bundle 3 none: the fiber is in bundles 0 (1.5) and 1 (1)."""
    a = np.zeros((21, 3))
    a[:, 0] = 40.0 + 2.0 * np.arange(21)
    a[:, 1] = 60.0
    a[:, 2] = 70.0
    shifts = [(3.0, 0), (1.5, 0), (1.0, 1), (2.0, 1), (5.0, 2)]
    cen = np.stack([a + np.array([0.0, t, 0.0]) for t, _ in shifts]).astype(F32)
    bid = np.array([b for _, b in shifts], np.int32)
    thr = np.array([2.0, 2.5, 4.0, 9.0], F32)
    fib = np.stack([a, a[::-1]]).astype(F32)
    for mode in (BRUTE, CUT):
        off, bun, dst, cnt = O.segment_multi_f32(fib, cen, bid, thr, 0, mode=mode)
        assert off.tolist() == [0, 2, 4]
        assert bun.tolist() == [0, 1, 0, 1] and dst.tolist() == [1.5, 1.0, 1.5, 1.0]
        assert cnt.tolist() == [2, 2, 0, 0]


def pin_multi_single_consistency(O, seed=18):
    """The closest-bundle label is one of the fiber's bundles, at the smallest
    of its distances; unlabelled fibers have none; bundle counts are the
    histogram of the entries; bundles increase within a fiber."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _overlapping_set(rng)
    for flags in (0, TN, DIR, TN | DIR):
        off, bun, dst, cnt = O.segment_multi_f32(fib, cen, bid, thr, flags)
        lab, dist, _ = O.segment_ext_f32(fib, cen, bid, thr, flags)
        assert np.array_equal(cnt, np.bincount(bun, minlength=len(thr)))
        for f, (b, d) in enumerate(_rows(off, bun, dst)):
            assert (np.diff(b) > 0).all()
            if lab[f] < 0:
                assert b.size == 0
            else:
                assert lab[f] in b and d[list(b).index(lab[f])] == dist[f] == d.min()
        if flags == 0:
            assert (np.diff(off) >= 2).sum() > 30


def pin_multi_infinite_thresholds(O, seed=19):
    """T = +inf: every fiber is in every bundle with centroids, at the smallest
    d_ME over the bundle (NumPy float64 brute force); T < 0: in none."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _overlapping_set(rng, n=40)
    bid = bid.copy()
    bid[bid == 2] = 3  # bundle 2 has no centroids
    inf = np.full(len(thr), np.inf, F32)
    off, bun, dst, cnt = O.segment_multi_f32(fib, cen, bid, inf, 0)
    d64 = np_fp64.dme_matrix(fib, cen)  # [n, m]
    have = sorted(set(bid.tolist()))
    assert np.array_equal(np.diff(off), np.full(len(fib), len(have)))
    for f, (b, d) in enumerate(_rows(off, bun, dst)):
        assert b.tolist() == have
        want = np.array([d64[f, bid == k].min() for k in have])
        assert np.allclose(d, want, rtol=1e-5, atol=1e-5)
    assert cnt.tolist() == [len(fib) if k in have else 0 for k in range(len(thr))]
    off, bun, dst, cnt = O.segment_multi_f32(fib, cen, bid, np.full(len(thr), -1.0, F32), 0)
    assert off[-1] == 0 and cnt.sum() == 0


def pin_multi_cut_equals_brute(O, seed=20):
    """The paper's progressive discard gives the same entries as brute force."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _overlapping_set(rng, n=150)
    for flags in (0, TN, DIR):
        a = O.segment_multi_f32(fib, cen, bid, thr, flags, mode=BRUTE)
        b = O.segment_multi_f32(fib, cen, bid, thr, flags, mode=CUT)
        assert all(np.array_equal(x, y) for x, y in zip(a, b))


def pin_accepted_pairs(O, seed=21):
    """The accepted-pair list is the set {(f, c) : d_ME(f, c) <= T[bid[c]]}
    (section 2.3: a fiber is kept for a bundle only under that bundle's own
    threshold), in fiber-major then centroid order.  Checked against the NumPy
    float64 brute force on pairs away from the boundary, and exactly on the
    special thresholds: all +inf gives every one of the N*M pairs, all
    negative gives none, and one +inf bundle among negative ones gives exactly
    the pairs of that bundle's centroids."""
    rng = np.random.default_rng(seed)
    fib, cen, bid, thr = _random_set(rng, 60, 24, 6, near=0.7)
    n, m = len(fib), len(cen)
    d = np_fp64.dme_matrix(fib, cen)
    t = thr.astype(np.float64)[bid]
    acc = O.accepted_pairs_f32(fib, cen, bid, thr)
    assert acc.ndim == 2 and acc.shape[1] == 2
    key = acc[:, 0] * m + acc[:, 1]
    assert (np.diff(key) > 0).all(), "pairs not in fiber-major, centroid order"
    got = np.zeros((n, m), bool)
    got[acc[:, 0], acc[:, 1]] = True
    clear = np.abs(d - t[None, :]) > 1e-4 * t[None, :]
    want = d <= t[None, :]
    assert np.array_equal(got[clear], want[clear])
    assert clear.mean() > 0.99 and want.sum() > 30
    # the labels follow from the same set: a fiber is labelled iff it has a pair
    lab, _, best = O.segment_f32(fib, cen, bid, thr, mode=BRUTE)
    assert np.array_equal(lab >= 0, got.any(1))
    assert all(got[f, best[f]] for f in np.nonzero(lab >= 0)[0])
    nb = len(thr)
    acc = O.accepted_pairs_f32(fib, cen, bid, np.full(nb, np.inf, F32))
    ff, cc = np.meshgrid(np.arange(n), np.arange(m), indexing="ij")
    assert np.array_equal(acc, np.stack([ff.ravel(), cc.ravel()], 1))
    acc = O.accepted_pairs_f32(fib, cen, bid, np.full(nb, -1.0, F32))
    assert acc.shape == (0, 2)
    # the boundary itself: integer points 13 mm apart (exact in float32) are
    # accepted at T = 13 and not at the next float below
    a = np.stack([np.arange(21.0), np.zeros(21), np.zeros(21)], 1).astype(F32) + 50
    c = (a.astype(np.float64) + [3.0, 4.0, 12.0]).astype(F32)
    for t13, k in ((13.0, 1), (np.nextafter(F32(13.0), F32(0.0)), 0)):
        acc = O.accepted_pairs_f32(a[None], c[None], np.zeros(1, np.int32), np.array([t13], F32))
        assert len(acc) == k, (t13, acc)
    for k in (0, nb - 1):
        one = np.full(nb, -1.0, F32)
        one[k] = np.inf
        acc = O.accepted_pairs_f32(fib, cen, bid, one)
        cols = np.nonzero(bid == k)[0]
        want = np.stack([np.repeat(np.arange(n), len(cols)), np.tile(cols, n)], 1)
        assert np.array_equal(acc, want), k


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
    pin_tn_closed_form,
    pin_tn_properties,
    pin_variants_cut_equals_brute,
    pin_dir_closed_form,
    pin_dir_tie_direct,
    pin_dir_consistent_copies,
    pin_resample_closed_forms,
    pin_resample_uneven_line,
    pin_resample_vs_interp,
    pin_resample_invariants,
    pin_resample_rounding_corners,
    pin_multi_closed_form,
    pin_multi_single_consistency,
    pin_multi_infinite_thresholds,
    pin_multi_cut_equals_brute,
    pin_accepted_pairs,
]
