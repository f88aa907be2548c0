"""CPU oracle for fiber bundle segmentation (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does, and this package never
imports the GPU library: the two share no code.

``seg_oracle.c`` holds the float32 and float64 oracles (brute force over the
definition, and the paper's progressive discard); ``np_fp64`` is a separate
vectorised NumPy float64 brute force used to pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "seg_oracle.c")
LIB = os.path.join(HERE, "libseg_oracle.so")

BRUTE = 0
CUT = 1

# metric variants (flags of segment_ext_f32)
TN = 1    # length normalisation (Eq. 3)
DIR = 2   # direction inference (section 2.4)

# -ffp-contract=off: the float32 expression must be evaluated exactly as
# written (one explicit fmaf per step, nothing fused by the compiler).
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-std=c11", "-Wall"]


def compile_oracle(src: str, out: str) -> str:
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always recompiles when ``force``)."""
    if force or not os.path.exists(LIB):
        compile_oracle(SRC, LIB)
    return LIB


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int32
        L.oracle_segment_f32.argtypes = [P, i64, P, i64, P, P, i32, ctypes.c_int, ctypes.c_int,
                                         P, P, P]
        L.oracle_segment_f32.restype = ctypes.c_int
        L.oracle_segment_f64.argtypes = [P, i64, P, i64, P, P, i32, ctypes.c_int, P, P, P]
        L.oracle_segment_f64.restype = ctypes.c_int
        L.oracle_pair_f32.argtypes = [P, P, P, P]
        L.oracle_pair_f64.argtypes = [P, P, P, P]
        L.oracle_accepted_pairs_f32.argtypes = [P, i64, P, i64, P, P, i32, P, i64]
        L.oracle_accepted_pairs_f32.restype = ctypes.c_int64
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_segment_ext_f32.argtypes = [P, i64, P, i64, P, P, i32, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, P, P, P]
        L.oracle_segment_ext_f32.restype = ctypes.c_int
        L.oracle_arc_length_f32.argtypes = [P]
        L.oracle_arc_length_f32.restype = ctypes.c_float
        L.oracle_tn_f32.argtypes = [ctypes.c_float, ctypes.c_float]
        L.oracle_tn_f32.restype = ctypes.c_float
        L.oracle_segment_multi_f32.argtypes = [P, i64, P, i64, P, P, i32, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_int, P, P, P, i64, P]
        L.oracle_segment_multi_f32.restype = i64
        L.oracle_resample_f32.argtypes = [P, P, i64, i64, ctypes.c_int, P]
        L.oracle_resample_f32.restype = ctypes.c_int
        self.L = L
        self.path = path

    @staticmethod
    def _prep(fibers, centroids, bid, thr):
        f, pf = _c(fibers, np.float32)
        c, pc = _c(centroids, np.float32)
        b, pb = _c(bid, np.int32)
        t, pt = _c(thr, np.float32)
        if f.ndim != 3 or f.shape[1:] != (21, 3) or c.ndim != 3 or c.shape[1:] != (21, 3):
            raise ValueError("fibers and centroids must be [*, 21, 3]")
        if b.shape != (c.shape[0],):
            raise ValueError("one bundle id per centroid")
        return (f, c, b, t), pf, pc, pb, pt

    def segment_f32(self, fibers, centroids, bid, thr, mode: int = CUT, threads: int = 0):
        """float32 decision: (labels int32, dists float32, best centroid int32)."""
        keep, pf, pc, pb, pt = self._prep(fibers, centroids, bid, thr)
        f, c, b, t = keep
        n = f.shape[0]
        labels = np.empty(n, np.int32)
        dists = np.empty(n, np.float32)
        best = np.empty(n, np.int32)
        rc = self.L.oracle_segment_f32(pf, n, pc, c.shape[0], pb, pt, t.shape[0], mode, threads,
                                       labels.ctypes.data, dists.ctypes.data, best.ctypes.data)
        if rc:
            raise ValueError(f"oracle_segment_f32 failed ({rc})")
        return labels, dists, best

    def segment_ext_f32(self, fibers, centroids, bid, thr, flags: int, mode: int = CUT,
                        threads: int = 0):
        """float32 decision with metric variants (TN | DIR): (labels, dists, best)."""
        keep, pf, pc, pb, pt = self._prep(fibers, centroids, bid, thr)
        f, c, b, t = keep
        n = f.shape[0]
        labels = np.empty(n, np.int32)
        dists = np.empty(n, np.float32)
        best = np.empty(n, np.int32)
        rc = self.L.oracle_segment_ext_f32(pf, n, pc, c.shape[0], pb, pt, t.shape[0], mode, flags,
                                           threads, labels.ctypes.data, dists.ctypes.data,
                                           best.ctypes.data)
        if rc:
            raise ValueError(f"oracle_segment_ext_f32 failed ({rc})")
        return labels, dists, best

    def arc_length_f32(self, p) -> float:
        p, pp = _c(p, np.float32)
        return float(self.L.oracle_arc_length_f32(pp))

    def tn_f32(self, ls: float, lc: float) -> float:
        return float(self.L.oracle_tn_f32(ls, lc))

    def segment_multi_f32(self, fibers, centroids, bid, thr, flags: int = 0, mode: int = CUT,
                          threads: int = 0):
        """Every bundle each fiber passes: (offsets int64 [n + 1], bundles int32
        [total], dists float32 [total], bundle_counts int64 [nb]); fiber f's
        bundles (increasing) are bundles[offsets[f]:offsets[f + 1]]."""
        keep, pf, pc, pb, pt = self._prep(fibers, centroids, bid, thr)
        f, c, b, t = keep
        n = f.shape[0]
        offsets = np.zeros(n + 1, np.int64)
        counts = np.zeros(max(t.shape[0], 1), np.int64)
        total = self.L.oracle_segment_multi_f32(pf, n, pc, c.shape[0], pb, pt, t.shape[0], mode,
                                                flags, threads, offsets.ctypes.data, None, None,
                                                0, None)
        if total < 0:
            raise ValueError(f"oracle_segment_multi_f32 failed ({total})")
        bundles = np.zeros(max(total, 1), np.int32)
        dists = np.zeros(max(total, 1), np.float32)
        total2 = self.L.oracle_segment_multi_f32(pf, n, pc, c.shape[0], pb, pt, t.shape[0], mode,
                                                 flags, threads, offsets.ctypes.data,
                                                 bundles.ctypes.data, dists.ctypes.data, total,
                                                 counts.ctypes.data)
        assert total2 == total
        return offsets, bundles[:total], dists[:total], counts[:t.shape[0]]

    def resample_f32(self, points, offsets, threads: int = 0):
        """Raw streamlines (points [P, 3] float32, CSR offsets [n + 1] int64)
        to 21 points equidistant in arc length: float32 [n, 21, 3]."""
        p, pp = _c(points, np.float32)
        o, po = _c(offsets, np.int64)
        if p.ndim != 2 or p.shape[1] != 3 or o.ndim != 1 or o.shape[0] < 1:
            raise ValueError("points must be [P, 3] and offsets [n + 1]")
        n = o.shape[0] - 1
        out = np.empty((n, 21, 3), np.float32)
        rc = self.L.oracle_resample_f32(pp, po, n, p.shape[0], threads, out.ctypes.data)
        if rc:
            raise ValueError(f"oracle_resample_f32 failed ({rc})")
        return out

    def segment_f64(self, fibers, centroids, bid, thr, threads: int = 0):
        """float64 companion: (labels int32, dists float64, best centroid int32)."""
        keep, pf, pc, pb, pt = self._prep(fibers, centroids, bid, thr)
        f, c, b, t = keep
        n = f.shape[0]
        labels = np.empty(n, np.int32)
        dists = np.empty(n, np.float64)
        best = np.empty(n, np.int32)
        rc = self.L.oracle_segment_f64(pf, n, pc, c.shape[0], pb, pt, t.shape[0], threads,
                                       labels.ctypes.data, dists.ctypes.data, best.ctypes.data)
        if rc:
            raise ValueError(f"oracle_segment_f64 failed ({rc})")
        return labels, dists, best

    def pair_f32(self, a, b):
        """(max over direct order, max over inverse order) of float32 squared d_E."""
        a, pa = _c(a, np.float32)
        b, pb = _c(b, np.float32)
        d = np.zeros(2, np.float32)
        self.L.oracle_pair_f32(pa, pb, d.ctypes.data, d.ctypes.data + 4)
        return float(d[0]), float(d[1])

    def pair_f64(self, a, b):
        a, pa = _c(a, np.float32)
        b, pb = _c(b, np.float32)
        d = np.zeros(2, np.float64)
        self.L.oracle_pair_f64(pa, pb, d.ctypes.data, d.ctypes.data + 8)
        return float(d[0]), float(d[1])

    def accepted_pairs_f32(self, fibers, centroids, bid, thr, cap: int = 1 << 22):
        """All accepted pairs as an int64 array [K, 2] (fiber, centroid)."""
        keep, pf, pc, pb, pt = self._prep(fibers, centroids, bid, thr)
        f, c, b, t = keep
        out = np.empty((cap, 2), np.int64)
        k = self.L.oracle_accepted_pairs_f32(pf, f.shape[0], pc, c.shape[0], pb, pt, t.shape[0],
                                             out.ctypes.data, cap)
        if k < 0:
            raise ValueError(f"oracle_accepted_pairs_f32 failed ({k})")
        if k > cap:
            raise ValueError("accepted pair list exceeds capacity")
        return out[:k].copy()

    def max_threads(self) -> int:
        return int(self.L.oracle_max_threads())


_default: Optional[Oracle] = None


def get() -> Oracle:
    """The oracle built from ``seg_oracle.c`` (compiled on first use if absent)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build()
        _default = Oracle(LIB)
    return _default


def segment_f32(*a, **k):
    return get().segment_f32(*a, **k)


def segment_f64(*a, **k):
    return get().segment_f64(*a, **k)


def pair_f32(a, b):
    return get().pair_f32(a, b)


def pair_f64(a, b):
    return get().pair_f64(a, b)


def accepted_pairs_f32(*a, **k):
    return get().accepted_pairs_f32(*a, **k)


def segment_ext_f32(*a, **k):
    return get().segment_ext_f32(*a, **k)


def resample_f32(*a, **k):
    return get().resample_f32(*a, **k)


def segment_multi_f32(*a, **k):
    return get().segment_multi_f32(*a, **k)
