"""Python binding of libseg.so (argument marshalling only).

Every step of the segmentation runs in the library's HIP kernels; this module
passes device pointers, sizes and the current HIP stream through ctypes and
raises when the library reports an error.  PyTorch is used only to own device
memory and to name the stream.  There is no CPU fallback: if the library is
missing, or a tensor is not on the GPU, the call fails.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import List, Optional, Sequence, Tuple

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libseg.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "seg.h")

# seg_mode
DENSE = 0
PLAIN = 1
PREFILTER_BF16 = 2
PREFILTER_FP16 = 3
PREFILTER_FP8 = 4
PREFILTER_BF16_ORIENTED = 5

MODES = {
    "dense": DENSE,
    "plain": PLAIN,
    "bf16": PREFILTER_BF16,
    "fp16": PREFILTER_FP16,
    "fp8": PREFILTER_FP8,
    "bf16_oriented": PREFILTER_BF16_ORIENTED,
}

NOALLOC_MAX_CENTROIDS = 32768  # SEG_NOALLOC_MAX_CENTROIDS

STATUS = {0: "SEG_OK", -1: "SEG_EINVAL", -2: "SEG_EBUNDLE", -3: "SEG_ENONFINITE",
          -4: "SEG_EHIP", -5: "SEG_ENOMEM", -6: "SEG_ERANGE", -7: "SEG_EMODE",
          -8: "SEG_EOFFSETS", -9: "SEG_ECAPACITY"}


class SegError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("collect_stats", ctypes.c_int32),
                ("profile_events", ctypes.c_void_p), ("metric", ctypes.c_int32)]


# seg_metric flags (include/seg.h)
METRIC_LENGTH_NORM = 1
METRIC_DIRECTION = 2
METRICS = {"": 0, "tn": METRIC_LENGTH_NORM, "dir": METRIC_DIRECTION,
           "tn+dir": METRIC_LENGTH_NORM | METRIC_DIRECTION}


class Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("pairs", "filter_pass", "test2_pass", "test3_pass", "accepted", "labelled",
                 "drains", "bound_pairs", "survivor_rows")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libseg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1912_11494_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int32
        L.seg_segment.argtypes = [P, i64, P, i64, P, P, i32, P, P, ctypes.POINTER(Options), P]
        L.seg_segment.restype = ctypes.c_int
        L.seg_segment_noalloc.argtypes = [P, i64, P, i64, P, P, i32, P, P,
                                          ctypes.POINTER(Options), P]
        L.seg_segment_noalloc.restype = ctypes.c_int
        L.seg_default_options.argtypes = [ctypes.POINTER(Options)]
        L.seg_scratch_bytes.argtypes = [P]
        L.seg_scratch_bytes.restype = i64
        L.seg_last_error.restype = ctypes.c_char_p
        L.seg_version.restype = ctypes.c_int
        L.seg_atlas_create.argtypes = [P, i64, P, P, i32, P, ctypes.POINTER(P)]
        L.seg_atlas_create.restype = ctypes.c_int
        L.seg_atlas_destroy.argtypes = [P]
        L.seg_atlas_size.argtypes = [P]
        L.seg_atlas_size.restype = i64
        L.seg_segment_atlas.argtypes = [P, P, i64, P, P, ctypes.POINTER(Options), P]
        L.seg_segment_atlas.restype = ctypes.c_int
        L.seg_segment_batch.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(P),
                                        ctypes.POINTER(i64), i32, ctypes.POINTER(P),
                                        ctypes.POINTER(P), ctypes.POINTER(Options), P]
        L.seg_segment_batch.restype = ctypes.c_int
        L.seg_filter_pairs.argtypes = [P, i64, P, i64, P, P, i32, i32, P, i64,
                                       ctypes.POINTER(i64), P]
        L.seg_filter_pairs.restype = ctypes.c_int
        L.seg_query_stats.argtypes = [ctypes.POINTER(Stats)]
        L.seg_query_stats.restype = ctypes.c_int
        L.seg_autotune.argtypes = [P, P, i64, i32, i32, ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_float), P]
        L.seg_autotune.restype = ctypes.c_int
        L.seg_tune_save.argtypes = [ctypes.c_char_p]
        L.seg_tune_save.restype = ctypes.c_int
        L.seg_tune_load.argtypes = [ctypes.c_char_p]
        L.seg_tune_load.restype = ctypes.c_int
        L.seg_segment_multi.argtypes = [P, P, i64, i32, P, P, P, i64, ctypes.POINTER(i64), P,
                                        ctypes.POINTER(Options), P]
        L.seg_segment_multi.restype = ctypes.c_int
        L.seg_resample.argtypes = [P, i64, P, i64, P, i32, P]
        L.seg_resample.restype = ctypes.c_int
        L.seg_segment_streamlines.argtypes = [P, P, i64, P, i64, P, P, P,
                                              ctypes.POINTER(Options), P]
        L.seg_segment_streamlines.restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions() -> List[str]:
    """Names of the functions declared in include/seg.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(seg_[a-z_]+)\s*\(", txt)))


def _check(rc: int):
    if rc != 0:
        raise SegError(rc, lib().seg_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: torch.Tensor, dtype, shape_tail=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != shape_tail:
        raise ValueError(f"{name} must have shape [*, {', '.join(map(str, shape_tail))}]")
    return t


def _mode(mode) -> int:
    if isinstance(mode, str):
        if mode not in MODES:
            raise ValueError(f"unknown mode {mode!r}; one of {sorted(MODES)}")
        return MODES[mode]
    return int(mode)


def _metric(metric) -> int:
    if isinstance(metric, str):
        if metric not in METRICS:
            raise ValueError(f"unknown metric {metric!r}; one of {sorted(METRICS)}")
        return METRICS[metric]
    return int(metric)


def options(mode="plain", validate=False, tile=0, stats=False, events=None,
            metric=0) -> Options:
    """seg_options; `events` is an optional address of two hipEvent_t; `metric`
    is 0, an OR of METRIC_* flags, or one of "tn", "dir", "tn+dir"."""
    return Options(_mode(mode), int(bool(validate)), int(tile), int(bool(stats)), events,
                   _metric(metric))


def segment(fibers: torch.Tensor, centroids: torch.Tensor, centroid_bundle_id: torch.Tensor,
            bundle_thresholds: torch.Tensor, mode="plain", validate=False, tile=0, stats=False,
            out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, stream=None,
            events=None, metric=0) -> Tuple[torch.Tensor, torch.Tensor]:
    """labels (int32 [N]) and dists (float32 [N]) of each fiber; see include/seg.h."""
    _dev(fibers, torch.float32, (21, 3), "fibers")
    _dev(centroids, torch.float32, (21, 3), "centroids")
    _dev(centroid_bundle_id, torch.int32, None, "centroid_bundle_id")
    _dev(bundle_thresholds, torch.float32, None, "bundle_thresholds")
    n = fibers.shape[0]
    if out is None:
        labels = torch.empty(n, dtype=torch.int32, device=fibers.device)
        dists = torch.empty(n, dtype=torch.float32, device=fibers.device)
    else:
        labels, dists = out
        _dev(labels, torch.int32, None, "labels")
        _dev(dists, torch.float32, None, "dists")
    opt = options(mode, validate, tile, stats, events, metric)
    rc = lib().seg_segment(fibers.data_ptr(), n, centroids.data_ptr(), centroids.shape[0],
                           centroid_bundle_id.data_ptr(), bundle_thresholds.data_ptr(),
                           bundle_thresholds.shape[0], labels.data_ptr(), dists.data_ptr(),
                           ctypes.byref(opt), _stream(stream))
    _check(rc)
    return labels, dists


def segment_noalloc(fibers: torch.Tensor, centroids: torch.Tensor,
                    centroid_bundle_id: torch.Tensor, bundle_thresholds: torch.Tensor,
                    out: Tuple[torch.Tensor, torch.Tensor], mode="plain", validate=False, tile=0,
                    stats=False, stream=None, events=None, metric=0) -> Tuple[torch.Tensor,
                                                                              torch.Tensor]:
    """seg_segment_noalloc: `segment` with caller-owned outputs and library
    scratch in a fixed device array (dense and plain modes, at most
    NOALLOC_MAX_CENTROIDS centroids); see include/seg.h."""
    _dev(fibers, torch.float32, (21, 3), "fibers")
    _dev(centroids, torch.float32, (21, 3), "centroids")
    _dev(centroid_bundle_id, torch.int32, None, "centroid_bundle_id")
    _dev(bundle_thresholds, torch.float32, None, "bundle_thresholds")
    labels, dists = out
    _dev(labels, torch.int32, None, "labels")
    _dev(dists, torch.float32, None, "dists")
    n = fibers.shape[0]
    if labels.shape[0] < n or dists.shape[0] < n:
        raise ValueError("outputs must hold one entry per fiber")
    opt = options(mode, validate, tile, stats, events, metric)
    rc = lib().seg_segment_noalloc(fibers.data_ptr(), n, centroids.data_ptr(),
                                   centroids.shape[0], centroid_bundle_id.data_ptr(),
                                   bundle_thresholds.data_ptr(), bundle_thresholds.shape[0],
                                   labels.data_ptr(), dists.data_ptr(), ctypes.byref(opt),
                                   _stream(stream))
    _check(rc)
    return labels, dists


def scratch_bytes(stream=None) -> int:
    """Device bytes of library scratch held for the current device and stream."""
    return int(lib().seg_scratch_bytes(_stream(stream)))


def query_stats() -> dict:
    st = Stats()
    _check(lib().seg_query_stats(ctypes.byref(st)))
    return st.as_dict()


def filter_pairs(fibers, centroids, centroid_bundle_id, bundle_thresholds, mode="plain",
                 capacity: int = 1 << 20, stream=None) -> torch.Tensor:
    """Survivors of the first cut of `mode` as an int32 [K, 2] (fiber, centroid) tensor."""
    _dev(fibers, torch.float32, (21, 3), "fibers")
    _dev(centroids, torch.float32, (21, 3), "centroids")
    pairs = torch.empty((capacity, 2), dtype=torch.int32, device=fibers.device)
    cnt = ctypes.c_int64(0)
    rc = lib().seg_filter_pairs(fibers.data_ptr(), fibers.shape[0], centroids.data_ptr(),
                                centroids.shape[0], centroid_bundle_id.data_ptr(),
                                bundle_thresholds.data_ptr(), bundle_thresholds.shape[0],
                                _mode(mode), pairs.data_ptr(), capacity, ctypes.byref(cnt),
                                _stream(stream))
    _check(rc)
    if cnt.value > capacity:
        raise SegError(-5, f"{cnt.value} survivors exceed capacity {capacity}")
    return pairs[:cnt.value]


def _streamlines(points, offsets):
    _dev(points, torch.float32, (3,), "points")
    _dev(offsets, torch.int64, None, "offsets")
    if offsets.dim() != 1 or offsets.shape[0] < 1:
        raise ValueError("offsets must be [n + 1]")
    return offsets.shape[0] - 1


def resample(points: torch.Tensor, offsets: torch.Tensor, out: Optional[torch.Tensor] = None,
             validate=False, stream=None) -> torch.Tensor:
    """Raw streamlines (points float32 [P, 3], CSR offsets int64 [n + 1]) to
    21 points equidistant in arc length, float32 [n, 21, 3]; see include/seg.h."""
    n = _streamlines(points, offsets)
    if out is None:
        out = torch.empty((n, 21, 3), dtype=torch.float32, device=points.device)
    _dev(out, torch.float32, (21, 3), "out")
    rc = lib().seg_resample(points.data_ptr(), points.shape[0], offsets.data_ptr(), n,
                            out.data_ptr(), int(bool(validate)), _stream(stream))
    _check(rc)
    return out


class Atlas:
    """A prepared atlas held by the library (seg_atlas_create / seg_atlas_destroy)."""

    def __init__(self, centroids, centroid_bundle_id, bundle_thresholds, stream=None):
        _dev(centroids, torch.float32, (21, 3), "centroids")
        _dev(centroid_bundle_id, torch.int32, None, "centroid_bundle_id")
        _dev(bundle_thresholds, torch.float32, None, "bundle_thresholds")
        h = ctypes.c_void_p()
        rc = lib().seg_atlas_create(centroids.data_ptr(), centroids.shape[0],
                                    centroid_bundle_id.data_ptr(), bundle_thresholds.data_ptr(),
                                    bundle_thresholds.shape[0], _stream(stream), ctypes.byref(h))
        _check(rc)
        self.handle = h
        self.device = centroids.device
        self.n_bundles = int(bundle_thresholds.shape[0])

    def __len__(self):
        return int(lib().seg_atlas_size(self.handle))

    def close(self):
        if self.handle:
            lib().seg_atlas_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def segment(self, fibers, mode="plain", validate=False, tile=0, stats=False, stream=None,
                events=None, out=None, metric=0):
        _dev(fibers, torch.float32, (21, 3), "fibers")
        n = fibers.shape[0]
        if out is None:
            labels = torch.empty(n, dtype=torch.int32, device=fibers.device)
            dists = torch.empty(n, dtype=torch.float32, device=fibers.device)
        else:
            labels, dists = out
        opt = options(mode, validate, tile, stats, events, metric)
        rc = lib().seg_segment_atlas(self.handle, fibers.data_ptr(), n, labels.data_ptr(),
                                     dists.data_ptr(), ctypes.byref(opt), _stream(stream))
        _check(rc)
        return labels, dists

    def segment_multi(self, fibers, max_per_fiber=8, capacity=None, mode="fp16", validate=False,
                      tile=0, stats=False, stream=None, events=None, metric=0):
        """Every bundle each fiber passes (see seg_segment_multi): (offsets int64
        [n + 1], bundles int32 [total], dists float32 [total], bundle_counts
        int64 [n_bundles]).  Without `capacity`, a second call is made with the
        exact capacity when the first guess (2 per fiber) is too small."""
        _dev(fibers, torch.float32, (21, 3), "fibers")
        n = fibers.shape[0]
        dev = fibers.device
        nb = self.n_bundles
        offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
        counts = torch.empty(max(nb, 1), dtype=torch.int64, device=dev)
        opt = options(mode, validate, tile, stats, events, metric)
        cap = 2 * n if capacity is None else int(capacity)
        for attempt in range(2):
            bundles = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            dists = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
            total = ctypes.c_int64(0)
            rc = lib().seg_segment_multi(self.handle, fibers.data_ptr(), n, int(max_per_fiber),
                                         offsets.data_ptr(), bundles.data_ptr(), dists.data_ptr(),
                                         cap, ctypes.byref(total), counts.data_ptr(),
                                         ctypes.byref(opt), _stream(stream))
            if rc == -9 and capacity is None and attempt == 0:
                cap = int(total.value)
                continue
            _check(rc)
            break
        t = int(total.value)
        return offsets, bundles[:t], dists[:t], counts[:nb]

    def segment_streamlines(self, points, offsets, mode="plain", validate=False, tile=0,
                            stats=False, stream=None, fibers=None, out=None, metric=0):
        """Raw streamlines to (labels, dists, resampled fibers) in one library call."""
        n = _streamlines(points, offsets)
        dev = points.device
        if fibers is None:
            fibers = torch.empty((n, 21, 3), dtype=torch.float32, device=dev)
        _dev(fibers, torch.float32, (21, 3), "fibers")
        if out is None:
            labels = torch.empty(n, dtype=torch.int32, device=dev)
            dists = torch.empty(n, dtype=torch.float32, device=dev)
        else:
            labels, dists = out
        opt = options(mode, validate, tile, stats, None, metric)
        rc = lib().seg_segment_streamlines(self.handle, points.data_ptr(), points.shape[0],
                                           offsets.data_ptr(), n, fibers.data_ptr(),
                                           labels.data_ptr(), dists.data_ptr(), ctypes.byref(opt),
                                           _stream(stream))
        _check(rc)
        return labels, dists, fibers


def segment_batch(atlases: Sequence[Atlas], subjects: Sequence[torch.Tensor], mode="bf16",
                  tile=0, outs=None, stream=None, metric=0):
    """Labels/dists of every (subject, atlas) pair: a list over subjects of lists over atlases."""
    na, ns = len(atlases), len(subjects)
    for f in subjects:
        _dev(f, torch.float32, (21, 3), "fibers")
    if outs is None:
        outs = [[(torch.empty(f.shape[0], dtype=torch.int32, device=f.device),
                  torch.empty(f.shape[0], dtype=torch.float32, device=f.device))
                 for _ in range(na)] for f in subjects]
    P = ctypes.c_void_p
    ah = (P * max(na, 1))(*[a.handle.value for a in atlases])
    fp = (P * max(ns, 1))(*[f.data_ptr() for f in subjects])
    nf = (ctypes.c_int64 * max(ns, 1))(*[f.shape[0] for f in subjects])
    lp = (P * max(ns * na, 1))(*[outs[s][a][0].data_ptr() for s in range(ns) for a in range(na)])
    dp = (P * max(ns * na, 1))(*[outs[s][a][1].data_ptr() for s in range(ns) for a in range(na)])
    opt = options(mode, False, tile, False, None, metric)
    rc = lib().seg_segment_batch(ah, na, fp, nf, ns, lp, dp, ctypes.byref(opt), _stream(stream))
    _check(rc)
    return outs


def autotune(atlas: "Atlas", fibers: torch.Tensor, mode="bf16", reps: int = 3, stream=None):
    """Time every kernel configuration of `mode` on these inputs and remember
    the fastest for later calls with tile=0; returns (tile, ms)."""
    _dev(fibers, torch.float32, (21, 3), "fibers")
    best = ctypes.c_int32(0)
    ms = ctypes.c_float(0.0)
    rc = lib().seg_autotune(atlas.handle, fibers.data_ptr(), fibers.shape[0], _mode(mode), reps,
                            ctypes.byref(best), ctypes.byref(ms), _stream(stream))
    _check(rc)
    return int(best.value), float(ms.value)


def tune_save(path: str):
    _check(lib().seg_tune_save(path.encode()))


def tune_load(path: str):
    _check(lib().seg_tune_load(path.encode()))


def tune_clear():
    lib().seg_tune_clear()
