"""libseg.so loads, exports every function of include/seg.h, and rejects bad
arguments on the host before touching the GPU."""
import ctypes

import pytest

import paper_1912_11494_amd as P
from paper_1912_11494_amd import seg as S


def test_exports_every_header_function():
    L = P.lib()
    names = P.header_functions()
    assert len(names) >= 11
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert L.seg_version() == 1


def test_default_options():
    o = S.Options()
    P.lib().seg_default_options(ctypes.byref(o))
    assert (o.mode, o.validate, o.tile, o.collect_stats) == (S.PLAIN, 0, 0, 0)
    assert o.profile_events is None


def _call(n=10, m=5, nb=2, mode=S.PLAIN, fib=8, cen=16, bid=32, thr=48, lab=64, dist=80):
    o = S.Options(mode, 0, 0, 0, None)
    return P.lib().seg_segment(fib, n, cen, m, bid, thr, nb, lab, dist, ctypes.byref(o), None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-1), -1),
    (dict(m=-1), -1),
    (dict(nb=0), -1),
    (dict(m=1 << 24), -6),
    (dict(mode=9), -7),
    (dict(fib=None), -1),
    (dict(cen=None), -1),
    (dict(thr=None), -1),
    (dict(lab=None), -1),
    (dict(fib=10), -1),   # misaligned
])
def test_host_argument_errors(kw, code):
    assert _call(**kw) == code
    assert P.lib().seg_last_error().decode() != ""


def test_empty_subject_is_a_no_op():
    assert _call(n=0, fib=None, lab=None, dist=None) == 0


def test_filter_and_batch_host_errors():
    L = P.lib()
    cnt = ctypes.c_int64(7)
    assert L.seg_filter_pairs(8, 4, 16, 3, 32, 48, 1, 99, 64, 10, ctypes.byref(cnt), None) == -7
    assert L.seg_filter_pairs(8, -4, 16, 3, 32, 48, 1, 1, 64, 10, ctypes.byref(cnt), None) == -1
    o = S.Options(S.PLAIN, 0, 0, 0, None)
    assert L.seg_segment_batch(None, 1, None, None, 1, None, None, ctypes.byref(o), None) == -1
    h = ctypes.c_void_p()
    assert L.seg_atlas_create(16, -2, 32, 48, 1, None, ctypes.byref(h)) == -1
    assert L.seg_atlas_size(None) == -1
    L.seg_atlas_destroy(None)


def test_stats_without_call():
    st = S.Stats()
    assert P.lib().seg_query_stats(ctypes.byref(st)) == -1


def _noalloc(n=10, m=5, nb=2, mode=S.PLAIN, fib=8, cen=16, bid=32, thr=48, lab=64, dist=80):
    o = S.Options(mode, 0, 0, 0, None)
    return P.lib().seg_segment_noalloc(fib, n, cen, m, bid, thr, nb, lab, dist, ctypes.byref(o),
                                       None)


@pytest.mark.parametrize("kw,code", [
    (dict(mode=S.PREFILTER_FP16), -7),          # dense and plain only
    (dict(mode=S.PREFILTER_BF16_ORIENTED), -7),
    (dict(mode=9), -7),
    (dict(m=S.NOALLOC_MAX_CENTROIDS + 1), -6),  # beyond the fixed scratch
    (dict(m=1 << 24), -6),
    (dict(n=-1), -1),
    (dict(fib=None), -1),
    (dict(lab=13), -1),                         # misaligned output
])
def test_noalloc_host_argument_errors(kw, code):
    """The entry point that allocates nothing rejects, on the host, modes it
    does not run and atlases larger than its fixed scratch."""
    assert _noalloc(**kw) == code
    assert P.lib().seg_last_error().decode() != ""


def test_noalloc_empty_subject_is_a_no_op():
    assert _noalloc(n=0, fib=None, lab=None, dist=None) == 0
