"""Helpers for the GPU parity tests (run only on a machine with the GPU)."""
from __future__ import annotations

import numpy as np
import torch

import oracle


def dev():
    return torch.device("cuda:0")


def to_gpu(fib, cen, bid, thr):
    d = dev()
    return (torch.from_numpy(np.ascontiguousarray(fib, np.float32)).to(d),
            torch.from_numpy(np.ascontiguousarray(cen, np.float32)).to(d),
            torch.from_numpy(np.ascontiguousarray(bid, np.int32)).to(d),
            torch.from_numpy(np.ascontiguousarray(thr, np.float32)).to(d))


def run(seg, fib, cen, bid, thr, mode, tile=0, validate=False):
    f, c, b, t = to_gpu(fib, cen, bid, thr)
    lab, dist = seg.segment(f, c, b, t, mode=mode, tile=tile, validate=validate)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), dist.cpu().numpy()


def assert_parity(lab, dist, fib, cen, bid, thr, ctx="", o32=None, check_f64=True):
    """Labels bit-exact with the float32 oracle; distances bit-exact with it and
    within 1e-5 relative of the float64 oracle where the float64 labels agree."""
    if o32 is None:
        o32 = oracle.segment_f32(fib, cen, bid, thr, mode=oracle.CUT)
    l32, d32 = o32[0], o32[1]
    bad = np.nonzero(lab != l32)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} label differences, first {bad[:5]} " \
                          f"gpu {lab[bad[:5]]} oracle {l32[bad[:5]]}"
    same = (dist == d32) | (np.isinf(dist) & np.isinf(d32))
    badd = np.nonzero(~same)[0]
    assert badd.size == 0, f"{ctx}: {badd.size} distance differences, first {badd[:5]} " \
                           f"gpu {dist[badd[:5]]} oracle {d32[badd[:5]]}"
    if check_f64:
        l64, d64, _ = oracle.segment_f64(fib, cen, bid, thr)
        ok = (l64 == lab) & (lab >= 0)
        if ok.any():
            rel = np.abs(dist[ok].astype(np.float64) - d64[ok]) / np.maximum(d64[ok], 1e-30)
            assert rel.max() <= 1e-5, f"{ctx}: max relative distance error {rel.max()}"
        # fp32 and fp64 may legitimately disagree only at the boundary / ties
        assert (l64 != lab).mean() < 0.01, f"{ctx}: too many float32/float64 label differences"
