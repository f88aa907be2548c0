"""Vectorised NumPy float64 brute force of the segmentation definition.

Test infrastructure only.  Written independently of ``seg_oracle.c`` (array
expressions instead of loops) so the two can pin each other on small inputs.

Eq. 1: point distance ||a_i - b_i||; Eq. 2: the maximum over the 21 point
pairs, in direct order and in inverse order (a_i with b_{20-i}), and the
smaller of the two.  A pair is accepted when d_ME does not exceed the
threshold of the centroid's bundle (section 2.3); each fiber takes the bundle
of its closest accepted centroid, lowest centroid index on ties (Algorithm 1
keeps the first one found).
"""
from __future__ import annotations

import numpy as np


def dme_matrix(fibers: np.ndarray, centroids: np.ndarray) -> np.ndarray:
    """d_ME in float64 for every (fiber, centroid) pair, shape [N, M]."""
    a = np.asarray(fibers, np.float32).astype(np.float64)  # [N,21,3]
    b = np.asarray(centroids, np.float32).astype(np.float64)  # [M,21,3]
    direct = np.sqrt(((a[:, None, :, :] - b[None, :, :, :]) ** 2).sum(-1)).max(-1)
    inverse = np.sqrt(((a[:, None, :, :] - b[None, :, ::-1, :]) ** 2).sum(-1)).max(-1)
    return np.minimum(direct, inverse)


def segment(fibers, centroids, bid, thr):
    """(labels int32, dists float64, best centroid int64) by brute force."""
    d = dme_matrix(fibers, centroids)
    thr = np.asarray(thr, np.float32).astype(np.float64)
    bid = np.asarray(bid, np.int64)
    t = thr[bid]  # per centroid
    ok = (t[None, :] >= 0) & (d <= t[None, :])
    dm = np.where(ok, d, np.inf)
    n = dm.shape[0]
    if dm.shape[1] == 0:
        return np.full(n, -1, np.int32), np.full(n, np.inf), np.full(n, -1, np.int64)
    best = np.argmin(dm, axis=1)  # first occurrence = lowest index
    has = ok[np.arange(n), best]
    labels = np.where(has, bid[best], -1).astype(np.int32)
    dists = np.where(has, dm[np.arange(n), best], np.inf)
    return labels, dists, np.where(has, best, -1)
