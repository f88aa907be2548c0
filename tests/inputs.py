"""Full-size synthetic inputs of the GPU tests, drawn once per session.

The fiber generator draws large subjects in a pool of forked worker
processes.  A fork copies the parent's state, GPU state included, so the
inputs a GPU test module declares (``@pytest.mark.workloads(...)``) are drawn
by ``conftest.py`` right after collection, before any test touches the GPU,
and kept here for the session.  A test run without that pass (a single test
named on the command line still gets it) draws its inputs on first use; the
generator then works without a pool once the GPU is initialised.
"""
from __future__ import annotations

import os
import time

import synth

_CACHE = {}


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def fibers(wl: str, subject_idx: int = 0):
    """Fibers of subject ``subject_idx`` of workload ``wl`` (float32 [n, 21, 3])."""
    key = (wl, subject_idx)
    if key not in _CACHE:
        atl = synth.workload_atlases(wl)
        subj = synth.workload_subjects(wl)[subject_idx]
        _CACHE[key] = synth.make_fibers(atl, subj, synth.workload_seed(wl),
                                        subject_idx=subject_idx, workers=_workers())
    return _CACHE[key]


def pregenerate(names, log=print) -> None:
    """Draw every subject of each named workload (call before GPU use)."""
    for wl in names:
        t0 = time.time()
        subs = synth.workload_subjects(wl)
        for i in range(len(subs)):
            fibers(wl, i)
        log(f"inputs: {wl} drawn ({sum(s.n_fibers for s in subs):,} fibers, "
            f"{time.time() - t0:.1f} s)")
