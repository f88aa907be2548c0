"""Seeded synthetic inputs for fiber-bundle segmentation.

This package only draws inputs (atlas centroids, bundle thresholds and subject
fibers).  It holds none of the segmentation arithmetic, so the CPU oracle and
the GPU library can both be fed from it without sharing any of the method.
"""
from .fibers import (  # noqa: F401
    AtlasSpec,
    SubjectSpec,
    Atlas,
    WORKLOADS,
    bezier_curves,
    make_atlas,
    gpu_in_use,
    make_fibers,
    raw_streamlines,
    raw_streamlines_torch,
    workload_atlases,
    workload_subjects,
    workload_seed,
    small_case,
)
