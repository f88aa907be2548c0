"""MI355X-native atlas-based fiber bundle segmentation (dME + fast bundle discard).

The compute path lives in ``libseg.so`` (hand-written HIP kernels for gfx950
behind the C ABI of ``include/seg.h``); ``seg`` is its Python binding.
"""
from .seg import (  # noqa: F401
    Atlas,
    autotune,
    tune_clear,
    tune_load,
    tune_save,
    DENSE,
    MODES,
    PLAIN,
    PREFILTER_BF16,
    PREFILTER_BF16_ORIENTED,
    PREFILTER_FP16,
    PREFILTER_FP8,
    SegError,
    filter_pairs,
    header_functions,
    lib,
    query_stats,
    scratch_bytes,
    resample,
    segment,
    segment_noalloc,
    NOALLOC_MAX_CENTROIDS,
    segment_batch,
)
