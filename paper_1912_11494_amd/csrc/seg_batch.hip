// Batched launch: many subjects against one or two prepared atlases.
//
// The per-pair path is chosen by the mode: the plain pass or an MFMA
// prefilter.  Either way the whole batch is one launch of the fused kernel
// over a flattened work list of (subject, atlas, fiber block) items, ordered
// costliest atlas first and dispatched by the hardware in that order,
// preceded by the few preparation kernels; the sequence is captured once per
// launch shape into a HIP graph that is replayed on the caller's stream.
#include <hip/hip_runtime.h>

#include "seg_internal.hpp"

namespace seg {

int run_batch(int mode, int cfg, const BatchAtlas* atlases, int32_t n_atlases,
              const float* const* fibers, const int64_t* n_fibers, int32_t n_subjects,
              int32_t* const* labels, float* const* dists, int mflags, BatchBuf& bb,
              PrefilterBuf& pb, hipStream_t s) {
  (void)pb;
  if (n_atlases == 0 || n_subjects == 0) return 0;
  if (mode == 1)
    return plain_batch(cfg, atlases, n_atlases, fibers, n_fibers, n_subjects, labels, dists,
                       mflags, bb, s);
  if (mode >= 2 && mode <= 5)
    return prefilter_batch(mode, cfg, atlases, n_atlases, fibers, n_fibers, n_subjects, labels,
                           dists, mflags, bb, s);
  return -2;  // the dense pass has no batched form
}

}  // namespace seg
