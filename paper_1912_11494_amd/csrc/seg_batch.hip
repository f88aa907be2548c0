// Batched persistent launch (not built yet).
#include <hip/hip_runtime.h>

#include "seg_internal.hpp"

namespace seg {

int run_batch(int, int, const BatchAtlas*, int32_t, const float* const*, const int64_t*, int32_t,
              int32_t* const*, float* const*, BatchBuf&, PrefilterBuf&, hipStream_t) {
  return -2;
}

}  // namespace seg
