// MFMA prefilter modes (not built yet).
#include <hip/hip_runtime.h>

#include "seg_internal.hpp"

namespace seg {

int run_prefilter(int, int, const float*, int64_t, const float*, const float4*, int32_t,
                  const int32_t*, int32_t*, float*, unsigned long long*, PrefilterBuf&,
                  hipStream_t) {
  return -2;
}

int prefilter_pairs(int, const float*, int64_t, const float*, const float4*, int32_t, int32_t*,
                    int64_t, unsigned long long*, PrefilterBuf&, hipStream_t) {
  return -2;
}

}  // namespace seg
