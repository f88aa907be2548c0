// Resampling of raw streamlines to 21 points equidistant in arc length, the
// step before the comparison (section 2.3: subject fibers are resampled to 21
// equidistant points before classification; the atlas centroids carry 21
// equidistant points, section 2.2).
//
// Arithmetic (float32, the contract of seg_resample in seg.h):
//   g_j = sqrtf(fma(dz, dz, fma(dy, dy, dx*dx))), d = p[j+1] - p[j];
//   s_0 = 0, s_{j+1} = s_j + g_j (in point order), L = s_{P-1};
//   t_k = (k * L) / 20 for k = 1..19;
//   point k lies on the first segment j with t_k <= s_{j+1}, at weight
//   w = (t_k - s_j) / g_j clamped to [0, 1] (0 for g_j = 0):
//   out = fma(w, d, p[j]); a target beyond the last sum takes the last point;
//   out_0 = p[0], out_20 = p[P-1].
// The cumulative sum is a sequential chain per streamline, so one lane owns
// one streamline: a first pass finds L, a second walks the same sums again and
// emits each target as its segment comes by.  Both passes evaluate the same
// expressions in the same order, so the second pass reproduces the first
// pass's sums bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "seg_internal.hpp"

namespace seg {
namespace {

constexpr int RS_BLOCK = 256;

__device__ __forceinline__ float seg_len(float dx, float dy, float dz) {
  return sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
}

__device__ __forceinline__ void put3(float* __restrict__ o, float x, float y, float z) {
  o[0] = x;
  o[1] = y;
  o[2] = z;
}

__global__ __launch_bounds__(RS_BLOCK) void resample_kernel(
    const float* __restrict__ pts, int64_t npts, const int64_t* __restrict__ off, int64_t n,
    float* __restrict__ out, unsigned int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * RS_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int64_t b = off[i], e = off[i + 1];
  float* __restrict__ o = out + i * (3 * NP);
  if (!(b >= 0 && e > b && e <= npts)) {
    // empty streamline or offsets outside the points: no read, NaN output
    const float qnan = __int_as_float(0x7fc00000);
    for (int k = 0; k < 3 * NP; ++k) o[k] = qnan;
    if (flags) atomicOr(flags, FLAG_OFFSETS);
    return;
  }
  const float* __restrict__ p = pts + 3 * b;
  const int64_t P = e - b;
  const float x0 = p[0], y0 = p[1], z0 = p[2];
  const float* __restrict__ pl = p + 3 * (P - 1);
  const float xl = pl[0], yl = pl[1], zl = pl[2];

  // pass 1: length L
  float s = 0.0f;
  {
    float px = x0, py = y0, pz = z0;
#pragma unroll 4
    for (int64_t j = 1; j < P; ++j) {
      const float qx = p[3 * j], qy = p[3 * j + 1], qz = p[3 * j + 2];
      s = s + seg_len(qx - px, qy - py, qz - pz);
      px = qx;
      py = qy;
      pz = qz;
    }
  }
  const float L = s;

  // pass 2: the same sums again; each target is emitted on its segment
  put3(o, x0, y0, z0);
  int k = 1;
  float t = ((float)k * L) / 20.0f;
  s = 0.0f;
  float px = x0, py = y0, pz = z0;
  for (int64_t j = 1; j < P && k < NP - 1; ++j) {
    const float qx = p[3 * j], qy = p[3 * j + 1], qz = p[3 * j + 2];
    const float dx = qx - px, dy = qy - py, dz = qz - pz;
    const float g = seg_len(dx, dy, dz);
    const float s1 = s + g;
    while (k < NP - 1 && t <= s1) {
      float w = g > 0.0f ? (t - s) / g : 0.0f;
      w = w < 0.0f ? 0.0f : (w > 1.0f ? 1.0f : w);
      put3(o + 3 * k, __builtin_fmaf(w, dx, px), __builtin_fmaf(w, dy, py),
           __builtin_fmaf(w, dz, pz));
      ++k;
      t = ((float)k * L) / 20.0f;
    }
    s = s1;
    px = qx;
    py = qy;
    pz = qz;
  }
  for (; k < NP - 1; ++k) put3(o + 3 * k, xl, yl, zl);
  put3(o + 3 * (NP - 1), xl, yl, zl);
}

}  // namespace

int launch_resample(const float* pts, int64_t npts, const int64_t* off, int64_t n, float* out,
                    unsigned int* flags, hipStream_t s) {
  if (n <= 0) return 0;
  const int64_t blocks = (n + RS_BLOCK - 1) / RS_BLOCK;
  resample_kernel<<<(unsigned)blocks, RS_BLOCK, 0, s>>>(pts, npts, off, n, out, flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seg
