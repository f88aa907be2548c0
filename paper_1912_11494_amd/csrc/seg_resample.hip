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
// The cumulative sum is a sequential chain per streamline; everything else is
// parallel.  A block takes up to 16 consecutive streamlines, whose points are
// one contiguous range:
//   1. all threads read the range once, coalesced, and write the segment
//      lengths g_j to LDS;
//   2. one lane per streamline runs the chain s_{j+1} = s_j + g_j over LDS and
//      leaves s_{j+1} in place of g_j (the chains are spread over the block's
//      waves, so their SIMDs run them side by side);
//   3. one task per (streamline, output point) finds its segment by binary
//      search over the stored sums (they never decrease, so the first j with
//      t_k <= s_{j+1} is a lower bound) and interpolates from the two points,
//      which the block has just read (cache hits).
// The sums are the same float32 chain the definition runs, so the result is
// the same bit for bit.  A streamline whose points do not fit in the block's
// LDS window (a very long one) is done by one lane alone from global memory:
// a first pass finds L, a second walks the same sums again and emits each
// target as its segment comes by.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "seg_internal.hpp"

namespace seg {
namespace {


__device__ __forceinline__ float seg_len(float dx, float dy, float dz) {
  return sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
}

__device__ __forceinline__ void put3(float* __restrict__ o, float x, float y, float z) {
  o[0] = x;
  o[1] = y;
  o[2] = z;
}

// One streamline by one lane from global memory (two passes over its points).
__device__ void resample_lane(const float* __restrict__ p, int64_t P, float* __restrict__ o) {
  const float x0 = p[0], y0 = p[1], z0 = p[2];
  const float* __restrict__ pl = p + 3 * (P - 1);
  const float xl = pl[0], yl = pl[1], zl = pl[2];
  float s = 0.0f;
  {
    float px = x0, py = y0, pz = z0;
    for (int64_t j = 1; j < P; ++j) {
      const float qx = p[3 * j], qy = p[3 * j + 1], qz = p[3 * j + 2];
      s = s + seg_len(qx - px, qy - py, qz - pz);
      px = qx;
      py = qy;
      pz = qz;
    }
  }
  const float L = s;
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

enum : int { RS_BAD = 0, RS_LDS = 1, RS_GLOBAL = 2 };

// BLOCK threads take `per` (at most RS_S) streamlines and stage at most
// RS_CAP points.
template <int BLOCK, int RS_S, int RS_CAP>
__global__ __launch_bounds__(BLOCK) void resample_kernel(
    const float* __restrict__ pts, int64_t npts, const int64_t* __restrict__ off, int64_t n,
    int per, float* __restrict__ out, unsigned int* __restrict__ flags) {
  static_assert(RS_S <= BLOCK, "one chain lane per streamline");
  __shared__ float sarr[RS_CAP];  // g_j, then s_{j+1}, at index j - base
  __shared__ int64_t s_b[RS_S], s_e[RS_S];
  __shared__ float s_L[RS_S];
  __shared__ int s_kind[RS_S];
  __shared__ int64_t s_base, s_hi;
  const int tid = threadIdx.x;
  const int64_t first = (int64_t)blockIdx.x * per;
  const int cnt = (int)((n - first) < per ? (n - first) : per);

  if (tid == 0) {
    // the window [base, hi): from the first streamline's start, at most
    // RS_CAP points and never outside [0, npts] whatever the offsets hold
    int64_t base = off[first], hi = off[first + cnt];
    base = base < 0 ? 0 : (base > npts ? npts : base);
    hi = hi < base ? base : hi;
    hi = hi > npts ? npts : hi;
    hi = hi - base > RS_CAP ? base + RS_CAP : hi;
    s_base = base;
    s_hi = hi;
  }
  __syncthreads();
  const int64_t base = s_base, hi = s_hi;
  if (tid < cnt) {
    const int64_t b = off[first + tid], e = off[first + tid + 1];
    s_b[tid] = b;
    s_e[tid] = e;
    int kind = RS_BAD;
    if (b >= 0 && e > b && e <= npts) kind = (b >= base && e <= hi) ? RS_LDS : RS_GLOBAL;
    s_kind[tid] = kind;
    if (kind == RS_BAD && flags) atomicOr(flags, FLAG_OFFSETS);
  }
  // offsets that decrease somewhere can make two valid streamlines share
  // points (around an invalid one): then the block stages nothing and each
  // valid streamline takes the lane path, which shares no state
  if (__syncthreads_or(tid < cnt && s_kind[tid] == RS_BAD) && tid < cnt &&
      s_kind[tid] == RS_LDS)
    s_kind[tid] = RS_GLOBAL;

  __syncthreads();

  // 1. segment lengths of the window, coalesced; four points per thread and
  //    round, their loads issued together
  for (int64_t j0 = base + tid; j0 + 1 < hi; j0 += 4 * BLOCK) {
    float v[4][6];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + u * BLOCK;
      const float* __restrict__ q = pts + 3 * (j + 1 < hi ? j : j0);
#pragma unroll
      for (int c = 0; c < 6; ++c) v[u][c] = q[c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + u * BLOCK;
      if (j + 1 < hi)
        sarr[j - base] = seg_len(v[u][3] - v[u][0], v[u][4] - v[u][1], v[u][5] - v[u][2]);
    }
  }
  __syncthreads();

  // 2. the sequential chain of each staged streamline: streamline t on lane
  //    t / W of wave t % W (W waves), so the waves share the chains
  {
    const int t = (tid & 63) * (BLOCK / 64) + (tid >> 6);
    if (t < cnt && s_kind[t] == RS_LDS) {
      const int lo = (int)(s_b[t] - base), up = (int)(s_e[t] - base) - 1;
      float sum = 0.0f;
      int j = lo;
      for (; j + 8 <= up; j += 8) {  // eight reads in flight, then the chain
        float g[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) g[u] = sarr[j + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          sum = sum + g[u];
          sarr[j + u] = sum;
        }
      }
      for (; j < up; ++j) {
        sum = sum + sarr[j];
        sarr[j] = sum;
      }
      s_L[t] = sum;
    }
  }
  __syncthreads();

  // 3. one task per (streamline, output point)
  for (int task = tid; task < cnt * NP; task += BLOCK) {
    const int t = task / NP, k = task - t * NP;
    const int kind = s_kind[t];
    const int64_t b = s_b[t], e = s_e[t];
    float* __restrict__ o = out + (first + t) * (3 * NP);
    if (kind == RS_BAD) {
      const float qnan = __int_as_float(0x7fc00000);
      put3(o + 3 * k, qnan, qnan, qnan);
      continue;
    }
    if (kind == RS_GLOBAL) {
      if (k == 0) resample_lane(pts + 3 * b, e - b, o);
      continue;
    }
    const int64_t P = e - b;
    const float* __restrict__ p = pts + 3 * b;
    int64_t j = P - 1;  // segment index; P - 1 means none (the last point)
    if (k > 0 && k < NP - 1) {
      const float tk = ((float)k * s_L[t]) / 20.0f;
      // first j in [0, P-1) with tk <= s_{j+1}: the sums never decrease, so
      // walk from the guess of even spacing, j = k (P - 1) / 20, to where the
      // test changes (a step or two on streamlines with even steps; at most
      // P - 1 steps whatever the spacing)
      const float* __restrict__ sj1 = sarr + (b - base);
      const int m = (int)(P - 1);
      int jj = (int)(((int64_t)k * m) / 20);
      if (jj >= m) jj = m - 1;
      if (m == 0 || tk != tk) {
        jj = m;  // one point, or NaN: no segment qualifies
      } else if (tk <= sj1[jj]) {
        while (jj > 0 && tk <= sj1[jj - 1]) --jj;
      } else {
        ++jj;
        while (jj < m && !(tk <= sj1[jj])) ++jj;
      }
      j = jj;
      if (j < P - 1) {
        const float ax = p[3 * j], ay = p[3 * j + 1], az = p[3 * j + 2];
        const float dx = p[3 * j + 3] - ax, dy = p[3 * j + 4] - ay, dz = p[3 * j + 5] - az;
        const float g = seg_len(dx, dy, dz);
        const float sj = j == 0 ? 0.0f : sj1[j - 1];
        float w = g > 0.0f ? (tk - sj) / g : 0.0f;
        w = w < 0.0f ? 0.0f : (w > 1.0f ? 1.0f : w);
        put3(o + 3 * k, __builtin_fmaf(w, dx, ax), __builtin_fmaf(w, dy, ay),
             __builtin_fmaf(w, dz, az));
        continue;
      }
    }
    const float* __restrict__ q = k == 0 ? p : p + 3 * (P - 1);
    put3(o + 3 * k, q[0], q[1], q[2]);
  }
}

}  // namespace

int launch_resample(const float* pts, int64_t npts, const int64_t* off, int64_t n, float* out,
                    unsigned int* flags, hipStream_t s) {
  if (n <= 0) return 0;
  // two waves, up to 16 streamlines and 5,120 staged points (20 KB) per
  // block, eight blocks per CU; fewer streamlines per block when the average
  // streamline is long, so a block's points usually fit its window
  constexpr int BLOCK = 128, SMAX = 16, CAP = 5120;
  const double avg = (double)npts / (double)n;
  int per = avg > 0.0 ? (int)(0.8 * CAP / avg) : SMAX;
  per = per < 1 ? 1 : (per > SMAX ? SMAX : per);
  const int64_t blocks = (n + per - 1) / per;
  if (blocks > 0x7fffffffLL) return -1;
  resample_kernel<BLOCK, SMAX, CAP><<<(unsigned)blocks, BLOCK, 0, s>>>(pts, npts, off, n, per, out,
                                                                      flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seg
