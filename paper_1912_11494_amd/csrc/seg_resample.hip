// Resampling of raw streamlines to 21 points equidistant in arc length, the
// step before the comparison (section 2.3: subject fibers are resampled to 21
// equidistant points before classification; the atlas centroids carry 21
// equidistant points, section 2.2).
//
// Arithmetic (the contract of seg_resample in seg.h):
//   g_j = sqrtf(fma(dz, dz, fma(dy, dy, dx*dx))), d = p[j+1] - p[j];
//   q_j = g_j in units of 2^-24 mm, rounded to nearest even; 2^38 when
//         g_j >= 2^14 mm or g_j is not finite;
//   S_0 = 0, S_{j+1} = S_j + q_j, exact in 64 bits, L = S_{P-1};
//   t_k = floor(k L / 20) for k = 1..19;
//   point k lies on the first segment j with t_k <= S_{j+1}, at weight
//   w = fl(fl(t_k - S_j) / fl(q_j)) clamped to [0, 1] (0 for q_j = 0):
//   out = fma(w, d, p[j]); out_0 = p[0], out_20 = p[P-1].
// The sums are exact integers, so any order of summation gives them: one
// wave takes one streamline,
//   1. reads its points 64 segments at a time (four such chunks in flight),
//      computes q_j and an inclusive scan of each chunk across the wave
//      (DPP row shifts, then the row totals), adds the running total and
//      keeps S_{j+1} in the wave's LDS slice;
//   2. lanes 1..19 each find the segment of one target by walking the stored
//      sums from the guess of even spacing (the sums never decrease), read
//      that segment's two points (just read by the same wave) and
//      interpolate; lanes 0 and 20 copy the end points.
// A streamline with more segments than the LDS slice holds is done by one
// lane alone from global memory: a first pass finds L, a second walks the
// same sums again and emits each target as its segment comes by.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "seg_internal.hpp"

namespace seg {
namespace {

constexpr int64_t RS_MAXP = (int64_t)1 << 24;  // points per streamline at most
constexpr int RS_WAVES = 4;                     // waves (streamlines at a time) per block
constexpr int RS_CH = 10;                       // chunks of 64 segments kept per wave

// sqrtf(x) rounded to nearest for x >= 2^-96 (and +inf, NaN): the hardware
// square root (within one ulp) corrected by the sign of the residuals
// x - s- * s and x - s+ * s of its two neighbours, which decide on which side
// of the midpoints the exact root lies (x and the products are multiples of
// ulp(s)^2, so the residual is never strictly between 0 and the midpoint's
// ulp(s)^2 / 4 offset).  Below 2^-96 the result is below 2^-47, as is the
// rounded root: both give a fixed-point length of 0.
__device__ __forceinline__ float sqrt_rn_fixed(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sm = __uint_as_float(__float_as_uint(s) - 1u);
  const float sp = __uint_as_float(__float_as_uint(s) + 1u);
  const float rm = __builtin_fmaf(-sm, s, x), rp = __builtin_fmaf(-sp, s, x);
  float r = rm <= 0.0f ? sm : s;
  return rp > 0.0f ? sp : r;
}

// The fixed-point length as a float holding an integer (exact below 2^38):
// rint(g 2^24), or 2^38 for g >= 2^14 and NaN.
__device__ __forceinline__ float seg_fixed_f(float dx, float dy, float dz) {
  const float g = sqrt_rn_fixed(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
  return g < 16384.0f ? rintf(g * 16777216.0f) : 274877906944.0f;
}

// An integer-valued float in [0, 2^38] to 64 bits: the high word is
// trunc(r 2^-32), the low word r - high 2^32 (both steps exact).
__device__ __forceinline__ int64_t fixed_to_i64(float r) {
  const float hi = __builtin_truncf(r * 2.3283064365386963e-10f);
  const uint32_t lo = (uint32_t)__builtin_fmaf(hi, -4294967296.0f, r);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | lo);
}

// Length of the segment d in units of 2^-24 mm, 2^38 at or above 2^14 mm
// and for NaN / inf.
__device__ __forceinline__ int64_t seg_fixed(float dx, float dy, float dz) {
  return fixed_to_i64(seg_fixed_f(dx, dy, dz));
}

// floor(k L / 20) without forming k L.
__device__ __forceinline__ int64_t target(int64_t Lq, int64_t Lr, int k) {
  return Lq * k + (Lr * k) / 20;
}

__device__ __forceinline__ float weight(int64_t dt, int64_t q) {
  const float w = q > 0 ? (float)dt / (float)q : 0.0f;
  return w < 0.0f ? 0.0f : (w > 1.0f ? 1.0f : w);
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
  int64_t L = 0;
  {
    float px = x0, py = y0, pz = z0;
    for (int64_t j = 1; j < P; ++j) {
      const float qx = p[3 * j], qy = p[3 * j + 1], qz = p[3 * j + 2];
      L += seg_fixed(qx - px, qy - py, qz - pz);
      px = qx;
      py = qy;
      pz = qz;
    }
  }
  const int64_t Lq = L / 20, Lr = L % 20;
  put3(o, x0, y0, z0);
  int k = 1;
  int64_t t = target(Lq, Lr, k), s = 0;
  float px = x0, py = y0, pz = z0;
  for (int64_t j = 1; j < P && k < NP - 1; ++j) {
    const float qx = p[3 * j], qy = p[3 * j + 1], qz = p[3 * j + 2];
    const float dx = qx - px, dy = qy - py, dz = qz - pz;
    const int64_t q = seg_fixed(dx, dy, dz);
    const int64_t s1 = s + q;
    while (k < NP - 1 && t <= s1) {
      const float w = weight(t - s, q);
      put3(o + 3 * k, __builtin_fmaf(w, dx, px), __builtin_fmaf(w, dy, py),
           __builtin_fmaf(w, dz, pz));
      ++k;
      t = target(Lq, Lr, k);
    }
    s = s1;
    px = qx;
    py = qy;
    pz = qz;
  }
  for (; k < NP - 1; ++k) put3(o + 3 * k, xl, yl, zl);  // only without segments
  put3(o + 3 * (NP - 1), xl, yl, zl);
}

// x + (the value of the lane `ctrl` names, 0 where it names none or the
// lane's row is masked off), per 32-bit half.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int64_t dpp_add(int64_t x) {
  const int lo = (int)(uint32_t)x, hi = (int)(x >> 32);
  const uint32_t slo = (uint32_t)__builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
  const uint32_t shi = (uint32_t)__builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
  return x + (int64_t)(((uint64_t)shi << 32) | slo);
}

// x + (the value of the lane `ctrl` names, 0 where it names none or the
// lane's row is masked off).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_add32(uint32_t x) {
  return x + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}

// 32-bit form of wave_scan, for chunks whose sums stay below 2^32.
__device__ __forceinline__ uint32_t wave_scan32(uint32_t x) {
  x = dpp_add32<0x111, 0xf>(x);
  x = dpp_add32<0x112, 0xf>(x);
  x = dpp_add32<0x114, 0xf>(x);
  x = dpp_add32<0x118, 0xf>(x);
  x = dpp_add32<0x142, 0xa>(x);
  x = dpp_add32<0x143, 0xc>(x);
  return x;
}

// Inclusive scan across the 64 lanes (every lane active): a scan within each
// row of 16 lanes (row_shr 1, 2, 4, 8), then row 15's total into rows 1 and
// 3 (row_bcast:15) and lane 31's into rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ int64_t wave_scan(int64_t x) {
  x = dpp_add<0x111, 0xf>(x);
  x = dpp_add<0x112, 0xf>(x);
  x = dpp_add<0x114, 0xf>(x);
  x = dpp_add<0x118, 0xf>(x);
  x = dpp_add<0x142, 0xa>(x);
  x = dpp_add<0x143, 0xc>(x);
  return x;
}

__device__ __forceinline__ int64_t lane63(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), 63);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// LDS written by some lanes of a wave, then read by others of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One streamline [b, e) by the whole wave (all 64 lanes active): output i.
__device__ __forceinline__ void resample_wave(const float* __restrict__ pts, int64_t npts,
                                              int64_t b, int64_t e, float* __restrict__ o,
                                              unsigned int* __restrict__ flags,
                                              int64_t* __restrict__ S, int lane) {
  if (!(b >= 0 && e > b && e <= npts && e - b <= RS_MAXP)) {
    const float qnan = __int_as_float(0x7fc00000);
    if (lane < NP) put3(o + 3 * lane, qnan, qnan, qnan);
    if (lane == 0 && flags) atomicOr(flags, FLAG_OFFSETS);
    return;
  }
  const float* __restrict__ p = pts + 3 * b;
  const int64_t m = e - b - 1;  // segments
  if (m == 0) {
    if (lane < NP) put3(o + 3 * lane, p[0], p[1], p[2]);
    return;
  }
  if (m > (int64_t)RS_CH * 64) {
    if (lane == 0) resample_lane(p, m + 1, o);
    return;
  }
  const int mm = (int)m;
  const int nch = (mm + 63) >> 6;

  // 1. fixed-point lengths and their running sums, up to four chunks per round
  int64_t carry = 0;
  for (int c0 = 0; c0 < nch; c0 += 4) {
    float v[4][6];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c0 + u < nch) {
        const int j = (c0 + u) * 64 + lane;
        const float* __restrict__ q = p + 3 * (j < mm ? j : mm - 1);
#pragma unroll
        for (int c = 0; c < 6; ++c) v[u][c] = q[c];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c0 + u < nch) {
        const int j = (c0 + u) * 64 + lane;
        const float r =
            j < mm ? seg_fixed_f(v[u][3] - v[u][0], v[u][4] - v[u][1], v[u][5] - v[u][2]) : 0.0f;
        int64_t s1;
        if (__builtin_amdgcn_ballot_w64(r >= 67108864.0f) == 0) {
          // every length below 2^26 units: the chunk's sums fit 32 bits
          s1 = carry + (int64_t)wave_scan32((uint32_t)r);
        } else {
          s1 = carry + wave_scan(fixed_to_i64(r));
        }
        // always true here (nch <= RS_CH); with the test the compiler
        // schedules this loop markedly better (measured)
        if (c0 + u < RS_CH) S[(c0 + u) * 64 + lane] = s1;
        carry = lane63(s1);
      }
    }
  }
  const int64_t L = carry;
  wave_lds_sync();

  // 2. one target per lane
  if (lane < NP) {
    float x, y, z;
    if (lane == 0 || lane == NP - 1) {
      const float* __restrict__ q = lane == 0 ? p : p + 3 * mm;
      x = q[0];
      y = q[1];
      z = q[2];
    } else {
      const int64_t t = target(L / 20, L % 20, lane);
      // first j in [0, m) with t <= S_{j+1}; S_m = L >= t, so one exists
      int j = (lane * mm) / 20;
      if (t <= S[j]) {
        while (j > 0 && t <= S[j - 1]) --j;
      } else {
        ++j;
        while (j < mm && !(t <= S[j])) ++j;
        if (j >= mm) j = mm - 1;  // unreachable: keeps the reads in range
      }
      const int64_t sj = j == 0 ? 0 : S[j - 1];
      const float wgt = weight(t - sj, S[j] - sj);
      const float* __restrict__ a = p + 3 * j;
      const float ax = a[0], ay = a[1], az = a[2];
      x = __builtin_fmaf(wgt, a[3] - ax, ax);
      y = __builtin_fmaf(wgt, a[4] - ay, ay);
      z = __builtin_fmaf(wgt, a[5] - az, az);
    }
    put3(o + 3 * lane, x, y, z);
  }
  wave_lds_sync();  // the slice is rewritten by the next streamline
}

// Grid-stride over streamlines, one per wave at a time.
__global__ __launch_bounds__(64 * RS_WAVES) void resample_kernel(
    const float* __restrict__ pts, int64_t npts, const int64_t* __restrict__ off, int64_t n,
    float* __restrict__ out, unsigned int* __restrict__ flags) {
  __shared__ int64_t s_sum[RS_WAVES][RS_CH * 64];  // S_{j+1} at index j
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t i = (int64_t)blockIdx.x * RS_WAVES + w; i < n;
       i += (int64_t)gridDim.x * RS_WAVES)
    resample_wave(pts, npts, off[i], off[i + 1], out + i * (3 * NP), flags, s_sum[w], lane);
}

}  // namespace

int launch_resample(const float* pts, int64_t npts, const int64_t* off, int64_t n, float* out,
                    unsigned int* flags, hipStream_t s) {
  if (n <= 0) return 0;
  // four waves and 20 KB of LDS per block, eight blocks per CU; up to 65,536
  // blocks (32 per resident slot), each wave taking streamline after
  // streamline: faster than one streamline per wave or one resident grid
  const int64_t want = (n + RS_WAVES - 1) / RS_WAVES;
  const unsigned blocks = (unsigned)(want < 65536 ? want : 65536);
  resample_kernel<<<blocks, 64 * RS_WAVES, 0, s>>>(pts, npts, off, n, out, flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seg
