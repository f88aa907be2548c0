// Device-side building blocks shared by the segmentation kernels.
//
// Notation follows the paper (section 2.3): a fiber a and a centroid b have
// 21 points; the direct order pairs a_i with b_i, the inverse order pairs a_i
// with b_{20-i} (Eq. 2).  Everything is evaluated on squared distances and
// squared thresholds (T2 = T * T in float32).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace seg {

constexpr int NP = 21;       // points per curve
constexpr int NF = 3 * NP;   // floats per curve
constexpr int CTR = 10;      // center point, pairs with itself in both orders
constexpr int CREC = 64;     // floats per prepared centroid: 63 coordinates + T2
constexpr uint64_t NO_KEY = ~0ull;

// Squared point distance (Eq. 1 squared).  This is the one float32 expression
// of the library: three rounded differences, one rounded product, two fused
// multiply-adds.  Compiled with -ffp-contract=off so nothing else is fused.
__device__ __forceinline__ float d2(float ax, float ay, float az, float bx, float by, float bz) {
  float dx = ax - bx;
  float dy = ay - by;
  float dz = az - bz;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// Squared bundle threshold; -1 makes every comparison d2 <= T2 false.
__device__ __forceinline__ float thr2(float t) { return t >= 0.0f ? t * t : -1.0f; }

// Metric variants.  MF_TN: length normalisation (Eq. 3) -- an accepted pair
// (D <= T2) is kept when d_ME + TN <= T, and fibers take the bundle of the
// smallest d_ME + TN, which is also the reported distance.  MF_DIR: direction
// inference (section 2.4) -- the order with the smaller largest end-point
// distance (direct on ties) is the fiber's direction and D is the largest
// point distance of that order alone.
constexpr int MF_TN = 1;
constexpr int MF_DIR = 2;
struct Metric {
  const float* cext;  // per prepared centroid: arc length, threshold T
  int32_t flags;
};

// Arc length of a 21-point polyline: segment lengths
// sqrtf(fma(dz, dz, fma(dy, dy, dx * dx))) of p[i+1] - p[i], summed in order.
__device__ __forceinline__ float arc_length(const float* __restrict__ p) {
  float l = 0.0f;
#pragma unroll
  for (int i = 0; i + 1 < NP; ++i) {
    const float dx = p[3 * (i + 1)] - p[3 * i];
    const float dy = p[3 * (i + 1) + 1] - p[3 * i + 1];
    const float dz = p[3 * (i + 1) + 2] - p[3 * i + 2];
    l = l + sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
  }
  return l;
}

// TN of Eq. 3: (|lS - lC| / max(lS, lC) + 1)^2 - 1, each step rounded; 0 when
// both lengths are 0.
__device__ __forceinline__ float tn_term(float ls, float lc) {
  const float mx = ls > lc ? ls : lc;
  if (!(mx > 0.0f)) return 0.0f;
  const float r = fabsf(ls - lc) / mx;
  const float u = r + 1.0f;
  const float uu = u * u;
  return uu - 1.0f;
}

// Several labels per fiber: K slots per fiber, each 0 (empty) or
// (bundle + 1) << 32 | bits of the smallest value seen for that bundle (the
// values are non-negative floats, so their bits order like the values).  A
// fiber's slots only go from empty to a bundle and then down in value, so a
// stale read is never wrong for long: a failed compare-and-swap returns the
// current word.  A bundle that finds no free slot sets `flag`.
constexpr unsigned int FLAG_MULTI = 8u;

struct MultiOut {
  unsigned long long* slots;  // [n][K] in input fiber order
  int32_t K;
  const int32_t* bid;         // bundle of each prepared centroid
  unsigned int* flag;
};

__device__ __forceinline__ void multi_insert(unsigned long long* __restrict__ row, int K,
                                             uint32_t bundle, float v,
                                             unsigned int* __restrict__ flag) {
  const unsigned long long tag = (unsigned long long)(bundle + 1u);
  const unsigned long long e = (tag << 32) | (unsigned long long)__float_as_uint(v);
  for (int k = 0; k < K; ++k) {
    unsigned long long cur = __hip_atomic_load(row + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == 0ull) {
      cur = atomicCAS(row + k, 0ull, e);
      if (cur == 0ull) return;  // a new bundle of this fiber
    }
    if ((cur >> 32) == tag) {
      atomicMin(row + k, e);
      return;
    }
  }
  atomicOr(flag, FLAG_MULTI);
}

// Value the argmin compares for an accepted pair (D <= T2): D itself, or with
// MF_TN the complete metric sqrtf(D) + TN, which must not exceed T (else the
// pair is dropped).  `ls` is the fiber's arc length (MF_TN only).
__device__ __forceinline__ bool variant_value(float D, uint32_t c, float ls, const Metric& mt,
                                              float& v) {
  if (!(mt.flags & MF_TN)) {
    v = D;
    return true;
  }
  v = sqrtf(D) + tn_term(ls, mt.cext[2 * c]);
  return v <= mt.cext[2 * c + 1];
}

// Argmin key: D >= +0, so its bit pattern orders like the value; the low
// word breaks ties towards the lower centroid index.
__device__ __forceinline__ uint64_t make_key(float D, uint32_t c) {
  return ((uint64_t)__float_as_uint(D) << 32) | (uint64_t)c;
}

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ uint32_t bits_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Index j of the job holding work item `it`: the last j with
// start[j] <= it (start is ascending, start[0] = 0).
__device__ __forceinline__ int32_t find_job(const int64_t* __restrict__ start, int32_t njobs,
                                            int64_t it) {
  int32_t lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (start[mid] <= it) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// A value every lane holds equally, made visibly wave-uniform (kept in scalar
// registers, so addresses derived from it use scalar loads).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

struct Point {
  float x, y, z;
};

__device__ __forceinline__ Point ld(const float* __restrict__ r, int i) {
  return Point{r[3 * i], r[3 * i + 1], r[3 * i + 2]};
}

__device__ __forceinline__ float d2(const Point& a, const Point& b) {
  return d2(a.x, a.y, a.z, b.x, b.y, b.z);
}

// Survivor counters (filled only when statistics are requested).
struct StageCounts {
  unsigned long long* p;  // [0] filter pass, [1] test2, [2] test3, [3] accepted, [4] drains,
                          // [5] bound tiles, [6] survivor rows (tile-culled form)
};

// Exact stage for one (fiber, centroid) pair per lane: the paper's tests 2-4
// after its center test (section 2.3, "Progressive fiber discarding", and
// section 2.4: every point distance is compared with the threshold as soon as
// it is computed).  An order dies on its first point above T2; the pair is
// rejected when both orders died.  The wave leaves a test early when no lane
// has a live order.  Returns whether the pair is accepted and D (the smaller
// maximum of the live orders), which then equals the definition's
// min(max direct, max inverse).  Lanes with `active` false take part in the
// wave votes only; their `a`/`b` must still point to readable records.
template <bool STATS>
__device__ __forceinline__ bool exact_pair(const float* __restrict__ a,
                                           const float* __restrict__ b, bool active, float& D,
                                           StageCounts sc, int flags = 0) {
  const float t2 = b[NF];
  // test1: center point (orientation-free)
  float c = d2(ld(a, CTR), ld(b, CTR));
  bool ad = active && c <= t2;
  bool ai = ad;
  float md = c, mi = c;
  // test2: end points
  if (wave_any(ad || ai)) {
    Point a0 = ld(a, 0), a20 = ld(a, NP - 1), b0 = ld(b, 0), b20 = ld(b, NP - 1);
    float x0 = d2(a0, b0), x1 = d2(a20, b20);
    float y0 = d2(a0, b20), y1 = d2(a20, b0);
    ad = ad && x0 <= t2 && x1 <= t2;
    ai = ai && y0 <= t2 && y1 <= t2;
    if (flags & MF_DIR) {
      // the end points fix the direction; the other order is dropped
      const bool direct = fmaxf(x0, x1) <= fmaxf(y0, y1);
      ad = ad && direct;
      ai = ai && !direct;
    }
    md = fmaxf(md, fmaxf(x0, x1));
    mi = fmaxf(mi, fmaxf(y0, y1));
  }
  if (STATS) {
    uint64_t m = __ballot(ad || ai);
    if (lane_id() == 0 && m) atomicAdd(sc.p + 1, (unsigned long long)__popcll(m));
  }
  // test3: four intermediate points (a flip-symmetric choice)
  if (wave_any(ad || ai)) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = 4 + 4 * k;  // 4, 8, 12, 16
      Point ai_ = ld(a, i), bi = ld(b, i), bj = ld(b, NP - 1 - i);
      float x = d2(ai_, bi), y = d2(ai_, bj);
      ad = ad && x <= t2;
      ai = ai && y <= t2;
      md = fmaxf(md, x);
      mi = fmaxf(mi, y);
    }
  }
  if (STATS) {
    uint64_t m = __ballot(ad || ai);
    if (lane_id() == 0 && m) atomicAdd(sc.p + 2, (unsigned long long)__popcll(m));
  }
  // test4: the remaining 14 points, in groups, leaving when every order died
  constexpr int rest[14] = {1, 2, 3, 5, 6, 7, 9, 11, 13, 14, 15, 17, 18, 19};
#pragma unroll
  for (int g = 0; g < 14; g += 7) {
    if (wave_any(ad || ai)) {
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const int i = rest[g + k];
        Point ai_ = ld(a, i), bi = ld(b, i), bj = ld(b, NP - 1 - i);
        float x = d2(ai_, bi), y = d2(ai_, bj);
        ad = ad && x <= t2;
        ai = ai && y <= t2;
        md = fmaxf(md, x);
        mi = fmaxf(mi, y);
      }
    }
  }
  D = ad ? (ai ? fminf(md, mi) : md) : mi;
  bool ok = ad || ai;
  if (STATS) {
    uint64_t m = __ballot(ok);
    if (lane_id() == 0 && m) atomicAdd(sc.p + 3, (unsigned long long)__popcll(m));
  }
  return ok;
}

// Per-wave survivor queue in LDS.  An entry is (centroid << 8) | slot, where
// slot < 256 names one of the wave's fibers.  Entries are appended with a
// ballot and a prefix count (mbcnt), so the wave writes them without atomics.
struct WaveQueue {
  uint32_t* q;        // LDS, capacity entries
  uint64_t* keys;     // LDS, one argmin key per fiber slot of the wave
};

// Append the lanes of `mask` (each lane's own `entry`) at position n.
__device__ __forceinline__ void queue_push(WaveQueue wq, uint32_t& n, uint64_t mask,
                                           uint32_t entry) {
  if ((mask >> lane_id()) & 1ull) wq.q[n + bits_below(mask)] = entry;
  n += (uint32_t)__popcll(mask);
}

// Run the exact stage on the queued pairs and fold accepted ones into the
// per-fiber argmin keys.  `fib_base` points at the wave's first fiber record;
// `cprep` holds the prepared centroid records (63 coordinates + T2).
template <bool STATS>
__device__ __forceinline__ void queue_drain_body(WaveQueue wq, uint32_t n,
                                            const float* __restrict__ fib_base,
                                            const float* __restrict__ cprep, StageCounts sc,
                                            Metric mt) {
  const uint32_t lane = lane_id();
  if (STATS && lane == 0) {
    atomicAdd(sc.p + 0, (unsigned long long)n);
    atomicAdd(sc.p + 4, 1ull);
  }
  for (uint32_t r = 0; r < n; r += 64) {
    const uint32_t j = r + lane;
    const bool act = j < n;
    const uint32_t e = act ? wq.q[j] : 0u;
    const uint32_t slot = e & 0xffu;
    const uint32_t c = e >> 8;
    float D, v;
    const float* a = fib_base + (size_t)slot * NF;
    bool ok = exact_pair<STATS>(a, cprep + (size_t)c * CREC, act, D, sc, mt.flags);
    if (ok && variant_value(D, c, (mt.flags & MF_TN) ? arc_length(a) : 0.0f, mt, v))
      atomicMin((unsigned long long*)&wq.keys[slot], (unsigned long long)make_key(v, c));
  }
}

template <bool STATS>
__device__ __forceinline__ void queue_drain(WaveQueue wq, uint32_t n,
                                            const float* __restrict__ fib_base,
                                            const float* __restrict__ cprep, StageCounts sc,
                                            Metric mt) {
  queue_drain_body<STATS>(wq, n, fib_base, cprep, sc, mt);
}

// The same as a real call: drains are rare, and keeping the exact stage out
// of line lets a caller with many live registers (the MFMA accumulators of
// the prefilter) not reserve the exact stage's registers on top of its own.
template <bool STATS>
__device__ __noinline__ void queue_drain_call(WaveQueue wq, uint32_t n,
                                              const float* __restrict__ fib_base,
                                              const float* __restrict__ cprep, StageCounts sc,
                                              Metric mt) {
  queue_drain_body<STATS>(wq, n, fib_base, cprep, sc, mt);
}

// Final write of one fiber from its argmin key: the key holds D (the
// distance is sqrtf(D)) or, with MF_TN, the complete metric itself.
__device__ __forceinline__ void write_result(uint64_t key, const int32_t* __restrict__ bid,
                                             int32_t* __restrict__ label, float* __restrict__ dist,
                                             int flags = 0) {
  if (key == NO_KEY) {
    *label = -1;
    *dist = __builtin_inff();
  } else {
    const uint32_t c = (uint32_t)key;
    const float v = __uint_as_float((uint32_t)(key >> 32));
    *label = bid[c];
    *dist = (flags & MF_TN) ? v : sqrtf(v);
  }
}

}  // namespace seg
