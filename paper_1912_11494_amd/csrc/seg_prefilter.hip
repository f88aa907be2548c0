// MFMA prefilter: a conservative mean bound evaluated as one small GEMM per
// fiber tile, then the exact float32 stage on the survivors.
//
// Bound (from Eq. 2).  For any point order o of the centroid, the mean of
// the squared point distances is at most their maximum, so
//     sum_i |a_i - b_o(i)|^2 <= 21 * D_o.                               (*)
// Expanding |X(a) - X(b)|^2 = |X(a)|^2 + |X(b)|^2 - 2 X(a).X(b) turns the
// left side into a dot product that runs on the matrix cores.
//
// Feature maps X:
//  * symmetric (modes bf16 / fp16 / fp8): for a group i < 10 the midpoint
//    m_i = (p_i + p_{20-i}) / 2 and the half span n_i = |p_i - p_{20-i}| / 2;
//    for i = 10 the center p_10.  Both are unchanged when the point order of
//    p is reversed.  For either order o of b, with d_i = a_i - b_o(i):
//      |m_i(a) - m_i(b)|^2 + (n_i(a) - n_i(b))^2
//        <= |(d_i + d_{20-i}) / 2|^2 + |(d_i - d_{20-i}) / 2|^2
//         = (|d_i|^2 + |d_{20-i}|^2) / 2 <= D_o
//    (reverse triangle inequality on the half spans, parallelogram law), so
//    |X(a) - X(b)|^2 <= G * min(D_dir, D_inv) = G * d_ME^2 with G groups.
//    One product covers both orders.
//  * oriented (mode bf16_oriented): the 63 coordinates; every centroid gives
//    two columns (direct and reversed) and (*) applies per order.
//
// Safety margin (the cut never drops a pair the exact stage accepts):
//  * accepted => D_fp32 <= T2, and the exact D is at most D_fp32 / (1 - 8u)
//    (u = 2^-24), so |X(a) - X(b)| <= R = sqrt(G * T2 / (1 - 8u));
//  * features are computed in double from the float32 points (midpoints
//    exactly), quantised to bf16 / fp16 / fp8 and the quantisation error
//    e = |Xq - X| is measured per curve; |Xq(a) - Xq(b)| <= R + E + e_b with
//    E the largest fiber error (a device reduction);
//  * the MFMA accumulates in float32: its error is bounded by
//    g * (sum |x_k y_k| + |C|), g = 4 (K + 2) u, and folded into the
//    per-fiber and per-column constants below, which are rounded towards
//    passing.
// The test is  out = Xq(a).Xq(b) - Ha  >=  cb  with
//    Ha = |Xq(a)|^2 / 2 - g |Xq(a)|^2             (rows, MFMA C operand)
//    cb = (|Xq(b)|^2 - (R + E + e_b)^2) / 2 - g |Xq(b)|^2 / 2   (columns).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "seg_device.hpp"
#include "seg_internal.hpp"

namespace seg {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;

enum QT : int { Q_BF16 = 0, Q_F16 = 1, Q_FP8 = 2 };

// ------------------------------------------------------------------ formats

template <int Q> struct QTraits;
template <> struct QTraits<Q_BF16> {
  static constexpr int bytes = 2;
  static __device__ uint32_t enc(double x) {
    __hip_bfloat16 h = __float2bfloat16((float)x);
    return (uint32_t)__bfloat16_as_ushort(h);
  }
  static __device__ double dec(uint32_t b) {
    return (double)__uint_as_float(b << 16);
  }
};
template <> struct QTraits<Q_F16> {
  static constexpr int bytes = 2;
  static __device__ uint32_t enc(double x) {
    float f = (float)x;
    f = fminf(fmaxf(f, -65504.0f), 65504.0f);
    return (uint32_t)__half_as_ushort(__float2half_rn(f));
  }
  static __device__ double dec(uint32_t b) {
    return (double)__half2float(__ushort_as_half((unsigned short)b));
  }
};
// OCP e4m3 (bias 7, no infinities, max 448), round to nearest even, saturating.
template <> struct QTraits<Q_FP8> {
  static constexpr int bytes = 1;
  static __device__ uint32_t enc(double x) {
    uint32_t s = x < 0 ? 0x80u : 0u;
    double a = fabs(x);
    if (!(a < 464.0)) return s | 0x7Eu;  // beyond the rounding midpoint of 448: saturate
    if (a < 0.015625) {                  // subnormal range: multiples of 2^-9
      double q = rint(a * 512.0);        // ties to even
      return q >= 8.0 ? (s | 0x08u) : (s | (uint32_t)q);
    }
    int e;
    double f = frexp(a, &e);             // a = f * 2^e, f in [0.5, 1)
    double q = rint(f * 16.0);           // 1.mmm with 3 fraction bits, in [8, 16]
    if (q >= 16.0) {
      q = 8.0;
      e += 1;
    }
    const int E = e - 1 + 7;
    if (E > 15 || (E == 15 && q > 14.0)) return s | 0x7Eu;
    return s | ((uint32_t)E << 3) | ((uint32_t)q - 8u);
  }
  static __device__ double dec(uint32_t b) {
    const double sg = (b & 0x80u) ? -1.0 : 1.0;
    const uint32_t E = (b >> 3) & 0xFu, mnt = b & 7u;
    if (E == 0) return sg * mnt * (1.0 / 512.0);
    return sg * (1.0 + mnt / 8.0) * ldexp(1.0, (int)E - 7);
  }
};

// ------------------------------------------------------------------ feature maps

enum MAP : int { MAP_SYM = 0, MAP_ORIENTED = 1 };

template <int KP> struct SymGroups;
template <> struct SymGroups<16> {
  static constexpr int G = 4;
  static __device__ int grp(int g) {
    constexpr int t[4] = {10, 7, 4, 0};
    return t[g];
  }
};
template <> struct SymGroups<32> {
  static constexpr int G = 8;
  static __device__ int grp(int g) {
    constexpr int t[8] = {10, 8, 7, 5, 4, 2, 1, 0};
    return t[g];
  }
};
template <> struct SymGroups<48> {
  static constexpr int G = 11;
  static __device__ int grp(int g) { return 10 - g; }
};

template <int MAPK, int KP> struct MapInfo;
template <int KP> struct MapInfo<MAP_SYM, KP> {
  static constexpr int G = SymGroups<KP>::G;  // groups in the bound
  static constexpr int CPC = 1;               // columns per centroid
};
template <> struct MapInfo<MAP_ORIENTED, 64> {
  static constexpr int G = 21;
  static constexpr int CPC = 2;
};

// Features (double) of curve p relative to origin o; `rev` reverses the
// point order (oriented map only).
template <int MAPK, int KP>
__device__ void features(const float* __restrict__ p, const double* o, bool rev, double* x) {
  if constexpr (MAPK == MAP_SYM) {
    int k = 0;
#pragma unroll
    for (int g = 0; g < SymGroups<KP>::G; ++g) {
      const int i = SymGroups<KP>::grp(g);
      if (i == CTR) {
#pragma unroll
        for (int d = 0; d < 3; ++d) x[k++] = (double)p[3 * CTR + d] - o[d];
      } else {
        const int j = NP - 1 - i;
        double h2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double a = p[3 * i + d], b = p[3 * j + d];
          x[k++] = 0.5 * (a + b) - o[d];  // exact in double
          h2 += (a - b) * (a - b);
        }
        x[k++] = 0.5 * sqrt(h2);
      }
    }
    for (; k < KP; ++k) x[k] = 0.0;
  } else {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int s = rev ? NP - 1 - i : i;
#pragma unroll
      for (int d = 0; d < 3; ++d) x[3 * i + d] = (double)p[3 * s + d] - o[d];
    }
    for (int k = NF; k < KP; ++k) x[k] = 0.0;
  }
}

// Origin, fp8 scale: one block over the prepared centroid records.
struct PfParams {
  float o[3];
  float scale;  // features are stored multiplied by `scale` (a power of two)
  float scale2;
  unsigned int emax_bits;  // largest fiber quantisation error (float bits)
};

__global__ __launch_bounds__(1024) void pf_params_kernel(const float* __restrict__ cprep, int32_t m,
                                                         int q, PfParams* __restrict__ prm) {
  __shared__ float smin[3][1024], smax[3][1024];
  float lo[3] = {3.4e38f, 3.4e38f, 3.4e38f}, hi[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
  for (int64_t i = threadIdx.x; i < (int64_t)m * NP; i += blockDim.x) {
    const float* p = cprep + (i / NP) * CREC + 3 * (i % NP);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fminf(lo[d], p[d]);
      hi[d] = fmaxf(hi[d], p[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    smin[d][threadIdx.x] = lo[d];
    smax[d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        smin[d][threadIdx.x] = fminf(smin[d][threadIdx.x], smin[d][threadIdx.x + w]);
        smax[d][threadIdx.x] = fmaxf(smax[d][threadIdx.x], smax[d][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float ext = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      // origin: the middle of the atlas box, rounded to a whole millimetre
      const float c = rintf(0.5f * (smin[d][0] + smax[d][0]));
      prm->o[d] = c;
      ext = fmaxf(ext, fmaxf(smax[d][0] - c, c - smin[d][0]));
    }
    float s = 1.0f;
    if (q == Q_FP8) {
      // the largest feature is about sqrt(3) * ext; keep it under 448 with room
      s = exp2f(floorf(log2f(448.0f / fmaxf(2.0f * ext, 1e-3f))));
    }
    prm->scale = s;
    prm->scale2 = s * s;
    prm->emax_bits = 0u;
  }
}

__device__ __forceinline__ double gamma_acc(int kp) { return 4.0 * (kp + 2) * 0x1p-24; }

// One thread per fiber: quantised features (row-major [n_pad][KP]), the row
// constant -Ha (MFMA C operand) and the device maximum of the error.
template <int Q, int MAPK, int KP>
__global__ __launch_bounds__(256) void pf_fiber_kernel(const float* __restrict__ fibers, int64_t n,
                                                       int64_t n_pad, PfParams* __restrict__ prm,
                                                       uint8_t* __restrict__ feat,
                                                       float* __restrict__ negh) {
  using T = QTraits<Q>;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_pad) return;
  uint8_t* row = feat + f * (KP * T::bytes);
  if (f >= n) {  // padding rows: zero features, never pass
    for (int k = 0; k < KP * T::bytes; ++k) row[k] = 0;
    negh[f] = -__builtin_inff();
    return;
  }
  const double o[3] = {prm->o[0], prm->o[1], prm->o[2]};
  const double s = prm->scale;
  double x[KP];
  features<MAPK, KP>(fibers + f * NF, o, false, x);
  double nq = 0.0, err = 0.0, nx = 0.0;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const uint32_t b = T::enc(x[k] * s);
    const double xq = T::dec(b) / s;  // exact (power-of-two scale)
    if constexpr (T::bytes == 2) {
      ((uint16_t*)row)[k] = (uint16_t)b;
    } else {
      row[k] = (uint8_t)b;
    }
    nq += xq * xq;
    err += (xq - x[k]) * (xq - x[k]);
    nx += x[k] * x[k];
  }
  if (!__builtin_isfinite(err + nx + nq)) {
    // a non-finite coordinate: bypass the cut (always survive) and leave the
    // error bound of the other fibers alone; the exact stage decides
    negh[f] = __builtin_inff();
    return;
  }
  // error of the double features themselves (square roots): 2^-50 relative
  const double e = sqrt(err) * (1.0 + 0x1p-40) + 0x1p-50 * sqrt(nx) + 1e-30;
  const double g = gamma_acc(KP);
  const double ha = (0.5 - g) * nq * (1.0 - 0x1p-40);  // round towards passing
  negh[f] = __double2float_ru(-ha * prm->scale2);
  atomicMax(&prm->emax_bits, __float_as_uint(__double2float_ru(e)));
}

// One thread per column (centroid, or centroid x order): features and cb.
template <int Q, int MAPK, int KP>
__global__ __launch_bounds__(256) void pf_column_kernel(const float* __restrict__ cprep, int32_t m,
                                                        int32_t ncols_pad,
                                                        const PfParams* __restrict__ prm,
                                                        uint8_t* __restrict__ feat,
                                                        float* __restrict__ cb) {
  using T = QTraits<Q>;
  using MI = MapInfo<MAPK, KP>;
  const int32_t col = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (col >= ncols_pad) return;
  uint8_t* row = feat + (int64_t)col * (KP * T::bytes);
  const int32_t c = col / MI::CPC;
  if (c >= m) {  // padding columns never pass
    for (int k = 0; k < KP * T::bytes; ++k) row[k] = 0;
    cb[col] = __builtin_inff();
    return;
  }
  const float* p = cprep + (int64_t)c * CREC;
  const float t2 = p[NF];
  const double o[3] = {prm->o[0], prm->o[1], prm->o[2]};
  const double s = prm->scale;
  double x[KP];
  features<MAPK, KP>(p, o, (col % MI::CPC) == 1, x);
  double nq = 0.0, err = 0.0, nx = 0.0;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const uint32_t b = T::enc(x[k] * s);
    const double xq = T::dec(b) / s;
    if constexpr (T::bytes == 2) {
      ((uint16_t*)row)[k] = (uint16_t)b;
    } else {
      row[k] = (uint8_t)b;
    }
    nq += xq * xq;
    err += (xq - x[k]) * (xq - x[k]);
    nx += x[k] * x[k];
  }
  if (!(t2 >= 0.0f)) {  // bundle never matches
    cb[col] = __builtin_inff();
    return;
  }
  if (__builtin_isinf(t2) || !__builtin_isfinite(err + nx + nq)) {
    // bundle always matches, or a non-finite coordinate: always survive
    cb[col] = -__builtin_inff();
    return;
  }
  const double eb = sqrt(err) * (1.0 + 0x1p-40) + 0x1p-50 * sqrt(nx) + 1e-30;
  const double E = (double)__uint_as_float(prm->emax_bits);
  const double R = sqrt((double)MI::G * (double)t2 / (1.0 - 8.0 * 0x1p-24)) * (1.0 + 0x1p-40);
  const double S = (R + E + eb) * (1.0 + 0x1p-40);
  const double g = gamma_acc(KP);
  double v = 0.5 * (nq - S * S) - 0.5 * g * nq;
  v -= fabs(v) * 0x1p-40;  // round towards passing
  cb[col] = __double2float_rd(v * prm->scale2);
}

// ------------------------------------------------------------------ fused kernel

template <int Q> struct Frag;
template <> struct Frag<Q_BF16> {
  typedef bf16x8 T;
  static __device__ f32x16 mfma(T a, T b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Frag<Q_F16> {
  typedef f16x8 T;
  static __device__ f32x16 mfma(T a, T b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct Frag<Q_FP8> {
  typedef long T;
  static __device__ f32x16 mfma(T a, T b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, c, 0, 0, 0);
  }
};

// Row of lane l's output register r in a 32x32 MFMA tile.
__device__ __forceinline__ int out_row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

// Rows = fibers (A operand, held in registers for the whole kernel), columns
// = centroid columns (B operand, streamed 32 at a time).  Each wave owns GF
// groups of 32 fibers.  Per 32-column tile and group: KP/16 MFMAs starting
// from C = -Ha, then the largest of the lane's 16 outputs is compared with
// the column constant cb.  A lane above it has a survivor among its rows; the
// wave then pushes every (fiber, centroid) above cb into its LDS queue (ballot
// + prefix count), drained by the exact stage as in the plain pass.  With
// PAIRS, survivors are written to a global list instead (diagnostics).
template <int Q, int KP, int GF, int CPC, bool STATS, bool PAIRS>
__global__ __launch_bounds__(256) void prefilter_kernel(
    const uint8_t* __restrict__ ffeat, const float* __restrict__ fnegh,
    const uint8_t* __restrict__ cfeat, const float* __restrict__ cbias, int32_t ncols_pad,
    const float* __restrict__ fibers, int64_t n, const float* __restrict__ cprep,
    const int32_t* __restrict__ bid, int32_t* __restrict__ labels, float* __restrict__ dists,
    unsigned long long* __restrict__ counters, int32_t* __restrict__ pairs, int64_t cap) {
  using FT = typename Frag<Q>::T;
  constexpr int KS = KP / 16;
  constexpr int EB = QTraits<Q>::bytes;
  constexpr int WAVES = 4;
  constexpr int FPW = GF * 32;
  // A group of 32 fibers x 32 columns adds at most 1024 entries; the queue is
  // drained before a group whenever that might not fit.
  constexpr int QCAP = 2048;
  static_assert(FPW <= 256, "slot must fit 8 bits");
  __shared__ uint32_t s_queue[PAIRS ? 1 : WAVES][PAIRS ? 1 : QCAP];
  __shared__ uint64_t s_keys[PAIRS ? 1 : WAVES][PAIRS ? 1 : FPW];
  const int lane = (int)(threadIdx.x & 63u);
  const int wave = (int)(threadIdx.x >> 6);
  const int half = lane >> 5;
  const int64_t wbase = ((int64_t)blockIdx.x * WAVES + wave) * FPW;
  WaveQueue wq{PAIRS ? nullptr : s_queue[wave], PAIRS ? nullptr : s_keys[wave]};
  StageCounts sc{counters};

  FT afr[GF][KS];
  f32x16 negh[GF];
#pragma unroll
  for (int g = 0; g < GF; ++g) {
    const int64_t frow = wbase + g * 32 + (lane & 31);
#pragma unroll
    for (int s = 0; s < KS; ++s)
      afr[g][s] = *(const FT*)(ffeat + frow * (KP * EB) + (s * 16 + 8 * half) * EB);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = *(const float4*)(fnegh + wbase + g * 32 + 8 * q + 4 * half);
      negh[g][4 * q + 0] = v.x;
      negh[g][4 * q + 1] = v.y;
      negh[g][4 * q + 2] = v.z;
      negh[g][4 * q + 3] = v.w;
    }
  }
  if (!PAIRS) {
    for (int k = lane; k < FPW; k += 64) wq.keys[k] = NO_KEY;
  }
  const float* fib_base = fibers + (wbase < n ? wbase : 0) * NF;

  uint32_t qn = 0;
  const int32_t ntiles = ncols_pad / 32;
  for (int32_t t = 0; t < ntiles; ++t) {
    const int32_t col = t * 32 + (lane & 31);
    FT bfr[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
      bfr[s] = *(const FT*)(cfeat + (int64_t)col * (KP * EB) + (s * 16 + 8 * half) * EB);
    const float cb = cbias[col];
    f32x16 acc[GF];
    bool hit[GF];
    bool anyhit = false;
#pragma unroll
    for (int g = 0; g < GF; ++g) {
      acc[g] = Frag<Q>::mfma(afr[g][0], bfr[0], negh[g]);
#pragma unroll
      for (int s = 1; s < KS; ++s) acc[g] = Frag<Q>::mfma(afr[g][s], bfr[s], acc[g]);
      float mx = fmaxf(fmaxf(acc[g][0], acc[g][1]), acc[g][2]);
#pragma unroll
      for (int r = 3; r < 15; r += 2) mx = fmaxf(fmaxf(mx, acc[g][r]), acc[g][r + 1]);
      mx = fmaxf(mx, acc[g][15]);
      hit[g] = mx >= cb;
      anyhit = anyhit || hit[g];
    }
    if (!wave_any(anyhit)) continue;
    const uint32_t cent = (uint32_t)(col / CPC);
#pragma unroll
    for (int g = 0; g < GF; ++g) {
      if (!wave_any(hit[g])) continue;
      if (!PAIRS && qn > (uint32_t)(QCAP - 1024)) {
        queue_drain_call<STATS>(wq, qn, fib_base, cprep, sc);
        qn = 0;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int slot = g * 32 + out_row(lane, r);
        const bool p = hit[g] && acc[g][r] >= cb && wbase + slot < n;
        const uint64_t msk = __ballot(p);
        if (!msk) continue;
        if (PAIRS) {
          if (p) {
            const unsigned long long k = atomicAdd(counters, 1ull);
            if ((int64_t)k < cap) {
              pairs[2 * k] = (int32_t)(wbase + slot);
              pairs[2 * k + 1] = (int32_t)cent;
            }
          }
        } else {
          queue_push(wq, qn, msk, (cent << 8) | (uint32_t)slot);
        }
      }
    }
  }
  if (PAIRS) return;
  queue_drain_call<STATS>(wq, qn, fib_base, cprep, sc);
  for (int k = lane; k < FPW; k += 64) {
    const int64_t f = wbase + k;
    if (f < n) write_result(wq.keys[k], bid, labels + f, dists + f);
  }
}

// ------------------------------------------------------------------ host side

namespace {

int grow(void** p, size_t* have, size_t want) {
  if (want <= *have) return 0;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  if (hipMalloc(p, want) != hipSuccess) return -3;
  *have = want;
  return 0;
}

struct Cfg {
  int q, mapk, kp, gf;
};

// Mode -> (format, map); tile -> (KP, GF).
int resolve(int mode, int tile, Cfg* c) {
  switch (mode) {
    case 2: c->q = Q_BF16; c->mapk = MAP_SYM; break;
    case 3: c->q = Q_F16; c->mapk = MAP_SYM; break;
    case 4: c->q = Q_FP8; c->mapk = MAP_SYM; break;
    case 5: c->q = Q_BF16; c->mapk = MAP_ORIENTED; break;
    default: return -2;
  }
  if (c->mapk == MAP_ORIENTED) {
    c->kp = 64;
    switch (tile) {  // (K, fiber groups of 32 per wave)
      case 0:
      case 1: c->gf = 2; break;
      case 2: c->gf = 4; break;
      default: return -2;
    }
    return 0;
  }
  switch (tile) {  // symmetric map: (K, fiber groups of 32 per wave)
    case 0:
    case 1: c->kp = 16; c->gf = 2; break;
    case 2: c->kp = 16; c->gf = 4; break;
    case 3: c->kp = 16; c->gf = 8; break;
    case 4: c->kp = 32; c->gf = 2; break;
    case 5: c->kp = 32; c->gf = 4; break;
    case 6: c->kp = 48; c->gf = 2; break;
    case 7: c->kp = 48; c->gf = 4; break;
    default: return -2;
  }
  return 0;
}

template <int Q, int MAPK, int KP, int GF>
int launch_cfg(const float* fibers, int64_t n, const float* cprep, int32_t m, const int32_t* bid,
               int32_t* labels, float* dists, unsigned long long* counters, int32_t* pairs,
               int64_t cap, PrefilterBuf& pb, hipEvent_t* ev, hipStream_t s) {
  using MI = MapInfo<MAPK, KP>;
  constexpr int EB = QTraits<Q>::bytes;
  constexpr int FPB = 4 * GF * 32;  // fibers per block
  const int64_t n_pad = (n + FPB - 1) / FPB * FPB;
  const int32_t ncols = m * MI::CPC;
  const int32_t ncols_pad = (ncols + 31) / 32 * 32;
  int rc = grow(&pb.fib_feat, &pb.fib_feat_bytes, (size_t)n_pad * KP * EB);
  rc = rc ? rc : grow((void**)&pb.fib_h, &pb.fib_h_bytes, (size_t)n_pad * sizeof(float));
  rc = rc ? rc : grow(&pb.cen_feat, &pb.cen_feat_bytes,
                      (size_t)ncols_pad * (KP * EB + sizeof(float)));
  if (rc) return rc;
  if (!pb.emax && hipMalloc((void**)&pb.emax, sizeof(PfParams)) != hipSuccess) return -3;
  PfParams* prm = (PfParams*)pb.emax;
  uint8_t* cfeat = (uint8_t*)pb.cen_feat;
  float* cb = (float*)(cfeat + (size_t)ncols_pad * KP * EB);
  pf_params_kernel<<<1, 1024, 0, s>>>(cprep, m, Q, prm);
  pf_fiber_kernel<Q, MAPK, KP><<<(unsigned)((n_pad + 255) / 256), 256, 0, s>>>(
      fibers, n, n_pad, prm, (uint8_t*)pb.fib_feat, pb.fib_h);
  pf_column_kernel<Q, MAPK, KP><<<(unsigned)((ncols_pad + 255) / 256), 256, 0, s>>>(
      cprep, m, ncols_pad, prm, cfeat, cb);
  const unsigned blocks = (unsigned)(n_pad / FPB);
  if (pairs) {
    prefilter_kernel<Q, KP, GF, MI::CPC, false, true><<<blocks, 256, 0, s>>>(
        (const uint8_t*)pb.fib_feat, pb.fib_h, cfeat, cb, ncols_pad, fibers, n, cprep, bid,
        labels, dists, counters, pairs, cap);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return -1;
  if (counters)
    prefilter_kernel<Q, KP, GF, MI::CPC, true, false><<<blocks, 256, 0, s>>>(
        (const uint8_t*)pb.fib_feat, pb.fib_h, cfeat, cb, ncols_pad, fibers, n, cprep, bid,
        labels, dists, counters, nullptr, 0);
  else
    prefilter_kernel<Q, KP, GF, MI::CPC, false, false><<<blocks, 256, 0, s>>>(
        (const uint8_t*)pb.fib_feat, pb.fib_h, cfeat, cb, ncols_pad, fibers, n, cprep, bid,
        labels, dists, counters, nullptr, 0);
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dispatch(const Cfg& c, const float* fibers, int64_t n, const float* cprep, int32_t m,
             const int32_t* bid, int32_t* labels, float* dists, unsigned long long* counters,
             int32_t* pairs, int64_t cap, PrefilterBuf& pb, hipEvent_t* ev, hipStream_t s) {
#define SEG_PF(QQ, MM, KK, GG)                                                                   \
  if (c.q == QQ && c.mapk == MM && c.kp == KK && c.gf == GG)                                     \
    return launch_cfg<QQ, MM, KK, GG>(fibers, n, cprep, m, bid, labels, dists, counters, pairs, \
                                      cap, pb, ev, s);
  SEG_PF(Q_BF16, MAP_SYM, 16, 2)
  SEG_PF(Q_BF16, MAP_SYM, 16, 4)
  SEG_PF(Q_BF16, MAP_SYM, 16, 8)
  SEG_PF(Q_BF16, MAP_SYM, 32, 2)
  SEG_PF(Q_BF16, MAP_SYM, 32, 4)
  SEG_PF(Q_BF16, MAP_SYM, 48, 2)
  SEG_PF(Q_BF16, MAP_SYM, 48, 4)
  SEG_PF(Q_F16, MAP_SYM, 16, 2)
  SEG_PF(Q_F16, MAP_SYM, 16, 4)
  SEG_PF(Q_F16, MAP_SYM, 16, 8)
  SEG_PF(Q_F16, MAP_SYM, 32, 2)
  SEG_PF(Q_F16, MAP_SYM, 32, 4)
  SEG_PF(Q_F16, MAP_SYM, 48, 2)
  SEG_PF(Q_F16, MAP_SYM, 48, 4)
  SEG_PF(Q_FP8, MAP_SYM, 16, 2)
  SEG_PF(Q_FP8, MAP_SYM, 16, 4)
  SEG_PF(Q_FP8, MAP_SYM, 16, 8)
  SEG_PF(Q_FP8, MAP_SYM, 32, 2)
  SEG_PF(Q_FP8, MAP_SYM, 32, 4)
  SEG_PF(Q_FP8, MAP_SYM, 48, 2)
  SEG_PF(Q_FP8, MAP_SYM, 48, 4)
  SEG_PF(Q_BF16, MAP_ORIENTED, 64, 2)
  SEG_PF(Q_BF16, MAP_ORIENTED, 64, 4)
#undef SEG_PF
  return -2;
}

}  // namespace

int run_prefilter(int mode, int cfg, const float* fibers, int64_t n, const float* cprep,
                  const float4* ccen, int32_t m, const int32_t* bid, int32_t* labels,
                  float* dists, unsigned long long* counters, PrefilterBuf& pb, hipEvent_t* ev,
                  hipStream_t s) {
  (void)ccen;
  Cfg c;
  if (resolve(mode, cfg, &c)) return -2;
  return dispatch(c, fibers, n, cprep, m, bid, labels, dists, counters, nullptr, 0, pb, ev, s);
}

int prefilter_pairs(int mode, const float* fibers, int64_t n, const float* cprep,
                    const float4* ccen, int32_t m, int32_t* pairs, int64_t cap,
                    unsigned long long* count, PrefilterBuf& pb, hipStream_t s) {
  (void)ccen;
  Cfg c;
  if (resolve(mode, 0, &c)) return -2;
  return dispatch(c, fibers, n, cprep, m, nullptr, nullptr, nullptr, count, pairs, cap, pb,
                  nullptr, s);
}

}  // namespace seg
