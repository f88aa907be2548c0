// Device code shared by the prefilter kernels: number formats of the
// quantised features, the feature maps, the coordinate frame, per-curve
// quantisation with its measured error, MFMA fragments and the 32 x 32
// output layout.  The bound these pieces implement is derived at the top of
// seg_prefilter.hip.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "seg_device.hpp"

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
  static __device__ float decf(uint32_t b) { return __uint_as_float(b << 16); }
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
  static __device__ float decf(uint32_t b) { return __half2float(__ushort_as_half((unsigned short)b)); }
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
  // the same value in float (exact: at most 4 significant bits)
  static __device__ float decf(uint32_t b) {
    const float sg = (b & 0x80u) ? -1.0f : 1.0f;
    const uint32_t E = (b >> 3) & 0xFu, mnt = b & 7u;
    if (E == 0) return sg * ldexpf((float)mnt, -9);
    return sg * ldexpf((float)(8u + mnt), (int)E - 10);
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
__device__ inline void features(const float* __restrict__ p, const double* o, bool rev, double* x) {
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
constexpr int EMAX_SLOTS = 64;

struct PfParams {
  // bounding box of the atlas points as order-preserving integers
  int lo[3], hi[3];
  // largest fiber quantisation error (float bits), spread over slots so that
  // the per-wave atomics do not all hit one address; the maximum is the
  // maximum over the slots
  unsigned int emax_bits[EMAX_SLOTS];
};

// float <-> int with the same order (for atomic min / max of floats)
__device__ __forceinline__ int ord(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float unord(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff); }

// Origin (the middle of the atlas box, rounded to a whole millimetre) and the
// power-of-two scale of the stored codes (1 except for fp8, where the largest
// feature, about sqrt(3) times the half extent, must stay under 448).
struct Frame {
  double o[3];
  double s, is, s2;
};

__device__ __forceinline__ Frame frame(const PfParams* __restrict__ prm, int q) {
  Frame fr;
  float ext = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float lo = unord(prm->lo[d]), hi = unord(prm->hi[d]);
    const float c = rintf(0.5f * lo + 0.5f * hi);
    fr.o[d] = c;
    ext = fmaxf(ext, fmaxf(hi - c, c - lo));
  }
  float sc = 1.0f;
  if (q == Q_FP8) sc = exp2f(floorf(log2f(448.0f / fmaxf(2.0f * ext, 1e-3f))));
  fr.s = sc;
  fr.is = 1.0 / (double)sc;  // exact: a power of two
  fr.s2 = (double)sc * sc;
  return fr;
}

__device__ __forceinline__ double gamma_acc(int kp) { return 4.0 * (kp + 2) * 0x1p-24; }

// Quantise the features of one curve: packs the KP codes into `row` (16-byte
// stores), returns |Xq|^2 in *nq and the error bound |Xq - X| in *e; both are
// non-finite when a coordinate is.  With BOX, also returns in `xlo` / `xhi`
// float bounds that contain each exact (unquantised) feature (a template flag
// rather than a null test: comparing the address of a caller's local array
// with null keeps that array in scratch memory).
template <int Q, int MAPK, int KP, bool BOX = false>
__device__ __forceinline__ void quantise_row(const float* __restrict__ p, bool rev,
                                             const PfParams* __restrict__ prm,
                                             uint8_t* __restrict__ row, double* nq_out,
                                             double* e_out, float* xlo = nullptr,
                                             float* xhi = nullptr) {
  using T = QTraits<Q>;
  const Frame fr = frame(prm, Q);
  const double s = fr.s, is = fr.is;
  double x[KP];
  features<MAPK, KP>(p, fr.o, rev, x);
  double nq = 0.0, err = 0.0, nx = 0.0;
  constexpr int PER = 16 / T::bytes;  // codes per 16-byte store
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const uint32_t b = T::enc(x[k] * s);
    const double xq = T::dec(b) * is;  // exact (power-of-two scale)
    const int j = k % PER;
    const int word = j * T::bytes / 4, sh = (j * T::bytes % 4) * 8;
    w[word] = (sh == 0 ? 0u : w[word]) | (b << sh);
    if (j == PER - 1) *(uint4*)(row + (k / PER) * 16) = make_uint4(w[0], w[1], w[2], w[3]);
    nq += xq * xq;
    err += (xq - x[k]) * (xq - x[k]);
    nx += x[k] * x[k];
    if (BOX) {
      // the double feature is within 2^-50 relative of the exact one
      const double sl = fabs(x[k]) * 0x1p-48;
      xlo[k] = __double2float_rd(x[k] - sl);
      xhi[k] = __double2float_ru(x[k] + sl);
    }
  }
  *nq_out = nq;
  // the double features themselves (square roots) carry 2^-50 relative error
  *e_out = sqrt(err) * (1.0 + 0x1p-40) + 0x1p-50 * sqrt(nx) + 1e-30;
  if (!__builtin_isfinite(err + nx + nq)) {
    // a non-finite coordinate: the curve bypasses the bound (its constant
    // makes every product pass), so its codes must not turn the product into
    // NaN; a bf16 code of an infinite feature would (inf * 0, inf - inf)
    *e_out = __builtin_nan("");
#pragma unroll
    for (int k = 0; k < KP * T::bytes; k += 16) *(uint4*)(row + k) = make_uint4(0, 0, 0, 0);
  }
}

// Features of fiber row f (quantised codes, the row constant -Ha and the
// fiber's error bound).
template <int Q, int MAPK, int KP>
__device__ __forceinline__ void fiber_feature_row(const float* __restrict__ p, int64_t f,
                                                  int64_t n, const PfParams* __restrict__ prm,
                                                  uint8_t* __restrict__ row,
                                                  float* __restrict__ negh, float* e_out) {
  if (f >= n) {  // padding rows: zero features, never pass
#pragma unroll
    for (int k = 0; k < KP * QTraits<Q>::bytes; k += 16) *(uint4*)(row + k) = make_uint4(0, 0, 0, 0);
    negh[f] = -__builtin_inff();
    return;
  }
  double nq, e;
  quantise_row<Q, MAPK, KP>(p, false, prm, row, &nq, &e);
  if (!__builtin_isfinite(e)) {
    // a non-finite coordinate: bypass the cut (always survive) and leave the
    // error bound of the other fibers alone; the exact stage decides
    negh[f] = __builtin_inff();
    return;
  }
  const double g = gamma_acc(KP);
  const double ha = (0.5 - g) * nq * (1.0 - 0x1p-40);  // round towards passing
  negh[f] = __double2float_ru(-ha * frame(prm, Q).s2);
  *e_out = __double2float_ru(e);
}

// Features and column constant cb of centroid record p (point order
// reversed for `rev`).  cb = +inf: the column never passes (T < 0); -inf: it
// always passes (T = +inf, or a non-finite coordinate).  With BOX, also
// bounds of the exact features in `xlo` / `xhi` (empty for a column that
// never passes, unbounded for one that always does) and in `r2` the squared
// radius G * T2 / (1 - 8u) that contains |X(a) - X(b)|^2 of every accepted
// pair.
template <int Q, int MAPK, int KP, bool BOX = false>
__device__ __forceinline__ float column_row(const float* __restrict__ p, bool rev,
                                            const PfParams* __restrict__ prm,
                                            uint8_t* __restrict__ row, float* xlo = nullptr,
                                            float* xhi = nullptr, float* r2 = nullptr) {
  using MI = MapInfo<MAPK, KP>;
  const float t2 = p[NF];
  double nq, eb;
  quantise_row<Q, MAPK, KP, BOX>(p, rev, prm, row, &nq, &eb, xlo, xhi);
  if (!(t2 >= 0.0f)) {  // bundle never matches
    if (BOX) {
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        xlo[k] = __builtin_inff();
        xhi[k] = -__builtin_inff();
      }
      *r2 = -__builtin_inff();
    }
    return __builtin_inff();
  }
  if (__builtin_isinf(t2) || !__builtin_isfinite(eb)) {
    // bundle always matches, or a non-finite coordinate: always survive
    if (BOX) {
      if (!__builtin_isfinite(eb))
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          xlo[k] = -__builtin_inff();
          xhi[k] = __builtin_inff();
        }
      *r2 = __builtin_inff();
    }
    return -__builtin_inff();
  }
  unsigned int eb_bits = 0u;
#pragma unroll 8
  for (int i = 0; i < EMAX_SLOTS; ++i) eb_bits = max(eb_bits, prm->emax_bits[i]);
  const double E = (double)__uint_as_float(eb_bits);
  const double R2 = (double)MI::G * (double)t2 / (1.0 - 8.0 * 0x1p-24) * (1.0 + 0x1p-40);
  if (BOX) *r2 = __double2float_ru(R2);
  const double R = sqrt(R2) * (1.0 + 0x1p-40);
  const double S = (R + E + eb) * (1.0 + 0x1p-40);
  const double g = gamma_acc(KP);
  double v = 0.5 * (nq - S * S) - 0.5 * g * nq;
  v -= fabs(v) * 0x1p-40;  // round towards passing
  return __double2float_rd(v * frame(prm, Q).s2);
}

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

// Largest of a lane's 16 outputs as a tree of three-input maxima (depth 3,
// so the reduction does not serialise on one dependency chain).
__device__ __forceinline__ float max16(const f32x16& a) {
  const float m0 = __builtin_fmaxf(__builtin_fmaxf(a[0], a[1]), a[2]);
  const float m1 = __builtin_fmaxf(__builtin_fmaxf(a[3], a[4]), a[5]);
  const float m2 = __builtin_fmaxf(__builtin_fmaxf(a[6], a[7]), a[8]);
  const float m3 = __builtin_fmaxf(__builtin_fmaxf(a[9], a[10]), a[11]);
  const float m4 = __builtin_fmaxf(__builtin_fmaxf(a[12], a[13]), a[14]);
  const float n0 = __builtin_fmaxf(__builtin_fmaxf(m0, m1), m2);
  const float n1 = __builtin_fmaxf(__builtin_fmaxf(m3, m4), a[15]);
  return __builtin_fmaxf(n0, n1);
}

// Row of lane l's output register r in a 32x32 MFMA tile.
__device__ __forceinline__ int out_row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

}  // namespace seg
