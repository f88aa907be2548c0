// Several labels per fiber: the classification of the algorithm's previous
// version (section 2.4, "Classification of fibers"), where a fiber belongs to
// every bundle whose threshold test it passes, at the smallest distance over
// that bundle's passing centroids.
//
// The exact stage leaves, per fiber, up to K slots of (bundle + 1) << 32 |
// value bits (multi_insert), which fills a row's lowest empty slot first: a
// row's entries are a prefix of it.  Here:
//   1. multi_rows_kernel counts each row's prefix (reading only up to its
//      first empty slot) and sorts it when it has two entries or more (the
//      bundle sits in the high word, so the 64-bit order is the bundle order);
//   2. an exclusive scan turns the counts into CSR row offsets (n + 1);
//   3. multi_emit_kernel writes (bundle, distance) entries at the offsets,
//      counts the members of each bundle (per-block LDS histograms when the
//      atlas has at most 4,096 bundles, a bounded number of blocks) and
//      clears the slots it read, so the table is all zero for the next call.
// Every step is deterministic: the output does not depend on the order in
// which the exact stage found the pairs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "seg_internal.hpp"

namespace seg {
namespace {

constexpr int KMAX = 16;           // slots per fiber at most
constexpr int SCAN_T = 256;        // scan threads per block
constexpr int SCAN_V = 8;          // items per scan thread
constexpr int SCAN_ITEMS = SCAN_T * SCAN_V;
constexpr int HIST_MAX = 4096;     // bundles counted in LDS

__global__ __launch_bounds__(256) void multi_rows_kernel(unsigned long long* __restrict__ slots,
                                                         int K, int64_t n,
                                                         int64_t* __restrict__ counts) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= n) return;
  unsigned long long* __restrict__ row = slots + f * K;
  int c = 0;
  while (c < K && row[c] != 0ull) ++c;
  if (c >= 2) {
    unsigned long long r[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) r[k] = k < c ? row[k] : ~0ull;
    // odd-even transposition sort; the padding (~0) stays last
#pragma unroll
    for (int pass = 0; pass < KMAX; ++pass) {
#pragma unroll
      for (int k = pass & 1; k + 1 < KMAX; k += 2) {
        const unsigned long long a = r[k], b = r[k + 1];
        r[k] = b < a ? b : a;
        r[k + 1] = b < a ? a : b;
      }
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < c) row[k] = r[k];
  }
  counts[f] = c;
}

// Sum of each block's SCAN_ITEMS counts.
__global__ __launch_bounds__(SCAN_T) void scan_sums_kernel(const int64_t* __restrict__ v, int64_t n,
                                                           int64_t* __restrict__ part) {
  __shared__ int64_t s_sum[SCAN_T];
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_ITEMS;
  int64_t acc = 0;
  for (int i = threadIdx.x; i < SCAN_ITEMS; i += SCAN_T) {
    const int64_t j = b0 + i;
    acc += j < n ? v[j] : 0;
  }
  s_sum[threadIdx.x] = acc;
  __syncthreads();
  for (int w = SCAN_T / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s_sum[0];
}

// Exclusive scan of the block sums by one block, in chunks, with a carry;
// part[nblk] receives the total.
__global__ __launch_bounds__(SCAN_T) void scan_parts_kernel(int64_t* __restrict__ part,
                                                            int64_t nblk) {
  __shared__ int64_t s[SCAN_T];
  const int tid = threadIdx.x;
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nblk; c0 += SCAN_T) {
    const int64_t j = c0 + tid;
    const int64_t x = j < nblk ? part[j] : 0;
    s[tid] = x;
    __syncthreads();
    for (int w = 1; w < SCAN_T; w <<= 1) {
      const int64_t add = tid >= w ? s[tid - w] : 0;
      __syncthreads();
      s[tid] += add;
      __syncthreads();
    }
    const int64_t incl = s[tid];
    const int64_t chunk = s[SCAN_T - 1];
    if (j < nblk) part[j] = carry + incl - x;
    carry += chunk;
    __syncthreads();
  }
  if (tid == 0) part[nblk] = carry;
}

// Counts -> exclusive offsets, in place; offsets[n] = total.
__global__ __launch_bounds__(SCAN_T) void scan_apply_kernel(int64_t* __restrict__ v, int64_t n,
                                                            const int64_t* __restrict__ part,
                                                            int64_t nblk) {
  __shared__ int64_t s[SCAN_T];
  const int tid = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_ITEMS + (int64_t)tid * SCAN_V;
  int64_t x[SCAN_V];
  int64_t sum = 0;
#pragma unroll
  for (int i = 0; i < SCAN_V; ++i) {
    x[i] = b0 + i < n ? v[b0 + i] : 0;
    sum += x[i];
  }
  s[tid] = sum;
  __syncthreads();
  for (int w = 1; w < SCAN_T; w <<= 1) {
    const int64_t add = tid >= w ? s[tid - w] : 0;
    __syncthreads();
    s[tid] += add;
    __syncthreads();
  }
  int64_t run = part[blockIdx.x] + s[tid] - sum;
#pragma unroll
  for (int i = 0; i < SCAN_V; ++i) {
    if (b0 + i < n) v[b0 + i] = run;
    run += x[i];
  }
  if (blockIdx.x == 0 && tid == 0) v[n] = part[nblk];
}

__global__ __launch_bounds__(256) void multi_emit_kernel(
    unsigned long long* __restrict__ slots, int K, int64_t n,
    const int64_t* __restrict__ offsets, int32_t* __restrict__ bundles, float* __restrict__ dists,
    int64_t capacity, unsigned long long* __restrict__ bcount, int32_t nb, int mflags) {
  __shared__ unsigned int s_hist[HIST_MAX];
  const bool lds = nb <= HIST_MAX;
  if (lds)
    for (int i = threadIdx.x; i < nb; i += 256) s_hist[i] = 0u;
  __syncthreads();
  for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < n; f += (int64_t)gridDim.x * 256) {
    const int64_t o = offsets[f];
    const int c = (int)(offsets[f + 1] - o);
    unsigned long long* __restrict__ row = slots + f * K;
    for (int k = 0; k < c; ++k) {
      const unsigned long long e = row[k];
      row[k] = 0ull;
      const int32_t b = (int32_t)(e >> 32) - 1;
      const float v = __uint_as_float((uint32_t)e);
      if (b < 0 || b >= nb) continue;  // bundle ids were checked with the atlas
      if (o + k < capacity) {
        bundles[o + k] = b;
        dists[o + k] = (mflags & MF_TN) ? v : sqrtf(v);
      }
      if (bcount) {
        if (lds)
          atomicAdd(&s_hist[b], 1u);
        else
          atomicAdd(bcount + b, 1ull);
      }
    }
  }
  __syncthreads();
  if (lds && bcount)
    for (int i = threadIdx.x; i < nb; i += 256)
      if (s_hist[i]) atomicAdd(bcount + i, (unsigned long long)s_hist[i]);
}

__global__ __launch_bounds__(256) void fill_zero_u64_kernel(unsigned long long* __restrict__ p,
                                                            int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

int multi_collect(unsigned long long* slots, int32_t K, int64_t n, int64_t* offsets,
                  int32_t* bundles, float* dists, int64_t capacity, int64_t* bundle_counts,
                  int32_t nb, int mflags, void** scan_buf, size_t* scan_bytes, hipStream_t s) {
  if (K < 1 || K > KMAX) return -2;
  const int64_t nblk = n > 0 ? (n + SCAN_ITEMS - 1) / SCAN_ITEMS : 0;
  const size_t need = (size_t)(nblk + 1) * sizeof(int64_t);
  if (need > *scan_bytes) {
    if (*scan_buf) (void)hipFree(*scan_buf);
    *scan_buf = nullptr;
    *scan_bytes = 0;
    if (hipMalloc(scan_buf, need) != hipSuccess) return -3;
    *scan_bytes = need;
  }
  int64_t* part = (int64_t*)*scan_buf;
  unsigned long long* bc = (unsigned long long*)bundle_counts;
  if (bc && nb > 0)
    fill_zero_u64_kernel<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(bc, nb);
  if (n == 0) {
    fill_zero_u64_kernel<<<1, 256, 0, s>>>((unsigned long long*)offsets, 1);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const unsigned fb = (unsigned)((n + 255) / 256);
  multi_rows_kernel<<<fb, 256, 0, s>>>(slots, K, n, offsets);
  scan_sums_kernel<<<(unsigned)nblk, SCAN_T, 0, s>>>(offsets, n, part);
  scan_parts_kernel<<<1, SCAN_T, 0, s>>>(part, nblk);
  scan_apply_kernel<<<(unsigned)nblk, SCAN_T, 0, s>>>(offsets, n, part, nblk);
  const unsigned eb = fb < 2048u ? fb : 2048u;  // grid-stride: one histogram flush per block
  multi_emit_kernel<<<eb, 256, 0, s>>>(slots, K, n, offsets, bundles, dists, capacity, bc, nb,
                                       mflags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill_zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n > 0) fill_zero_u64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seg
