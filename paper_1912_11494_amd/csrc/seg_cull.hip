// Sorted, tile-culled MFMA prefilter (symmetric feature map, K = 16).
//
// The streaming prefilter evaluates its bound on every (fiber, centroid)
// pair.  Most pairs are far apart, and that can be decided for whole tiles:
// every accepted pair satisfies |X(a) - X(b)|^2 <= R2(b) = G * T2 / (1 - 8u)
// for the exact features X (the bound derived at the top of
// seg_prefilter.hip).  If a box (lowest and highest value per feature) holds
// the features of a group of fibers and another box those of a tile of
// centroid columns, then every pair of the two is at least
//     gap^2 = sum_k max(0, lo_B,k - hi_A,k, lo_A,k - hi_B,k)^2
// apart, and the tile cannot hold a match for any fiber of the group when
// gap^2 exceeds the largest R2 of the tile.  The float gap computation
// rounds each difference and the sum to nearest, which overstates gap^2 by at
// most 2^-19 relative; the stored tile radius carries a factor 1 + 2^-17.
// A fiber's box is its quantised features widened by its quantisation error
// bound |Xq - X| (which bounds every component's error).
//
// Small boxes need neighbours in consecutive order, so fibers and centroids
// are ordered by the cell of their center point (point 10) in a 32 x 32 x 32
// grid over the atlas box, cells in Morton order (15-bit keys): a stable
// least-significant-digit radix sort with two passes of 8 and 7 bits.  Each
// pass counts digits per block, scans the (digit, block) counts, and
// scatters with ranks from wave ballots, so equal keys keep their input
// order and the permutation is deterministic.
//
// Fiber features are computed in input order (coalesced reads of the
// records); the culled kernel reads its rows through the permutation.
//
// Work per block (4 waves, 256 consecutive sorted rows = 8 groups of 32), in
// rounds of 256 centroid tiles:
//   A. each thread tests one tile against the union box of the block;
//      passing tiles are appended to an LDS list;
//   B. each wave tests the listed tiles against its two groups and runs the
//      MFMA bound on the (tile, group) pairs left, loading the next tile's
//      fragment while the current one is computed; pairs at or above the
//      column constant go to the wave's queue and the exact stage, as in the
//      streaming prefilter.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <atomic>
#include <cstring>

#include "seg_device.hpp"
#include "seg_internal.hpp"
#include "seg_pf.hpp"

namespace seg {

namespace {

constexpr int CELL_AXIS_BITS = 5;
constexpr int KPC = 16;                // feature width of the culled path
constexpr int BOXD = KPC;              // boxed feature dimensions
constexpr int GBOX = 2 * BOXD;         // floats per group box: lo[16], hi[16]
constexpr int TROWS = 2 * BOXD + 1;    // tile box rows: lo[16], hi[16], radius
constexpr float GAP_SLACK = 1.0f + 0x1p-17f;
// survivor queue per wave (entries); handed on before a push when fewer
// than 64 places are left
constexpr int CULL_QCAP = 512;
constexpr uint32_t RESCUE = 0x80000000u;  // a wave's survivor count: overflowed

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < CELL_AXIS_BITS; ++b) r |= ((v >> b) & 1u) << (3 * b);
  return r;
}

// Cell of a curve's center point in the atlas box, Morton order.  Points
// outside the box (or NaN) clamp into the grid: the cell only orders.
__device__ __forceinline__ uint32_t center_cell(const float* __restrict__ rec,
                                                const PfParams* __restrict__ prm) {
  constexpr int SIDE = 1 << CELL_AXIS_BITS;
  uint32_t code = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float lo = unord(prm->lo[d]), hi = unord(prm->hi[d]);
    const float ext = hi - lo;
    const float t = (rec[3 * CTR + d] - lo) * ((float)SIDE / (ext > 0.0f ? ext : 1.0f));
    const int q = t >= 0.0f ? (t < (float)(SIDE - 1) ? (int)t : SIDE - 1) : 0;
    code |= spread3((uint32_t)q) << d;
  }
  return code;
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort of 15-bit keys with int32 values, 8-bit digits.
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;                        // rounds of 64 items per wave
constexpr int RS_IPW = 64 * RS_ROUNDS;               // items per wave
constexpr int RS_IPB = RS_IPW * (RS_THREADS / 64);   // items per block
constexpr int RS_BINS = 256;

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int shift) {
  return (key >> shift) & (RS_BINS - 1);
}

// Digit counts of each block: hist[digit][block].
__global__ __launch_bounds__(RS_THREADS) void rs_hist_kernel(const uint32_t* __restrict__ keys,
                                                             int64_t n, int shift,
                                                             uint32_t* __restrict__ hist,
                                                             int32_t nblocks) {
  __shared__ uint32_t s_cnt[RS_BINS];
  const int tid = (int)threadIdx.x;
  s_cnt[tid] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_IPB;
  for (int j = 0; j < RS_IPB / RS_THREADS; ++j) {
    const int64_t i = base + (int64_t)j * RS_THREADS + tid;
    if (i < n) atomicAdd(&s_cnt[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nblocks + blockIdx.x] = s_cnt[tid];
}

// Block-wide exclusive scan of one value per thread (256 threads); returns
// the exclusive prefix and the total in *tot.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp,
                                                          uint32_t* tot) {
  const int tid = (int)threadIdx.x;
  s_tmp[tid] = v;
  __syncthreads();
  for (int off = 1; off < RS_THREADS; off <<= 1) {
    const uint32_t x = tid >= off ? s_tmp[tid - off] : 0u;
    __syncthreads();
    s_tmp[tid] += x;
    __syncthreads();
  }
  const uint32_t incl = s_tmp[tid];
  *tot = s_tmp[RS_THREADS - 1];
  __syncthreads();
  return incl - v;
}

// One block per digit: exclusive scan of hist[digit][*] in place; the
// digit's total goes to tot[digit].
__global__ __launch_bounds__(RS_THREADS) void rs_scan_rows_kernel(uint32_t* __restrict__ hist,
                                                                  int32_t nblocks,
                                                                  uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_tmp[RS_THREADS];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  const int tid = (int)threadIdx.x;
  uint32_t carry = 0;
  for (int32_t c0 = 0; c0 < nblocks; c0 += RS_THREADS * 4) {
    uint32_t v[4];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int32_t i = c0 + tid * 4 + k;
      v[k] = i < nblocks ? row[i] : 0u;
      sum += v[k];
    }
    uint32_t chunk;
    uint32_t run = carry + block_exclusive_scan(sum, s_tmp, &chunk);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int32_t i = c0 + tid * 4 + k;
      if (i < nblocks) row[i] = run;
      run += v[k];
    }
    carry += chunk;
  }
  if (tid == 0) tot[blockIdx.x] = carry;
}

// Stable scatter.  Item i of wave w of block b has the block-local position
//   (items of smaller digits in b) + (items of digit d in earlier waves of b)
//   + (items of digit d earlier in this wave's range),
// the last term from a per-wave running count and, within a round of 64,
// the lanes below with the same digit (a match mask built from 8 ballots).
// Items are first placed in LDS at that position, then written out in
// block-local order: item k of digit d goes to
//   start[d] + hist[d][b] + (k - local start of d),
// where start[d] (the exclusive scan of the digit totals) is computed by
// every block from the totals,
// so each digit's run of the block is written contiguously.  With PAYLOAD,
// the 64-byte record of each item's value moves along (the last pass of the
// fiber sort gathers the fiber payloads into sorted order).
template <bool PAYLOAD>
__global__ __launch_bounds__(RS_THREADS) void rs_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in, int64_t n,
    int shift, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dtot,
    int32_t nblocks, uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out,
    const uint4* __restrict__ pay_in, uint4* __restrict__ pay_out) {
  constexpr int WAVES = RS_THREADS / 64;
  __shared__ uint32_t s_cnt[WAVES][RS_BINS];
  __shared__ uint32_t s_lstart[RS_BINS];
  __shared__ uint32_t s_gstart[RS_BINS];
  __shared__ uint32_t s_tmp[RS_THREADS];
  __shared__ uint32_t s_key[RS_IPB];
  __shared__ int32_t s_val[RS_IPB];
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  for (int w = 0; w < WAVES; ++w) s_cnt[w][tid] = 0u;
  __syncthreads();
  const int64_t bstart = (int64_t)blockIdx.x * RS_IPB;
  const int64_t wb = bstart + (int64_t)wave * RS_IPW;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = wb + r * 64 + lane;
    if (i < n) atomicAdd(&s_cnt[wave][digit_of(keys_in[i], shift)], 1u);
  }
  __syncthreads();
  {
    const int d = tid;  // RS_THREADS == RS_BINS
    uint32_t c[WAVES], tot = 0;
    for (int w = 0; w < WAVES; ++w) {
      c[w] = s_cnt[w][d];
      tot += c[w];
    }
    uint32_t all;
    uint32_t l = block_exclusive_scan(tot, s_tmp, &all);
    // start of digit d over all blocks: exclusive scan of the digit totals
    const uint32_t dstart = block_exclusive_scan(dtot[d], s_tmp, &all);
    s_lstart[d] = l;
    s_gstart[d] = dstart + hist[(int64_t)d * nblocks + blockIdx.x];
    for (int w = 0; w < WAVES; ++w) {
      s_cnt[w][d] = l;
      l += c[w];
    }
  }
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1ull;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = wb + r * 64 + lane;
    const bool valid = i < n;
    const uint32_t key = valid ? keys_in[i] : 0u;
    const uint32_t d = digit_of(key, shift);
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      mask &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(mask & below);
    const uint32_t start = s_cnt[wave][d];  // read by every lane before the leader moves it
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) s_cnt[wave][d] = start + (uint32_t)__popcll(mask);
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      s_key[start + rank] = key;
      s_val[start + rank] = vals_in ? vals_in[i] : (int32_t)i;
    }
  }
  __syncthreads();
  const int64_t items = n - bstart < RS_IPB ? n - bstart : RS_IPB;
  for (int64_t k = tid; k < items; k += RS_THREADS) {
    const uint32_t key = s_key[k];
    const uint32_t d = digit_of(key, shift);
    const uint32_t g = s_gstart[d] + (uint32_t)k - s_lstart[d];
    const int32_t v = s_val[k];
    if (keys_out) keys_out[g] = key;
    vals_out[g] = v;
    if (PAYLOAD) {
#pragma unroll
      for (int q = 0; q < 4; ++q) pay_out[(int64_t)g * 4 + q] = pay_in[(int64_t)v * 4 + q];
    }
  }
}

// Center-cell keys of fibers (stride NF) or prepared centroids (stride CREC).
__global__ __launch_bounds__(256) void cell_key_kernel(const float* __restrict__ recs, int64_t n,
                                                       int32_t stride,
                                                       const PfParams* __restrict__ prm,
                                                       uint32_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = center_cell(recs + i * stride, prm);
}

// Per-fiber payload, 64 bytes (4 x uint4), written in input order:
//   words 0-1  the quantised feature codes (16 codes; fp8 uses word 0)
//   word 2     (-Ha, error bound |Xq - X|, input index, 0)
//   word 3     zero
// A fiber with a non-finite coordinate gets -Ha = +inf (it bypasses the cut)
// and error bound +inf (its box is unbounded).
constexpr int PAY_WORDS = 4;

// One lane per fiber: a block takes batches of CF_BLOCK fibers (grid-stride,
// as many blocks as the device holds at once);
// a batch's contiguous records (CF_BLOCK x 252 bytes) come in with coalesced
// 16-byte loads into registers, go to LDS, and the loads of the block's next
// batch are issued before the lanes quantise the current one, each its own
// record from LDS (a stride of 63 words, no bank conflict), and write its
// payload, its center-cell key and the reset value of its argmin key.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
constexpr int CF_BLOCK = 128;
constexpr int CF_V = (CF_BLOCK * NF / 4 + CF_BLOCK - 1) / CF_BLOCK;  // loads per lane

__device__ __forceinline__ void cf_load(const float* __restrict__ fibers, int64_t n, int64_t b,
                                        int tid, f4u* v) {
  const int64_t f0 = b * CF_BLOCK;
  const int cnt = (int)(n - f0 < CF_BLOCK ? n - f0 : CF_BLOCK);
  const int n4 = (cnt * NF) >> 2;
  const float* __restrict__ src = fibers + f0 * NF;
#pragma unroll
  for (int u = 0; u < CF_V; ++u) {
    const int i = tid + u * CF_BLOCK;
    if (i < n4) v[u] = *(const f4u*)(src + 4 * i);
  }
}

template <int Q>
__global__ __launch_bounds__(CF_BLOCK) void cull_fiber_kernel(const float* __restrict__ fibers,
                                                              int64_t n,
                                                              PfParams* __restrict__ prm,
                                                              uint4* __restrict__ pay,
                                                              uint32_t* __restrict__ keys,
                                                              unsigned long long* __restrict__ fkeys) {
  __shared__ float s_rec[CF_BLOCK * NF];
  const int tid = (int)threadIdx.x;
  const int64_t nb = (n + CF_BLOCK - 1) / CF_BLOCK;
  f4u v[CF_V];
  int64_t b = blockIdx.x;
  if (b < nb) cf_load(fibers, n, b, tid, v);
  float e32 = 0.0f;
  for (; b < nb; b += gridDim.x) {
    const int64_t f0 = b * CF_BLOCK;
    const int cnt = (int)(n - f0 < CF_BLOCK ? n - f0 : CF_BLOCK);
    {
      const int nfl = cnt * NF;
      const int n4 = nfl >> 2;
#pragma unroll
      for (int u = 0; u < CF_V; ++u) {
        const int i = tid + u * CF_BLOCK;
        if (i < n4) {
          s_rec[4 * i] = v[u].x;
          s_rec[4 * i + 1] = v[u].y;
          s_rec[4 * i + 2] = v[u].z;
          s_rec[4 * i + 3] = v[u].w;
        }
      }
      if (tid < nfl - 4 * n4) s_rec[4 * n4 + tid] = fibers[f0 * NF + 4 * n4 + tid];
    }
    __syncthreads();
    if (b + gridDim.x < nb) cf_load(fibers, n, b + gridDim.x, tid, v);
    const int64_t f = f0 + tid;
    if (tid < cnt) {
      float rec[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) rec[k] = s_rec[tid * NF + k];
      uint4* P = pay + f * PAY_WORDS;
      if (QTraits<Q>::bytes == 1) P[1] = make_uint4(0u, 0u, 0u, 0u);
      double nq, e;
      quantise_row<Q, MAP_SYM, KPC>(rec, false, prm, (uint8_t*)P, &nq, &e);
      float nh, er;
      if (!__builtin_isfinite(e)) {
        nh = __builtin_inff();
        er = __builtin_inff();
      } else {
        const double g = gamma_acc(KPC);
        const double ha = (0.5 - g) * nq * (1.0 - 0x1p-40);  // round towards passing
        nh = __double2float_ru(-ha * frame(prm, Q).s2);
        er = __double2float_ru(e);
        e32 = fmaxf(e32, er);
      }
      P[2] = make_uint4(__float_as_uint(nh), __float_as_uint(er), (uint32_t)f, 0u);
      P[3] = make_uint4(0u, 0u, 0u, 0u);
      keys[f] = center_cell(rec, prm);
      fkeys[f] = NO_KEY;
    }
    __syncthreads();  // the records are read before the next batch lands
  }
  for (int off = 32; off > 0; off >>= 1) e32 = fmaxf(e32, __shfl_xor(e32, off));
  if ((tid & 63) == 0)
    atomicMax(&prm->emax_bits[(blockIdx.x * (CF_BLOCK / 64) + (tid >> 6)) % EMAX_SLOTS],
              __float_as_uint(e32));
}

// Blocks of cull_fiber_kernel<Q> that the device holds at once (register- or
// LDS-bound), queried once per process and quantisation.
template <int Q>
int64_t cf_grid() {
  static std::atomic<int64_t> g{0};
  int64_t v = g.load(std::memory_order_relaxed);
  if (v == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cull_fiber_kernel<Q>, CF_BLOCK, 0) !=
            hipSuccess ||
        cus <= 0 || per <= 0)
      return 1024;
    v = (int64_t)cus * per;
    g.store(v, std::memory_order_relaxed);
  }
  return v;
}

// Lowest / highest over the 32 lanes of each half wave.
__device__ __forceinline__ void half_wave_box(float* lo, float* hi, int nd) {
  for (int k = 0; k < nd; ++k) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
      hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
    }
  }
}

// Sorted columns: column j is centroid cperm[j]; each half wave writes the
// box and largest radius of its tile of 32 columns (struct of arrays,
// row-major [TROWS][ntiles]).
template <int Q>
__global__ __launch_bounds__(256) void cull_column_kernel(const float* __restrict__ cprep,
                                                          int32_t m, int32_t ncols_pad,
                                                          const int32_t* __restrict__ cperm,
                                                          const PfParams* __restrict__ prm,
                                                          uint8_t* __restrict__ feat,
                                                          float* __restrict__ cb,
                                                          int32_t* __restrict__ ccent,
                                                          float* __restrict__ tbox) {
  using T = QTraits<Q>;
  const int32_t col = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  float lo[BOXD], hi[BOXD];
  float r2 = -__builtin_inff();
#pragma unroll
  for (int k = 0; k < BOXD; ++k) {
    lo[k] = __builtin_inff();
    hi[k] = -__builtin_inff();
  }
  if (col < ncols_pad) {
    uint8_t* row = feat + (int64_t)col * (KPC * T::bytes);
    if (col >= m) {  // padding columns never pass
#pragma unroll
      for (int k = 0; k < KPC * T::bytes; k += 16) *(uint4*)(row + k) = make_uint4(0, 0, 0, 0);
      cb[col] = __builtin_inff();
      ccent[col] = 0;
    } else {
      const int32_t c = cperm[col];
      ccent[col] = c;
      cb[col] = column_row<Q, MAP_SYM, KPC>(cprep + (int64_t)c * CREC, false, prm, row, lo, hi,
                                            &r2);
    }
  }
  half_wave_box(lo, hi, BOXD);
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) r2 = fmaxf(r2, __shfl_xor(r2, off));
  const int32_t tile = col >> 5;
  const int32_t ntiles = ncols_pad >> 5;
  if ((threadIdx.x & 31) == 0 && tile < ntiles) {
#pragma unroll
    for (int k = 0; k < BOXD; ++k) {
      tbox[(int64_t)k * ntiles + tile] = lo[k];
      tbox[(int64_t)(BOXD + k) * ntiles + tile] = hi[k];
    }
    tbox[(int64_t)(2 * BOXD) * ntiles + tile] = r2 * GAP_SLACK;
  }
}

struct CullJob {
  const uint4* pay;      // fiber payloads in input order [n][PAY_WORDS]
  const int32_t* perm;   // sorted position -> input index
  const PfParams* prm;   // frame (code scale)
  const uint8_t* cfeat;  // sorted columns [ncols_pad][16]
  const float* cbias;    // cb per sorted column
  const int32_t* ccent;  // centroid of each sorted column
  const float* tbox;     // tile boxes [TROWS][ntiles]
  int32_t ntiles;
  const float* fibers;   // the subject's fiber records (input order)
  int64_t n;
  const float* cprep;    // prepared centroid records (63 coordinates + T2)
  unsigned long long* keys;  // per-fiber argmin keys (input order)
  int2* list;                // per wave: QCAP survivor pairs (fiber, centroid)
  uint32_t* list_n;          // per wave: pairs in its part of `list`
  int2* ovf;                 // survivor pairs beyond a wave's part, shared
  unsigned long long* ovf_count;  // entries reserved in `ovf`
  int64_t ovf_cap;
};

// Full metric of one (fiber, centroid) pair held in registers (Eq. 2): the
// largest point distance of each order, an order dying on a point above T2
// as in the exact stage, D the smaller maximum of the live orders.  Every
// point is evaluated (no early exit); the accepted set and D equal those of
// exact_pair (with the same metric flags).
__device__ __forceinline__ bool dense_pair(const float* a, const float* b, float t2, float& D,
                                           int flags) {
  float md = 0.0f, mi = 0.0f;
  bool ad = true, ai = true;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int j = NP - 1 - i;
    const float x = d2(a[3 * i], a[3 * i + 1], a[3 * i + 2], b[3 * i], b[3 * i + 1], b[3 * i + 2]);
    const float y = d2(a[3 * i], a[3 * i + 1], a[3 * i + 2], b[3 * j], b[3 * j + 1], b[3 * j + 2]);
    ad = ad && x <= t2;
    ai = ai && y <= t2;
    md = fmaxf(md, x);
    mi = fmaxf(mi, y);
  }
  if (flags & MF_DIR) {
    // the order with the smaller largest end-point distance (direct on ties)
    const float x0 = d2(a[0], a[1], a[2], b[0], b[1], b[2]);
    const float x1 = d2(a[60], a[61], a[62], b[60], b[61], b[62]);
    const float y0 = d2(a[0], a[1], a[2], b[60], b[61], b[62]);
    const float y1 = d2(a[60], a[61], a[62], b[0], b[1], b[2]);
    const bool direct = fmaxf(x0, x1) <= fmaxf(y0, y1);
    ad = ad && direct;
    ai = ai && !direct;
  }
  D = ad ? (ai ? fminf(md, mi) : md) : mi;
  return ad || ai;
}

// The exact stage on the survivors the culled kernel queued: wave w's own
// pairs list[w * QCAP + j], j < list_n[w], then its share of the overflow
// list.  Each lane loads its
// fiber record (252 bytes, 4-byte aligned) and centroid record (256 bytes)
// with 16-byte loads, all at once, then evaluates the pair; accepted pairs
// fold into the per-fiber keys (with MULTI, into the fiber's bundle slots).
// With STATS the staged exact_pair runs instead, to count its tests.
template <bool STATS, int QCAP, bool MULTI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MULTI ? 3 : 4))) void exact_list_kernel(const int2* __restrict__ list,
                                                         const uint32_t* __restrict__ list_n,
                                                         int64_t nwaves,
                                                         const int2* __restrict__ ovf,
                                                         const unsigned long long* __restrict__ ovf_count,
                                                         int64_t ovf_cap,
                                                         const int32_t* __restrict__ perm,
                                                         int64_t n,
                                                         const float* __restrict__ fibers,
                                                         const float* __restrict__ cprep,
                                                         unsigned long long* __restrict__ keys,
                                                         unsigned long long* __restrict__ counters,
                                                         Metric mt, MultiOut mo) {
  StageCounts sc{counters};
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nwaves) return;
  const int lane = (int)(threadIdx.x & 63);
  // the input indices of the wave's 64 sorted rows, read up front: the rows
  // of its own list lie in this window
  const int64_t prow = w * 64 + lane;
  const int32_t pwin = perm[prow < n ? prow : n - 1];
  // 64 pairs per step, one per lane.  An entry is (sorted row, centroid);
  // row -1 marks an unused entry, and the rows of a rescued wave are left to
  // the rescue kernel.
  // `own`: the wave's own list, whose rows are all the wave's own (its flag
  // was tested already); the overflow list mixes rows of every wave
  // `first`: the entry of this lane in the first 64, when read already
  auto run = [&](const int2* __restrict__ src, int64_t cnt, bool own, const int2* first) {
    for (int64_t j0 = 0; j0 < cnt; j0 += 64) {
      const int64_t j = j0 + lane;
      const bool pre = j0 == 0 && first;  // the same on every lane
      int2 e = j < cnt ? (pre ? *first : src[j]) : make_int2(-1, 0);
      bool act = e.x >= 0 && (own || !(list_n[e.x >> 6] & RESCUE));
      int32_t fi;
      if (pre)
        fi = __shfl(pwin, (int)(e.x - w * 64) & 63);  // every lane takes part
      else
        fi = act ? perm[e.x] : 0;
      e = act ? make_int2(fi, e.y) : make_int2(0, 0);
      const float* ar = fibers + (int64_t)e.x * NF;
      const float* br = cprep + (size_t)e.y * CREC;
      float D, v;
      bool ok;
      if (STATS) {
        ok = exact_pair<true>(ar, br, act, D, sc, mt.flags);
      } else {
        float a[NF], b[CREC];
#pragma unroll
        for (int k = 0; k < 15; ++k) {
          const f4u v = *(const f4u*)(ar + 4 * k);
          a[4 * k] = v.x;
          a[4 * k + 1] = v.y;
          a[4 * k + 2] = v.z;
          a[4 * k + 3] = v.w;
        }
        a[60] = ar[60];
        a[61] = ar[61];
        a[62] = ar[62];
#pragma unroll
        for (int k = 0; k < CREC / 4; ++k) {
          const float4 v = *(const float4*)(br + 4 * k);
          b[4 * k] = v.x;
          b[4 * k + 1] = v.y;
          b[4 * k + 2] = v.z;
          b[4 * k + 3] = v.w;
        }
        ok = act && dense_pair(a, b, b[NF], D, mt.flags);
      }
      if (ok && variant_value(D, (uint32_t)e.y, (mt.flags & MF_TN) ? arc_length(ar) : 0.0f, mt, v)) {
        if (MULTI)
          multi_insert(mo.slots + (int64_t)e.x * mo.K, mo.K, (uint32_t)mo.bid[e.y], v, mo.flag);
        else
          atomicMin(&keys[e.x], (unsigned long long)make_key(v, (uint32_t)e.y));
      }
    }
  };
  // the wave's first 64 entries are read with its count, not after it (the
  // wave's part of the list always exists; entries past the count are unused)
  const int2 first = list[w * QCAP + lane];
  const uint32_t cnt = list_n[w];
  if (!(cnt & RESCUE)) run(list + w * QCAP, cnt, true, &first);  // else: the rescue kernel
  // the shared overflow list, 64 entries per wave in turn
  const int64_t total = (int64_t)*ovf_count < ovf_cap ? (int64_t)*ovf_count : ovf_cap;
  for (int64_t i0 = w * 64; i0 < total; i0 += nwaves * 64)
    run(ovf + i0, total - i0 < 64 ? total - i0 : 64, false, nullptr);
}

// Waves of the culled kernel whose survivors overflowed: each lane takes one
// of the wave's 64 sorted rows and evaluates its fiber against every
// centroid (the full metric, no cut), keeping the lexicographic minimum of
// (D, centroid) over accepted centroids (with MULTI, every accepted pair goes
// to the fiber's bundle slots).  Only for degenerate inputs (more than 512
// survivors per 64 fibers).
template <bool STATS, bool MULTI>
__global__ __launch_bounds__(256) void rescue_kernel(const uint32_t* __restrict__ list_n,
                                                     int64_t nwaves,
                                                     const int32_t* __restrict__ perm, int64_t n,
                                                     const float* __restrict__ fibers,
                                                     const float* __restrict__ cprep, int32_t m,
                                                     unsigned long long* __restrict__ keys,
                                                     unsigned long long* __restrict__ counters,
                                                     Metric mt, MultiOut mo) {
  // a bounded grid walks every wave's flag; almost all are clear
  for (int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); w < nwaves;
       w += (int64_t)gridDim.x * 4) {
    if (!(list_n[w] & RESCUE)) continue;
    unsigned long long naccepted = 0;
    const int64_t row = w * 64 + (threadIdx.x & 63);
    const bool act = row < n;
    const int64_t f = act ? (int64_t)perm[row] : 0;
    float a[NF];
    const float* ar = fibers + f * NF;
#pragma unroll
    for (int k = 0; k < NF; ++k) a[k] = ar[k];
    const float ls = (mt.flags & MF_TN) ? arc_length(a) : 0.0f;
    unsigned long long best = NO_KEY;
    for (int32_t c = 0; c < m; ++c) {
      const float* b = cprep + (size_t)c * CREC;  // the same for every lane
      float D, v;
      if (act && dense_pair(a, b, b[NF], D, mt.flags)) {
        ++naccepted;
        if (variant_value(D, (uint32_t)c, ls, mt, v)) {
          if (MULTI) {
            multi_insert(mo.slots + f * mo.K, mo.K, (uint32_t)mo.bid[c], v, mo.flag);
          } else {
            const unsigned long long k = make_key(v, (uint32_t)c);
            best = k < best ? k : best;
          }
        }
      }
    }
    if (!MULTI && act) keys[f] = best;
    if (STATS && naccepted) atomicAdd(counters + 3, naccepted);
  }
}

// labels / distances of every fiber from its key.
__global__ __launch_bounds__(256) void finalize_kernel(const unsigned long long* __restrict__ keys,
                                                       int64_t n, const int32_t* __restrict__ bid,
                                                       int32_t* __restrict__ labels,
                                                       float* __restrict__ dists, int flags) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f < n) write_result(keys[f], bid, labels + f, dists + f, flags);
}

__global__ __launch_bounds__(256) void fill_u64_n_kernel(unsigned long long* __restrict__ p,
                                                         int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <int Q, bool STATS>
__global__ __launch_bounds__(256) void cull_kernel(CullJob job,
                                                   unsigned long long* __restrict__ counters) {
  using FT = typename Frag<Q>::T;
  constexpr int EB = QTraits<Q>::bytes;
  constexpr int WAVES = 4;
  constexpr int FPW = 64;
  constexpr int QCAP = CULL_QCAP;
  constexpr int CH = 6;      // candidate tiles per LDS chunk
  __shared__ int32_t s_cand[256];
  __shared__ uint8_t s_code[WAVES][256];
  __shared__ FT s_feat[3][CH][2][32];
  __shared__ float s_cb[3][CH][32];
  __shared__ uint32_t s_cent[3][CH][32];
  __shared__ uint32_t s_ncand;
  __shared__ float s_bbox[GBOX];
  __shared__ float s_gbox[2 * WAVES][GBOX];
  __shared__ uint32_t s_queue[WAVES][QCAP];
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5;
  const int64_t bbase = (int64_t)blockIdx.x * 256;
  const int64_t wbase = bbase + wave * FPW;
  const int64_t n = job.n;
  const int32_t ntiles = job.ntiles;
  uint32_t* wq = s_queue[wave];

  // the wave's two groups of 32 sorted positions: rows through the
  // permutation (a position past n is a padding row: zero codes, never
  // passes, empty box)
  // -Ha of the wave's 64 rows: the MFMA C operand, read when a product runs
  __shared__ __attribute__((aligned(16))) float s_nh[WAVES][FPW];
  const double is = frame(job.prm, Q).is;
  // both groups' permutation entries, then both groups' payloads, in flight
  // together (one dependent step each, not four in a row)
  FT afr[2];
  uint4 w2s[2];
  int32_t prow[2];
  // (unconditional loads at clamped positions, n >= 1; padding rows are
  // replaced after the loads)
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int64_t p = wbase + g * 32 + (lane & 31);
    prow[g] = job.perm[p < n ? p : n - 1];
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const uint4* P = job.pay + (int64_t)prow[g] * PAY_WORDS;
    afr[g] = *(const FT*)((const uint8_t*)P + 8 * half * EB);
    w2s[g] = P[2];
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    if (!(wbase + g * 32 + (lane & 31) < n)) {
      __builtin_memset(&afr[g], 0, sizeof(FT));
      w2s[g] = make_uint4(__float_as_uint(-__builtin_inff()), 0u, 0u, 0u);
    }
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const bool valid = wbase + g * 32 + (lane & 31) < n;
    const uint4 w2 = w2s[g];
    const float nh = __uint_as_float(w2.x);
    const float er = __uint_as_float(w2.y);
    if (half == 0) s_nh[wave][g * 32 + (lane & 31)] = nh;
    // this lane's 8 features of the row, widened by the row's error bound
    float lo[8], hi[8];
    uint8_t codes[sizeof(FT)];
    __builtin_memcpy(codes, &afr[g], sizeof(FT));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uint32_t b;
      if (EB == 2)
        b = (uint32_t)codes[2 * k] | ((uint32_t)codes[2 * k + 1] << 8);
      else
        b = codes[k];
      const float xq = (float)(QTraits<Q>::dec(b) * is);  // exact
      const float l = xq - er, h = xq + er;
      // one rounding each: widen by a relative 2^-23 (and a tiny absolute)
      lo[k] = l - fabsf(l) * 0x1p-23f - 0x1p-126f;
      hi[k] = h + fabsf(h) * 0x1p-23f + 0x1p-126f;
      if (!valid) {
        lo[k] = __builtin_inff();
        hi[k] = -__builtin_inff();
      } else if (!(er < __builtin_inff())) {
        lo[k] = -__builtin_inff();
        hi[k] = __builtin_inff();
      }
    }
    half_wave_box(lo, hi, 8);
    if ((lane & 31) == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        s_gbox[2 * wave + g][8 * half + k] = lo[k];
        s_gbox[2 * wave + g][BOXD + 8 * half + k] = hi[k];
      }
    }
  }
  if (tid == 0) s_ncand = 0;
  __syncthreads();
  // union of the block's 8 group boxes
  if (tid < GBOX) {
    float v = s_gbox[0][tid];
    for (int j = 1; j < 2 * WAVES; ++j)
      v = tid < BOXD ? fminf(v, s_gbox[j][tid]) : fmaxf(v, s_gbox[j][tid]);
    s_bbox[tid] = v;
  }
  __syncthreads();

  auto negh = [&](int g) {
    f32x16 c;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = *(const float4*)&s_nh[wave][g * 32 + 8 * q + 4 * half];
      c[4 * q + 0] = v.x;
      c[4 * q + 1] = v.y;
      c[4 * q + 2] = v.z;
      c[4 * q + 3] = v.w;
    }
    return c;
  };
  uint32_t qn = 0;
  // The first time the queue is handed on, it goes to the wave's part of the
  // survivor list; later hand-overs reserve room in the shared overflow list
  // (one atomic each).  The exact-stage kernel runs both.  Without room, the
  // reserved slots that exist are marked unused and the wave is marked for
  // the rescue kernel (top bit of its count), which evaluates its fibers
  // against every centroid; the exact-stage kernel then skips the wave's
  // own part.
  const int64_t wid = wbase / FPW;
  bool listed = false;
  auto flush = [&]() {
    if (STATS && lane == 0 && qn) atomicAdd(counters + 0, (unsigned long long)qn);
    if (!listed) {
      for (uint32_t j = lane; j < qn; j += 64) {
        const uint32_t e = wq[j];
        job.list[wid * QCAP + j] = make_int2((int32_t)(wbase + (e & 0xffu)), (int32_t)(e >> 8));
      }
      if (lane == 0) job.list_n[wid] = qn;
      listed = true;
    } else if (qn) {
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(job.ovf_count, (unsigned long long)qn);
      base = __shfl(base, 0);
      const bool room = (int64_t)(base + qn) <= job.ovf_cap;
      for (uint32_t j = lane; j < qn; j += 64) {
        if ((int64_t)(base + j) >= job.ovf_cap) break;
        const uint32_t e = wq[j];
        job.ovf[base + j] =
            room ? make_int2((int32_t)(wbase + (e & 0xffu)), (int32_t)(e >> 8)) : make_int2(-1, 0);
      }
      if (!room && lane == 0) job.list_n[wid] = RESCUE;
    }
    qn = 0;
  };
  // survivors of one (tile, group) product: every (fiber, column) at or
  // above the column constant is queued
  auto extract = [&](const f32x16& a, int g, uint32_t cent, float cbv) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int slot = g * 32 + out_row(lane, r);
      const bool p = a[r] >= cbv && wbase + slot < n;
      const uint64_t msk = __ballot(p);
      if (!msk) continue;
      if (qn > (uint32_t)(QCAP - 64)) flush();
      if ((msk >> lane) & 1ull) wq[qn + bits_below(msk)] = (cent << 8) | (uint32_t)slot;
      qn += (uint32_t)__popcll(msk);
    }
  };
  // candidate tiles pass through three LDS chunk buffers of CH tiles: thread
  // tid < 32 * CH owns column tid % 32 of tile tid / 32 of a chunk
  static_assert(32 * CH <= 256, "one chunk column per thread");
  FT gfe[2];
  float gcb = 0.0f;
  uint32_t gcent = 0;
  auto gload = [&](int32_t chunk, int32_t nc) {
    const int32_t i = chunk * CH + (tid >> 5);
    if (tid < 32 * CH && i < nc) {
      const int32_t col = s_cand[i] * 32 + (tid & 31);
      const uint8_t* src = job.cfeat + (int64_t)col * (KPC * EB);
      gfe[0] = *(const FT*)(src);
      gfe[1] = *(const FT*)(src + 8 * EB);
      gcb = job.cbias[col];
      gcent = (uint32_t)job.ccent[col];
    }
  };
  auto lstore = [&](int b, int32_t chunk, int32_t nc) {
    const int32_t i = chunk * CH + (tid >> 5);
    if (tid < 32 * CH && i < nc) {
      const int tl = tid >> 5, j = tid & 31;
      s_feat[b][tl][0][j] = gfe[0];
      s_feat[b][tl][1][j] = gfe[1];
      s_cb[b][tl][j] = gcb;
      s_cent[b][tl][j] = gcent;
    }
  };

  const float* gb0 = s_gbox[2 * wave];
  const float* gb1 = s_gbox[2 * wave + 1];
  for (int32_t t0 = 0; t0 < ntiles; t0 += 256) {
    // A: tiles against the block's box
    {
      const int32_t t = t0 + tid;
      bool pass = false;
      if (t < ntiles) {
        float s0 = 0.0f;
#pragma unroll 4
        for (int k = 0; k < BOXD; ++k) {
          const float tl = job.tbox[(int64_t)k * ntiles + t];
          const float th = job.tbox[(int64_t)(BOXD + k) * ntiles + t];
          const float g = fmaxf(fmaxf(tl - s_bbox[BOXD + k], s_bbox[k] - th), 0.0f);
          s0 = __builtin_fmaf(g, g, s0);
        }
        pass = !(s0 > job.tbox[(int64_t)(2 * BOXD) * ntiles + t]);
      }
      const uint64_t msk = __ballot(pass);
      uint32_t base = 0;
      if (lane == 0 && msk) base = atomicAdd(&s_ncand, (uint32_t)__popcll(msk));
      base = __shfl(base, 0);
      if (pass) s_cand[base + bits_below(msk)] = t;
    }
    __syncthreads();
    const int32_t nc = (int32_t)s_ncand;
    // B: the listed tiles against the wave's two groups (a code per
    // candidate: bit 0 group 0 runs, bit 1 group 1 runs)
    for (int32_t i = lane; i < nc; i += 64) {
      const int32_t t = s_cand[i];
      float s0 = 0.0f, s1 = 0.0f;
#pragma unroll 4
      for (int k = 0; k < BOXD; ++k) {
        const float tl = job.tbox[(int64_t)k * ntiles + t];
        const float th = job.tbox[(int64_t)(BOXD + k) * ntiles + t];
        const float g0 = fmaxf(fmaxf(tl - gb0[BOXD + k], gb0[k] - th), 0.0f);
        const float g1 = fmaxf(fmaxf(tl - gb1[BOXD + k], gb1[k] - th), 0.0f);
        s0 = __builtin_fmaf(g0, g0, s0);
        s1 = __builtin_fmaf(g1, g1, s1);
      }
      const float r2 = job.tbox[(int64_t)(2 * BOXD) * ntiles + t];
      const bool p0 = !(s0 > r2) && wbase < n;  // a group of padding rows never runs
      const bool p1 = !(s1 > r2) && wbase + 32 < n;
      s_code[wave][i] = (uint8_t)(p0 | (p1 << 1));
      if (STATS) {
        const uint64_t m0 = __ballot(p0), m1 = __ballot(p1);
        if (lane == 0 && (m0 | m1))
          atomicAdd(counters + 5, (unsigned long long)(__popcll(m0) + __popcll(m1)));
      }
    }
    // C: the MFMA bound on the (tile, group) pairs left, chunk by chunk
    const int32_t nchunks = (nc + CH - 1) / CH;
    gload(0, nc);
    lstore(0, 0, nc);
    gload(1, nc);
    lstore(1, 1, nc);
    __syncthreads();
    int buf = 0;
    for (int32_t k = 0; k < nchunks; ++k) {
      gload(k + 2, nc);
      const int32_t ulim = nc - k * CH < CH ? nc - k * CH : CH;
      for (int u = 0; u < ulim; ++u) {
        const uint32_t code = __builtin_amdgcn_readfirstlane(s_code[wave][k * CH + u]);
        if (!code) continue;
        const FT b = s_feat[buf][u][half][lane & 31];
        const float cbv = s_cb[buf][u][lane & 31];
        if (code & 1u) {
          const f32x16 a = Frag<Q>::mfma(afr[0], b, negh(0));
          if (wave_any(max16(a) >= cbv)) extract(a, 0, s_cent[buf][u][lane & 31], cbv);
        }
        if (code & 2u) {
          const f32x16 a = Frag<Q>::mfma(afr[1], b, negh(1));
          if (wave_any(max16(a) >= cbv)) extract(a, 1, s_cent[buf][u][lane & 31], cbv);
        }
      }
      // chunk k+2 goes into the buffer of chunk k-1 (nobody reads it any more)
      lstore(buf == 0 ? 2 : buf - 1, k + 2, nc);
      __syncthreads();
      buf = buf == 2 ? 0 : buf + 1;
    }
    __syncthreads();
    if (tid == 0) s_ncand = 0;
    __syncthreads();
  }
  flush();
}

int grow(void** p, size_t* have, size_t want) {
  if (want <= *have) return 0;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  if (hipMalloc(p, want) != hipSuccess) return -3;
  *have = want;
  return 0;
}

// Stable sort of n keys (15 bits) into a permutation: vals_b[k] = index of
// the k-th smallest key, and with `pay_in`, pay_out[k] = pay_in[vals_b[k]]
// (64-byte records).  keys_a holds the keys on entry; keys_b, vals_a, vals_b
// and hist (RS_BINS * nblocks + RS_BINS) are scratch.
int radix_sort(int64_t n, uint32_t* keys_a, uint32_t* keys_b, int32_t* vals_a, int32_t* vals_b,
               uint32_t* hist, const uint4* pay_in, uint4* pay_out, hipStream_t s) {
  if (n <= 0) return 0;
  const int32_t nblocks = (int32_t)((n + RS_IPB - 1) / RS_IPB);
  uint32_t* tot = hist + (size_t)RS_BINS * nblocks;
  // pass 1: bits 0-7, input order as values; pass 2: bits 8-14
  for (int pass = 0; pass < 2; ++pass) {
    const int shift = 8 * pass;
    const uint32_t* kin = pass == 0 ? keys_a : keys_b;
    rs_hist_kernel<<<nblocks, RS_THREADS, 0, s>>>(kin, n, shift, hist, nblocks);
    rs_scan_rows_kernel<<<RS_BINS, RS_THREADS, 0, s>>>(hist, nblocks, tot);
    if (pass == 0)
      rs_scatter_kernel<false><<<nblocks, RS_THREADS, 0, s>>>(
          keys_a, nullptr, n, shift, hist, tot, nblocks, keys_b, vals_a, nullptr, nullptr);
    else if (pay_in)
      rs_scatter_kernel<true><<<nblocks, RS_THREADS, 0, s>>>(
          keys_b, vals_a, n, shift, hist, tot, nblocks, nullptr, vals_b, pay_in, pay_out);
    else
      rs_scatter_kernel<false><<<nblocks, RS_THREADS, 0, s>>>(
          keys_b, vals_a, n, shift, hist, tot, nblocks, nullptr, vals_b, nullptr, nullptr);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int Q>
int cull_launch(const float* fibers, int64_t n, const float* cprep, int32_t m, const int32_t* bid,
                int32_t* labels, float* dists, unsigned long long* counters, Metric mt,
                PrefilterBuf& pb, hipEvent_t* ev, hipStream_t s, const MultiOut* mo,
                const int32_t* cperm_cached) {
  constexpr int EB = QTraits<Q>::bytes;
  const int64_t n_pad = (n + 255) / 256 * 256;
  const int32_t ncols_pad = (m + 31) / 32 * 32;
  const int32_t ntiles = ncols_pad / 32;
  const int64_t nk = std::max<int64_t>(std::max<int64_t>(n, m), 1);  // sort capacity
  const int64_t nblocks = (nk + RS_IPB - 1) / RS_IPB;
  const int64_t nwaves = n_pad / 64;
  // scratch: fiber payloads (input order), sort state, columns
  // and tile boxes, per-fiber keys, per-wave survivor lists
  const size_t pay_bytes = (size_t)n * PAY_WORDS * sizeof(uint4);
  int rc = grow(&pb.fib_feat, &pb.fib_feat_bytes, pay_bytes);
  rc = rc ? rc : grow(&pb.keys, &pb.keys_bytes, (size_t)nk * 2 * sizeof(uint32_t));
  rc = rc ? rc : grow(&pb.vals, &pb.vals_bytes, (size_t)nk * 2 * sizeof(int32_t));
  rc = rc ? rc : grow(&pb.hist, &pb.hist_bytes, (size_t)RS_BINS * (nblocks + 1) * 4);
  rc = rc ? rc : grow(&pb.cperm, &pb.cperm_bytes, (size_t)std::max<int32_t>(m, 1) * 4);
  rc = rc ? rc : grow(&pb.cen_feat, &pb.cen_feat_bytes,
                      (size_t)ncols_pad * (KPC * EB + 2 * sizeof(float)));
  rc = rc ? rc : grow(&pb.tbox, &pb.tbox_bytes, (size_t)TROWS * ntiles * sizeof(float));
  rc = rc ? rc : grow(&pb.fkeys, &pb.fkeys_bytes, (size_t)(n + 1) * sizeof(unsigned long long));
  // shared overflow list (its counter sits after the per-fiber keys): 32
  // entries per fiber (256 bytes, a fiber record's size), enough for the
  // loose fp8 bound on large subjects (19 survivors per fiber at 10M x 20k)
  const int64_t ovf_cap = std::min<int64_t>(std::max<int64_t>(32 * n, (int64_t)1 << 20),
                                            (int64_t)1 << 30);
  rc = rc ? rc : grow(&pb.list, &pb.list_bytes,
                      (size_t)nwaves * (CULL_QCAP * sizeof(int2) + sizeof(uint32_t)) +
                          (size_t)ovf_cap * sizeof(int2));
  if (rc) return rc;
  if (!pb.emax && hipMalloc((void**)&pb.emax, sizeof(PfParams)) != hipSuccess) return -3;
  PfParams* prm = (PfParams*)pb.emax;
  uint4* pay = (uint4*)pb.fib_feat;
  uint8_t* cfeat = (uint8_t*)pb.cen_feat;
  float* cbias = (float*)(cfeat + (size_t)ncols_pad * KPC * EB);
  int32_t* ccent = (int32_t*)(cbias + ncols_pad);
  uint32_t* keys_a = (uint32_t*)pb.keys;
  uint32_t* keys_b = keys_a + nk;
  int32_t* vals_a = (int32_t*)pb.vals;
  int32_t* vals_b = vals_a + nk;
  int32_t* cperm = (int32_t*)pb.cperm;
  uint32_t* hist = (uint32_t*)pb.hist;
  if (launch_pf_setup(prm, cprep, m, s)) return -1;
  // fibers: payloads and cell keys in input order, then the sort
  unsigned long long* fkeys = (unsigned long long*)pb.fkeys;
  unsigned long long* ovf_count = fkeys + n;
  {
    const int64_t nb = (n + CF_BLOCK - 1) / CF_BLOCK, g = cf_grid<Q>();
    cull_fiber_kernel<Q><<<(unsigned)(nb < g ? nb : g), CF_BLOCK, 0, s>>>(fibers, n, prm, pay,
                                                                          keys_a, fkeys);
  }
  if (radix_sort(n, keys_a, keys_b, vals_a, vals_b, hist, nullptr, nullptr, s)) return -1;
  // centroids: cell keys and sort (unless the prepared atlas holds the
  // order), then sorted columns with tile boxes
  if (m > 0 && !cperm_cached) {
    cell_key_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(cprep, m, CREC, prm, keys_a);
    if (radix_sort(m, keys_a, keys_b, vals_a, cperm, hist, nullptr, nullptr, s)) return -1;
  }
  cull_column_kernel<Q><<<(unsigned)((ncols_pad + 255) / 256), 256, 0, s>>>(
      cprep, m, ncols_pad, cperm_cached ? cperm_cached : cperm, prm, cfeat, cbias, ccent,
      (float*)pb.tbox);
  fill_u64_n_kernel<<<1, 64, 0, s>>>(ovf_count, 1, 0ull);
  int2* list = (int2*)pb.list;
  int2* ovf = list + nwaves * CULL_QCAP;
  uint32_t* list_n = (uint32_t*)(ovf + ovf_cap);
  const CullJob job{pay, vals_b, prm, cfeat, cbias, ccent, (const float*)pb.tbox, ntiles, fibers,
                    n, cprep, fkeys, list, list_n, ovf, ovf_count, ovf_cap};
  const unsigned blocks = (unsigned)(n_pad / 256);
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return -1;
  if (counters)
    cull_kernel<Q, true><<<blocks, 256, 0, s>>>(job, counters);
  else
    cull_kernel<Q, false><<<blocks, 256, 0, s>>>(job, counters);
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return -1;
  const MultiOut mout = mo ? *mo : MultiOut{nullptr, 0, nullptr, nullptr};
  auto exact = [&](auto stats, auto multi) {
    constexpr bool ST = decltype(stats)::value, MU = decltype(multi)::value;
    exact_list_kernel<ST, CULL_QCAP, MU><<<blocks, 256, 0, s>>>(
        list, list_n, nwaves, ovf, ovf_count, ovf_cap, vals_b, n, fibers, cprep, fkeys, counters,
        mt, mout);
    rescue_kernel<ST, MU><<<blocks < 1024u ? blocks : 1024u, 256, 0, s>>>(
        list_n, nwaves, vals_b, n, fibers, cprep, m, fkeys, counters, mt, mout);
  };
  using T = std::true_type;
  using F = std::false_type;
  if (counters)
    mo ? exact(T{}, T{}) : exact(T{}, F{});
  else
    mo ? exact(F{}, T{}) : exact(F{}, F{});
  if (!mo)
    finalize_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(fkeys, n, bid, labels, dists,
                                                                mt.flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int run_cull(int q, const float* fibers, int64_t n, const float* cprep, int32_t m,
             const int32_t* bid, int32_t* labels, float* dists, unsigned long long* counters,
             Metric mt, PrefilterBuf& pb, hipEvent_t* ev, hipStream_t s, const MultiOut* mo,
             const int32_t* cperm) {
  if (n <= 0) return 0;
  if (n >= ((int64_t)1 << 31)) return -4;  // sorted rows are indexed with 32 bits
  switch (q) {
    case 0: return cull_launch<Q_BF16>(fibers, n, cprep, m, bid, labels, dists, counters, mt, pb, ev, s, mo, cperm);
    case 1: return cull_launch<Q_F16>(fibers, n, cprep, m, bid, labels, dists, counters, mt, pb, ev, s, mo, cperm);
    case 2: return cull_launch<Q_FP8>(fibers, n, cprep, m, bid, labels, dists, counters, mt, pb, ev, s, mo, cperm);
    default: return -2;
  }
}

int cull_sort_centroids(const float* cprep, int32_t m, int32_t* cperm_out, PrefilterBuf& pb,
                        hipStream_t s) {
  if (m <= 0) return 0;
  const int64_t nblocks = (m + RS_IPB - 1) / RS_IPB;
  int rc = grow(&pb.keys, &pb.keys_bytes, (size_t)m * 2 * sizeof(uint32_t));
  rc = rc ? rc : grow(&pb.vals, &pb.vals_bytes, (size_t)m * 2 * sizeof(int32_t));
  rc = rc ? rc : grow(&pb.hist, &pb.hist_bytes, (size_t)RS_BINS * (nblocks + 1) * 4);
  if (rc) return rc;
  if (!pb.emax && hipMalloc((void**)&pb.emax, sizeof(PfParams)) != hipSuccess) return -3;
  PfParams* prm = (PfParams*)pb.emax;
  uint32_t* keys_a = (uint32_t*)pb.keys;
  int32_t* vals_a = (int32_t*)pb.vals;
  if (launch_pf_setup(prm, cprep, m, s)) return -1;
  cell_key_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(cprep, m, CREC, prm, keys_a);
  if (radix_sort(m, keys_a, keys_a + m, vals_a, cperm_out, (uint32_t*)pb.hist, nullptr, nullptr, s))
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seg
