// Sorted, tile-culled MFMA prefilter with the exact stage fused in
// (symmetric feature map, K = 16).
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
// Fiber payloads (feature codes and error bound, the row constant with
// 1-byte codes; arc length and subject where needed) are computed in input
// order, four lanes per fiber, and written as whole memory lines; the culled
// kernel gathers its rows through the permutation.
//
// Work per wave (64 consecutive sorted rows = 2 groups of 32; the four
// waves of a block run independently):
//   A. the union box of the wave's rows (widened by their largest error
//      bound) is tested against the boxes of the super-tiles (8 tiles of 32
//      columns), then against the tiles of the passing super-tiles, one
//      tile per lane; passing tiles go to an LDS list, 256 per round;
//   B. for each listed tile, the MFMA bound on its products with each group
//      (group 1 only when it holds a row), the columns of the next three
//      tiles loading meanwhile; pairs at or above the column constant go to
//      the wave's LDS survivor queue;
//   C. the exact float32 stage on the queued pairs (when the queue fills and
//      at the end), four lanes per pair, each lane taking the point pairs
//      (i, 20 - i) of three values of i; accepted pairs fold into the
//      per-row argmin keys in LDS;
//   D. each row with an accepted centroid writes its label and distance (the
//      fiber kernel wrote -1 / +inf to every fiber before).
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <atomic>
#include <cstring>

#include "seg_device.hpp"
#include "seg_graph.hpp"
#include "seg_internal.hpp"
#include "seg_pf.hpp"

namespace seg {

namespace {

constexpr int CELL_AXIS_BITS = 5;
constexpr int KPC = 16;                // feature width of the culled path
constexpr int BOXD = KPC;              // boxed feature dimensions
constexpr int TROWS = 2 * BOXD + 1;    // tile box rows: lo[16], hi[16], radius
constexpr float GAP_SLACK = 1.0f + 0x1p-17f;

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
  const int32_t bx = (int32_t)blockIdx.x;
  s_cnt[tid] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)bx * RS_IPB;
  uint32_t kr[RS_IPB / RS_THREADS];
#pragma unroll
  for (int j = 0; j < RS_IPB / RS_THREADS; ++j) {
    const int64_t i = base + (int64_t)j * RS_THREADS + tid;
    kr[j] = i < n ? keys[i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < RS_IPB / RS_THREADS; ++j)
    if (base + (int64_t)j * RS_THREADS + tid < n) atomicAdd(&s_cnt[digit_of(kr[j], shift)], 1u);
  __syncthreads();
  hist[(int64_t)tid * nblocks + bx] = s_cnt[tid];
}

// Block-wide exclusive scan of one value per thread (256 threads); returns
// the exclusive prefix and the total in *tot.  Each wave scans its 64 values
// with lane shuffles, then one exchange of the four wave totals through LDS.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp,
                                                          uint32_t* tot) {
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_tmp[w] = x;
  __syncthreads();
  uint32_t pre = 0, all = 0;
#pragma unroll
  for (int k = 0; k < RS_THREADS / 64; ++k) {
    const uint32_t t = s_tmp[k];
    pre += k < w ? t : 0u;
    all += t;
  }
  *tot = all;
  __syncthreads();  // s_tmp may be rewritten after this
  return pre + x - v;
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
// every block from the totals, so each digit's run of the block is written
// contiguously.
// (block bx of the scatter, with its LDS in `L`; also run by blocks of a
// launch that carries other work beside it)
struct ScatterLds {
  uint32_t cnt[RS_THREADS / 64][RS_BINS];
  uint32_t lstart[RS_BINS];
  uint32_t gstart[RS_BINS];
  uint32_t tmp[RS_THREADS];
  uint32_t key[RS_IPB];
  int32_t val[RS_IPB];
};
__device__ __forceinline__ void rs_scatter_block(
    int32_t bx, const uint32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in,
    int64_t n, int shift, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dtot,
    int32_t nblocks, uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out,
    ScatterLds& L) {
  constexpr int WAVES = RS_THREADS / 64;
  auto& s_cnt = L.cnt;
  auto& s_lstart = L.lstart;
  auto& s_gstart = L.gstart;
  auto& s_tmp = L.tmp;
  auto& s_key = L.key;
  auto& s_val = L.val;
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  for (int w = 0; w < WAVES; ++w) s_cnt[w][tid] = 0u;
  const int64_t bstart = (int64_t)bx * RS_IPB;
  const int64_t wb = bstart + (int64_t)wave * RS_IPW;
  // the wave's keys and values, all loads in flight at once (the ranking
  // below depends on LDS state round by round, so loads issued there would
  // each wait a full memory latency)
  uint32_t kr[RS_ROUNDS];
  int32_t vr[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = wb + r * 64 + lane;
    kr[r] = i < n ? keys_in[i] : 0u;
    vr[r] = i < n ? (vals_in ? vals_in[i] : (int32_t)i) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = wb + r * 64 + lane;
    if (i < n) atomicAdd(&s_cnt[wave][digit_of(kr[r], shift)], 1u);
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
    s_gstart[d] = dstart + hist[(int64_t)d * nblocks + bx];
    for (int w = 0; w < WAVES; ++w) {
      s_cnt[w][d] = l;
      l += c[w];
    }
  }
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = wb + r * 64 + lane;
    const bool valid = i < n;
    const uint32_t key = kr[r];
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
      s_val[start + rank] = vr[r];
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
  }
}
__global__ __launch_bounds__(RS_THREADS) void rs_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in, int64_t n,
    int shift, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dtot,
    int32_t nblocks, uint32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out) {
  __shared__ ScatterLds L;
  rs_scatter_block((int32_t)blockIdx.x, keys_in, vals_in, n, shift, hist, dtot, nblocks, keys_out,
                   vals_out, L);
}

// Center-cell keys of fibers (stride NF) or prepared centroids (stride CREC).
__global__ __launch_bounds__(256) void cell_key_kernel(const float* __restrict__ recs, int64_t n,
                                                       int32_t stride,
                                                       const PfParams* __restrict__ prm,
                                                       uint32_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = center_cell(recs + i * stride, prm);
}

// Per-fiber payload in input (row) order, as arrays that the fiber kernel
// writes whole (a partial memory line costs a read-modify-write) and the
// culled kernel gathers a row at a time:
//   codes  the quantised feature codes, 16 x the code size.  Feature 15 of
//          the symmetric map is zero; with 2-byte codes its slot holds the
//          row's error bound |Xq - X| instead, as an fp16 value rounded up
//          (+inf for a row that bypasses the cut), so a row is one 32-byte
//          read and the culled kernel derives -Ha from the codes itself
//   cst    (-Ha, error bound) for 1-byte codes
//   ext    (arc length, subject, index within the subject, 0) with the
//          length-normalised metric or in a batch (`ext_on`)
// A fiber with a non-finite coordinate gets -Ha = +inf (it bypasses the cut),
// error bound +inf (its box is unbounded) and zero codes.  The arc length is
// that of arc_length.
struct Payload {
  uint8_t* codes;
  float2* cst;
  float4* ext;
  int ext_on;
};
constexpr size_t PAY_BYTES = 32 + 8 + 16;  // per row, the largest layout

// The payload arrays carved from one allocation of rows * PAY_BYTES.
inline Payload payload_of(void* base, int64_t rows, bool ext_on) {
  Payload p;
  p.codes = (uint8_t*)base;
  p.cst = (float2*)(p.codes + (size_t)rows * 32);
  p.ext = (float4*)(p.cst + rows);
  p.ext_on = ext_on ? 1 : 0;
  return p;
}

// Order the wave's LDS writes before its later LDS reads (lanes read what
// other lanes of the same wave wrote).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Four lanes per fiber (a quad); a block takes batches of CF_FIB fibers
// (grid-stride, as many blocks as the device holds at once).  Lane s of the
// quad loads and quantises feature group s of the symmetric map: s = 0 the
// center point (features 0-2, and the zero feature 15), s = 1, 2, 3 the point
// pairs (7, 13), (4, 16), (0, 20) (features 3-6, 7-10, 11-14), each feature
// with the same double arithmetic as quantise_row.  The quad adds its partial
// sums (|Xq|^2, |Xq - X|^2, |X|^2) with two lane permutations, the same sums
// in every lane, and every lane derives the row constant and the error bound
// from them; lane s then stores codes 4s .. 4s+3 (its own and the first of
// lane s + 1), so the quad writes the code words whole.  Each wave takes 16
// fibers of a batch: their records (4032 bytes in a row) come in with
// coalesced 16-byte loads into registers, issued one batch ahead, and go
// through the wave's part of LDS to the lanes that need them.  Lane 0 writes
// the cell key, lanes 1 and 2 the empty result (-1, +inf) when `labels` is
// not null, lane 2 the row constants (with 1-byte codes) and the extra word
// (arc length, from the record in LDS, and subject).
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f4v __attribute__((ext_vector_type(4)));  // 16-byte aligned
// one point: exactly 12 bytes (a three-element vector type would load 16)
struct Pt3 {
  float x, y, z;
};
constexpr int CF_FIB = 64;              // fibers per block and batch
constexpr int CF_THREADS = 4 * CF_FIB;  // four lanes each

// One subject of a batch as the kernels see it.
struct SubDev {
  const float* fibers;  // [n][21][3]
  int64_t n;
  int64_t row0;         // its first row among the rows of the batch
  int64_t blk0;         // its first CF_FIB batch of the payload kernel
};

// Where the fibers of payload batch b come from.  One subject: fibers
// [b * CF_FIB, ...) of `fibers`.  A batch of subjects (`subs`, ascending
// blk0): subject `cur`, which the caller keeps current as b grows (SubCursor).
struct BatchSrc {
  const float* src;  // first record
  int cnt;           // records (at most CF_FIB)
  int64_t row;       // row of the first record (payload, keys)
  int64_t local;     // index of the first record within its subject
  int32_t sub;       // subject
};

// The subject of a growing batch index: found by bisection once, then
// advanced one subject at a time (a block's batches only increase), so a
// batch costs no dependent loads.
struct SubCursor {
  int32_t cur;
  SubDev sd;
  int64_t next;  // first batch of subject cur + 1

  __device__ void seek(int64_t b, const SubDev* __restrict__ subs, int32_t nsub) {
    int32_t lo = 0, hi = nsub - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (subs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
    }
    set(lo, subs, nsub);
  }
  __device__ void set(int32_t c, const SubDev* __restrict__ subs, int32_t nsub) {
    cur = c;
    sd = subs[c];
    next = c + 1 < nsub ? subs[c + 1].blk0 : INT64_MAX;
  }
  __device__ void advance(int64_t b, const SubDev* __restrict__ subs, int32_t nsub) {
    while (b >= next) set(cur + 1, subs, nsub);
  }
};

template <bool BATCH>
__device__ __forceinline__ BatchSrc batch_src(int64_t b, const float* __restrict__ fibers,
                                              int64_t n, const SubCursor& sc) {
  BatchSrc r;
  if (!BATCH) {
    r.local = b * CF_FIB;
    r.row = r.local;
    r.sub = 0;
    r.src = fibers + r.local * NF;
    r.cnt = (int)(n - r.local < CF_FIB ? n - r.local : CF_FIB);
  } else {
    r.local = (b - sc.sd.blk0) * CF_FIB;
    r.row = sc.sd.row0 + r.local;
    r.sub = sc.cur;
    r.src = sc.sd.fibers + r.local * NF;
    r.cnt = (int)(sc.sd.n - r.local < CF_FIB ? sc.sd.n - r.local : CF_FIB);
  }
  return r;
}

struct FiberOut {
  Payload pay;
  uint32_t* keys;      // [rows] cell
  int32_t* labels;     // one subject: [n] or null
  float* dists;        // one subject: [n] or null
  // a batch of subjects
  const SubDev* subs;
  int32_t nsub;
  int64_t nblk;               // payload batches of all subjects
  int32_t* const* out_lab;    // [nsub * na]: subject s against atlas a at s * na + a
  float* const* out_dst;
  int32_t na;
};

// Sum of a double over the four lanes of each quad (every lane gets the same
// value: the two additions are commutative).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double quad_sum(double v) {
  v = v + dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]
  return v + dpp_f64<0x4E>(v);  // quad_perm [2,3,0,1]
}

template <int Q, bool BATCH, bool TN>
__global__ __launch_bounds__(CF_THREADS) void cull_fiber_kernel(const float* __restrict__ fibers,
                                                                int64_t n,
                                                                PfParams* __restrict__ prm,
                                                                FiberOut fo) {
  using T = QTraits<Q>;
  constexpr int EB = T::bytes;
  constexpr int SIDE = 1 << CELL_AXIS_BITS;
  constexpr int WF = 16;            // fibers per wave and batch
  constexpr int WV = WF * NF / 4;   // their 16-byte words
  __shared__ __attribute__((aligned(16))) float s_rec[CF_THREADS / 64][WF * NF];
  const int tid = (int)threadIdx.x;
  const int sl = tid & 3;   // feature group of this lane
  const int fb = tid >> 2;  // fiber within the batch
  const int lane = tid & 63, wv = tid >> 6;
  const int fq = lane >> 2;  // fiber within the wave's 16
  float* const srec = s_rec[wv];
  const int64_t nb = BATCH ? fo.nblk : (n + CF_FIB - 1) / CF_FIB;
  // the frame and the cell grid, once
  const Frame fr = frame(prm, Q);
  float clo[3], csc[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    clo[d] = unord(prm->lo[d]);
    const float ext = unord(prm->hi[d]) - clo[d];
    csc[d] = (float)SIDE / (ext > 0.0f ? ext : 1.0f);
  }
  // this lane's points: i and its partner 20 - i (the center point twice)
  const int pi = sl == 0 ? CTR : SymGroups<KPC>::grp(sl);
  const int pj = NP - 1 - pi;
  const double g = gamma_acc(KPC);
  float e32 = 0.0f;
  SubCursor cursor{};
  // the records of this wave's fibers of batch bs: full 16-byte words into
  // registers (a partial last record's tail words are read when staged)
  f4u v[4];
  auto wave_cnt = [&](const BatchSrc& bs) {
    const int c = bs.cnt - WF * wv;
    return c < 0 ? 0 : (c > WF ? WF : c);
  };
  auto load = [&](const BatchSrc& bs) {
    const float* src = bs.src + (int64_t)WF * wv * NF;
    const int n4 = (wave_cnt(bs) * NF) >> 2;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = lane + 64 * u;
      if (i < n4) v[u] = *(const f4u*)(src + 4 * i);
    }
  };
  BatchSrc bs{};
  if ((int64_t)blockIdx.x < nb) {
    if (BATCH) cursor.seek(blockIdx.x, fo.subs, fo.nsub);
    bs = batch_src<BATCH>(blockIdx.x, fibers, n, cursor);
    load(bs);
  }
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const BatchSrc cur = bs;
    {
      const int nfl = wave_cnt(cur) * NF, n4 = nfl >> 2;
      const float* src = cur.src + (int64_t)WF * wv * NF;
      wave_lds_sync();  // the previous batch's reads are done
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = lane + 64 * u;
        if (i < n4) *(f4v*)(srec + 4 * i) = v[u];
      }
      if (lane < nfl - 4 * n4) srec[4 * n4 + lane] = src[4 * n4 + lane];
      wave_lds_sync();
    }
    if (b + gridDim.x < nb) {  // the next batch's loads, in flight meanwhile
      if (BATCH) cursor.advance(b + gridDim.x, fo.subs, fo.nsub);
      bs = batch_src<BATCH>(b + gridDim.x, fibers, n, cursor);
      load(bs);
    }
    if (fb >= cur.cnt) continue;  // the whole quad
    const float* rec = srec + fq * NF;
    const Pt3 A = *(const Pt3*)(rec + 3 * pi);
    const Pt3 B = *(const Pt3*)(rec + 3 * pj);
    // features: the center point's coordinates, or a pair's midpoint and
    // half distance (exactly as in `features`); lane 0's fourth is feature
    // 15, zero
    double x[4];
    if (sl == 0) {
      x[0] = (double)A.x - fr.o[0];
      x[1] = (double)A.y - fr.o[1];
      x[2] = (double)A.z - fr.o[2];
      x[3] = 0.0;
    } else {
      double h2 = 0.0;
      const float a3[3] = {A.x, A.y, A.z}, b3[3] = {B.x, B.y, B.z};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double a = a3[d], bb = b3[d];
        x[d] = 0.5 * (a + bb) - fr.o[d];
        h2 += (a - bb) * (a - bb);
      }
      x[3] = 0.5 * sqrt(h2);
    }
    uint32_t c[4];
    double nq = 0.0, err = 0.0, nx = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = T::enc(x[k] * fr.s);
      const double xq = T::dec(c[k]) * fr.is;  // exact (power-of-two scale)
      nq += xq * xq;
      err += (xq - x[k]) * (xq - x[k]);
      nx += x[k] * x[k];
    }
    nq = quad_sum(nq);
    err = quad_sum(err);
    nx = quad_sum(nx);
    const bool finite = __builtin_isfinite(err + nx + nq);
    // codes 4 sl .. 4 sl + 3: lane 0 its own three and lane 1's first, lane
    // s > 0 its last three and lane s + 1's first (lane 3: feature 15, zero)
    const uint32_t nxt = (uint32_t)__builtin_amdgcn_mov_dpp((int)c[0], 0xF9, 0xF, 0xF, false);
    uint32_t o0 = sl == 0 ? c[0] : c[1], o1 = sl == 0 ? c[1] : c[2];
    uint32_t o2 = sl == 0 ? c[2] : c[3], o3 = sl == 3 ? 0u : nxt;
    if (!finite) o0 = o1 = o2 = o3 = 0u;  // a bypassing row: zero codes
    float nh, er;
    if (!finite) {
      nh = __builtin_inff();
      er = __builtin_inff();
    } else {
      // the double features themselves (square roots) carry 2^-50 relative
      // error
      const double e = sqrt(err) * (1.0 + 0x1p-40) + 0x1p-50 * sqrt(nx) + 1e-30;
      const double ha = (0.5 - g) * nq * (1.0 - 0x1p-40);  // round towards passing
      nh = __double2float_ru(-ha * fr.s2);
      er = __double2float_ru(e);
      e32 = fmaxf(e32, er);
    }
    // 2-byte codes: the error bound in the slot of feature 15
    if (EB == 2 && sl == 3) o3 = (uint32_t)__half_as_ushort(__float2half_ru(er));
    const int64_t f = cur.row + fb;     // payload row
    const int64_t loc = cur.local + fb;  // index within the subject
    uint8_t* C = fo.pay.codes + f * (16 * EB);
    if (EB == 2)
      *(uint2*)(C + 8 * sl) = make_uint2(o0 | (o1 << 16), o2 | (o3 << 16));
    else
      *(uint32_t*)(C + 4 * sl) = o0 | (o1 << 8) | (o2 << 16) | (o3 << 24);
    if (sl == 0) {
      uint32_t code = 0;
      const float a3[3] = {A.x, A.y, A.z};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float t = (a3[d] - clo[d]) * csc[d];
        const int q = t >= 0.0f ? (t < (float)(SIDE - 1) ? (int)t : SIDE - 1) : 0;
        code |= spread3((uint32_t)q) << d;
      }
      fo.keys[f] = code;
    } else if (sl == 2) {
      float len = 0.0f;
      if (TN) {
        len = arc_length(rec);
      }
      if (EB == 1) fo.pay.cst[f] = make_float2(nh, er);
      if (fo.pay.ext_on)
        fo.pay.ext[f] = make_float4(len, __int_as_float(BATCH ? cur.sub : 0),
                                    __int_as_float(BATCH ? (int32_t)loc : 0), 0.0f);
    }
    if (BATCH) {
      if (sl == 1)
        for (int32_t a = 0; a < fo.na; ++a) fo.out_lab[cur.sub * fo.na + a][loc] = -1;
      else if (sl == 2)
        for (int32_t a = 0; a < fo.na; ++a) fo.out_dst[cur.sub * fo.na + a][loc] = __builtin_inff();
    } else if (fo.labels) {
      if (sl == 1) fo.labels[f] = -1;
      else if (sl == 2) fo.dists[f] = __builtin_inff();
    }
  }
  for (int off = 32; off > 0; off >>= 1) e32 = fmaxf(e32, __shfl_xor(e32, off));
  if ((tid & 63) == 0)
    atomicMax(&prm->emax_bits[(blockIdx.x * (CF_THREADS / 64) + (tid >> 6)) % EMAX_SLOTS],
              __float_as_uint(e32));
}

// Blocks of cull_fiber_kernel<Q, BATCH, TN> launched: three per compute unit
// (twelve waves), or fewer where fewer fit (queried once per process and
// kernel).  The kernel streams its reads: with more blocks in flight the
// reads and writes spread over a wider window of memory and it ran slower
// (0.230 ms at three blocks per unit against 0.238-0.248 ms at two, two and
// a half and four, with 2-byte codes at the paper's subject size).
constexpr int CF_BLOCKS_PER_CU = 3;
template <int Q, bool BATCH, bool TN>
int64_t cf_grid() {
  static std::atomic<int64_t> g{0};
  int64_t v = g.load(std::memory_order_relaxed);
  if (v == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cull_fiber_kernel<Q, BATCH, TN>,
                                                     CF_THREADS, 0) != hipSuccess ||
        cus <= 0 || per <= 0)
      return 1024;
    v = (int64_t)cus * std::min(per, CF_BLOCKS_PER_CU);
    g.store(v, std::memory_order_relaxed);
  }
  return v;
}


// Codes as order-preserving unsigned 16-bit values, two per word: 2-byte
// codes (fp16, bf16: sign and magnitude) map h to h | 0x8000 when positive
// and to ~h when negative; 1-byte codes (e4m3, one per 16-bit lane) the same
// within their low byte.
template <int EB>
__device__ __forceinline__ uint32_t ord_codes(uint32_t w) {
  if (EB == 2) {
    const uint32_t neg = (w >> 15) & 0x00010001u;
    return w ^ ((neg * 0xFFFFu) | 0x80008000u);
  } else {
    const uint32_t neg = (w >> 7) & 0x00010001u;
    return w ^ ((neg * 0xFFu) | 0x00800080u);
  }
}
template <int EB>
__device__ __forceinline__ uint32_t unord_code(uint32_t o) {
  if (EB == 2) return (o & 0x8000u) ? (o ^ 0x8000u) : (~o & 0xFFFFu);
  return (o & 0x80u) ? (o ^ 0x80u) : (~o & 0xFFu);
}
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_min_u16(uint32_t a, uint32_t b) {
  u16x2 x, y;
  __builtin_memcpy(&x, &a, 4);
  __builtin_memcpy(&y, &b, 4);
  const u16x2 r = __builtin_elementwise_min(x, y);
  uint32_t o;
  __builtin_memcpy(&o, &r, 4);
  return o;
}
__device__ __forceinline__ uint32_t pk_max_u16(uint32_t a, uint32_t b) {
  u16x2 x, y;
  __builtin_memcpy(&x, &a, 4);
  __builtin_memcpy(&y, &b, 4);
  const u16x2 r = __builtin_elementwise_max(x, y);
  uint32_t o;
  __builtin_memcpy(&o, &r, 4);
  return o;
}

// One DPP step of the packed minima and maxima (lane permutation CTRL; rows
// whose bit is clear in RMASK keep their values).
template <int CTRL, int RMASK>
__device__ __forceinline__ void dpp_pk_minmax(uint32_t* m, uint32_t* M) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp((int)m[j], (int)m[j], CTRL, RMASK, 0xF, false);
    const uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp((int)M[j], (int)M[j], CTRL, RMASK, 0xF, false);
    m[j] = pk_min_u16(m[j], a);
    M[j] = pk_max_u16(M[j], b);
  }
}

// The wave's union box from each lane's packed code minima / maxima (half 0:
// features 0-7, half 1: 8-15) and error bound: minima and maxima over each
// half wave (within rows of 16 lanes, then row 0 into 1 and row 2 into 3),
// the results of lanes 31 and 63 through LDS to lane f (lowest) and 16 + f
// (highest) of feature f, decoded and widened there by the largest error
// bound and a relative 2^-23 (one rounding each), then read out as
// wave-uniform values.  A non-finite error bound leaves the box unbounded.
template <int Q>
__device__ __forceinline__ void union_box(uint32_t* m, uint32_t* M, float emax, float isf,
                                          uint32_t* s_b, float* ulo, float* uhi) {
  constexpr int EB = QTraits<Q>::bytes;
  dpp_pk_minmax<0xB1, 0xF>(m, M);   // quad_perm [1,0,3,2]
  dpp_pk_minmax<0x4E, 0xF>(m, M);   // quad_perm [2,3,0,1]
  dpp_pk_minmax<0x124, 0xF>(m, M);  // row_ror:4
  dpp_pk_minmax<0x128, 0xF>(m, M);  // row_ror:8
  dpp_pk_minmax<0x142, 0xA>(m, M);  // row_bcast:15 into rows 1 and 3
  // the largest error bound (non-negative: its bits order as integers)
  int e = __float_as_int(emax);
  e = max(e, __builtin_amdgcn_update_dpp(e, e, 0xB1, 0xF, 0xF, false));
  e = max(e, __builtin_amdgcn_update_dpp(e, e, 0x4E, 0xF, 0xF, false));
  e = max(e, __builtin_amdgcn_update_dpp(e, e, 0x124, 0xF, 0xF, false));
  e = max(e, __builtin_amdgcn_update_dpp(e, e, 0x128, 0xF, 0xF, false));
  const int e0 = max(__builtin_amdgcn_readlane(e, 15), __builtin_amdgcn_readlane(e, 31));
  const int e1 = max(__builtin_amdgcn_readlane(e, 47), __builtin_amdgcn_readlane(e, 63));
  const float er = __int_as_float(max(e0, e1));
  const int lane = (int)lane_id();
  if ((lane & 31) == 31) {
    const int h = lane >> 5;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      s_b[4 * h + j] = m[j];      // 16-bit values of features 8h + 2j, 8h + 2j + 1
      s_b[8 + 4 * h + j] = M[j];
    }
  }
  wave_lds_sync();
  const uint32_t o = ((const unsigned short*)s_b)[lane & 31];
  const float x = QTraits<Q>::decf(unord_code<EB>(o)) * isf;  // exact
  float v;
  if ((lane & 31) < 16) {
    const float l = x - er;
    v = l - fabsf(l) * 0x1p-23f - 0x1p-126f;
    if (!(er < __builtin_inff())) v = -__builtin_inff();
  } else {
    const float h = x + er;
    v = h + fabsf(h) * 0x1p-23f + 0x1p-126f;
    if (!(er < __builtin_inff())) v = __builtin_inff();
  }
  const int vi = __float_as_int(v);
#pragma unroll
  for (int k = 0; k < BOXD; ++k) {
    ulo[k] = __int_as_float(__builtin_amdgcn_readlane(vi, k));
    uhi[k] = __int_as_float(__builtin_amdgcn_readlane(vi, 16 + k));
  }
}

// Lowest / highest over the 32 lanes of each half wave.
// One DPP step of a minimum (MAX false) or maximum over lanes: each lane
// whose row is in RMASK combines its value with the lane CTRL names.
template <int CTRL, int RMASK, bool MAX>
__device__ __forceinline__ float dpp_minmax(float v) {
  const float o = __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, RMASK, 0xF, false));
  return MAX ? fmaxf(v, o) : fminf(v, o);
}
// Minimum or maximum over each half wave (32 lanes), complete in lanes 31 and
// 63: within quads, then rows of 16 (row rotations by 4 and 8), then row 0
// (2) into row 1 (3) by row_bcast:15.  No LDS traffic, unlike shuffles.
template <bool MAX>
__device__ __forceinline__ float half_wave_minmax(float v) {
  v = dpp_minmax<0xB1, 0xF, MAX>(v);   // quad_perm [1,0,3,2]
  v = dpp_minmax<0x4E, 0xF, MAX>(v);   // quad_perm [2,3,0,1]
  v = dpp_minmax<0x124, 0xF, MAX>(v);  // row_ror:4
  v = dpp_minmax<0x128, 0xF, MAX>(v);  // row_ror:8
  return dpp_minmax<0x142, 0xA, MAX>(v);  // row_bcast:15 into rows 1 and 3
}
// The box of each half wave's 32 columns (and its largest radius), complete
// in the half's last lane.
__device__ __forceinline__ void half_wave_box(float* lo, float* hi, float* r2) {
#pragma unroll
  for (int k = 0; k < BOXD; ++k) {
    lo[k] = half_wave_minmax<false>(lo[k]);
    hi[k] = half_wave_minmax<true>(hi[k]);
  }
  *r2 = half_wave_minmax<true>(*r2);
}

// Sorted columns: column j is centroid cperm[j]; each half wave writes the
// box and largest radius of its tile of 32 columns, and each block (8 tiles)
// the box and largest radius of its super-tile (struct of arrays, row-major
// [TROWS][ntiles] and [TROWS][nsuper]).
constexpr int SUPER = 8;  // tiles per super-tile (one column block)
template <int Q>
__device__ __forceinline__ void column_block(int32_t bx, int32_t nsuper, const float* __restrict__ cprep,
                                                          int32_t m, int32_t ncols_pad,
                                                          const int32_t* __restrict__ cperm,
                                                          const PfParams* __restrict__ prm,
                                                          uint8_t* __restrict__ feat,
                                                          float* __restrict__ cb,
                                                          int32_t* __restrict__ ccent,
                                                          float* __restrict__ csort,
                                                          float* __restrict__ tbox,
                                                          float* __restrict__ sbox,
                                                          float (*s_t)[TROWS]) {
  using T = QTraits<Q>;
  const int32_t col = bx * 256 + (int32_t)threadIdx.x;
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
      const float* rec = cprep + (int64_t)c * CREC;
      cb[col] = column_row<Q, MAP_SYM, KPC, true>(rec, false, prm, row, lo, hi, &r2);
      // the record in column order, for the exact stage, in two halves
      // whose eight loads are all issued before their stores (left to
      // itself the compiler pairs each load with its store and waits for
      // every load in turn).  The empty asm (no instruction) takes the eight
      // values, so the loads come before it and the stores after it.
      const f4v* src = (const f4v*)rec;
      f4v* dst = (f4v*)(csort + (int64_t)col * CREC);
      f4v rv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) rv[k] = src[k];
      asm volatile("" ::"v"(rv[0]), "v"(rv[1]), "v"(rv[2]), "v"(rv[3]), "v"(rv[4]), "v"(rv[5]),
                   "v"(rv[6]), "v"(rv[7]), "v"(rv[8]), "v"(rv[9]), "v"(rv[10]), "v"(rv[11]),
                   "v"(rv[12]), "v"(rv[13]), "v"(rv[14]), "v"(rv[15])
                   : "memory");
#pragma unroll
      for (int k = 0; k < 16; ++k) dst[k] = rv[k];
    }
  }
  half_wave_box(lo, hi, &r2);
  const int32_t tile = col >> 5;
  const int32_t ntiles = ncols_pad >> 5;
  const int h = (int)(threadIdx.x >> 5);  // tile within the block
  if ((threadIdx.x & 31) == 31) {  // the half's last lane holds its box
#pragma unroll
    for (int k = 0; k < BOXD; ++k) {
      s_t[h][k] = lo[k];
      s_t[h][BOXD + k] = hi[k];
    }
    s_t[h][2 * BOXD] = r2 * GAP_SLACK;
    if (tile < ntiles) {
#pragma unroll
      for (int k = 0; k < BOXD; ++k) {
        tbox[(int64_t)k * ntiles + tile] = lo[k];
        tbox[(int64_t)(BOXD + k) * ntiles + tile] = hi[k];
      }
      tbox[(int64_t)(2 * BOXD) * ntiles + tile] = r2 * GAP_SLACK;
    }
  }
  __syncthreads();
  if (threadIdx.x < TROWS) {
    const int k = (int)threadIdx.x;
    float v = s_t[0][k];
    for (int j = 1; j < SUPER; ++j)
      v = k < BOXD ? fminf(v, s_t[j][k]) : fmaxf(v, s_t[j][k]);
    sbox[(int64_t)k * nsuper + bx] = v;
  }
}

// Arguments of the column blocks.
struct ColArgs {
  const float* cprep;
  int32_t m, ncols_pad, nsuper;
  const int32_t* cperm;
  const PfParams* prm;
  uint8_t* feat;
  float* cb;
  int32_t* ccent;
  float* csort;
  float* tbox;
  float* sbox;
};

template <int Q>
__global__ __launch_bounds__(256) void cull_column_kernel(ColArgs ca) {
  __shared__ float s_t[SUPER][TROWS];
  column_block<Q>((int32_t)blockIdx.x, ca.nsuper, ca.cprep, ca.m, ca.ncols_pad, ca.cperm, ca.prm,
                  ca.feat, ca.cb, ca.ccent, ca.csort, ca.tbox, ca.sbox, s_t);
}

// The columns of up to COL_MAX atlases (blocks [first[i], first[i + 1]) for
// atlas i: the longer work, dispatched first) and the first scatter of the
// fibers' sort (the remaining nb_sort blocks) in one launch: they depend on
// nothing of each other, so the small column grids, a chain of dependent
// loads and double arithmetic per column, run beside the scatter.
constexpr int COL_MAX = 4;
struct ColSet {
  ColArgs c[COL_MAX];
  int32_t first[COL_MAX + 1];
  int32_t n;
};
template <int Q>
__global__ __launch_bounds__(256) void scatter_column_kernel(
    const uint32_t* __restrict__ keys_in, int64_t n, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ dtot, int32_t nb_sort, uint32_t* __restrict__ keys_out,
    int32_t* __restrict__ vals_out, ColSet cs) {
  static_assert(RS_THREADS == 256, "one block size for both kinds of block");
  __shared__ union {
    ScatterLds sc;
    float t[SUPER][TROWS];
  } lds;  // one kind of block each: the two share the block's LDS
  const int32_t bx = (int32_t)blockIdx.x;
  if (bx < cs.first[cs.n]) {
    int i = 0;
#pragma unroll
    for (int k = 1; k < COL_MAX; ++k) i += (k < cs.n && bx >= cs.first[k]) ? 1 : 0;
    const ColArgs& ca = cs.c[i];
    column_block<Q>(bx - cs.first[i], ca.nsuper, ca.cprep, ca.m, ca.ncols_pad, ca.cperm, ca.prm,
                    ca.feat, ca.cb, ca.ccent, ca.csort, ca.tbox, ca.sbox, lds.t);
  } else {
    rs_scatter_block(bx - cs.first[cs.n], keys_in, nullptr, n, 0, hist, dtot, nb_sort, keys_out,
                     vals_out, lds.sc);
  }
}

// A chunk of at most this many subjects finds a row's subject from the
// subjects' first rows; a larger chunk (or the length-normalised metric)
// carries subject, index and arc length in the extra payload word.
constexpr int32_t BATCH_SUBS = 16;

struct CullJob {
  Payload pay;           // fiber payloads in input order
  const int32_t* perm;   // sorted position -> input index
  const PfParams* prm;   // frame (code scale)
  const uint8_t* cfeat;  // sorted columns [ncols_pad][16]
  const float* cbias;    // cb per sorted column
  const int32_t* ccent;  // centroid of each sorted column
  const float* tbox;     // tile boxes [TROWS][ntiles]
  const float* sbox;     // super-tile boxes [TROWS][nsuper]
  int32_t ntiles;
  int32_t nsuper;
  const float* fibers;   // the subject's fiber records (input order)
  int64_t n;
  const float* csort;    // the prepared records (63 coordinates + T2) in column order
  const int32_t* bid;    // bundle of each prepared centroid
  int32_t* labels;       // written for fibers with an accepted centroid
  float* dists;
  // a batch of subjects (rows of every subject, one atlas `atlas` of `na`)
  const SubDev* subs;
  int32_t* const* out_lab;  // subject s against atlas a at s * na + a
  float* const* out_dst;
  int32_t na, atlas;
  int32_t nsub;  // subjects of the chunk (with no extra payload word: at most BATCH_SUBS)
};

constexpr int CW = 4;          // waves per block (each works on its own)
constexpr int CROUND = 256;    // centroid tiles per candidate round
constexpr int CQ = 1280;       // survivor queue entries per wave
constexpr int CQ_ROOM = 1024;  // the most entries one (tile, group) product adds

// Nine consecutive floats (three points) from a 4-byte aligned address.
__device__ __forceinline__ void load9(const float* __restrict__ p, float* v) {
  const f4u a = *(const f4u*)p;
  const f4u b = *(const f4u*)(p + 4);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = a.z;
  v[3] = a.w;
  v[4] = b.x;
  v[5] = b.y;
  v[6] = b.z;
  v[7] = b.w;
  v[8] = p[8];
}

// Eq. 2 for one (fiber a, centroid b) pair, evaluated by the four lanes of a
// quad: sub-lane s takes the point pairs (i, 20 - i) for i = 3s, 3s+1, 3s+2
// (s = 3: i = 9, 10 and 11, whose pairs repeat ones of 9 and 10), i.e. the
// points 3s .. 3s+2 and 18-3s .. 20-3s of both curves, and computes for each
// i the direct distances d(a_i, b_i), d(a_j, b_j) and the inverse ones
// d(a_i, b_j), d(a_j, b_i) (j = 20 - i).  The largest distance and the
// all-within-threshold flag of each order are combined over the quad; as in
// the exact stage, an order dies on a point above T2, D is the smaller
// maximum of the live orders, and with MF_DIR only the order chosen by the
// end points (held by sub-lane 0) stays.  Every lane of the quad returns the
// same result; the maxima are exact, so the result is the one-lane result.
__device__ __forceinline__ bool quad_pair(const float* __restrict__ ar,
                                          const float* __restrict__ br, int sl, float& D,
                                          int flags) {
  float A1[9], A2[9], B1[9], B2[9];
  load9(ar + 9 * sl, A1);
  load9(ar + 54 - 9 * sl, A2);
  load9(br + 9 * sl, B1);
  load9(br + 54 - 9 * sl, B2);
  const float t2 = br[NF];
  float md = 0.0f, mi = 0.0f;
  bool ad = true, ai = true;
  float ex0 = 0.0f, ex1 = 0.0f, ey0 = 0.0f, ey1 = 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int p = 3 * k, q = 3 * (2 - k);  // point i in A1/B1, its partner 20 - i in A2/B2
    const float x = d2(A1[p], A1[p + 1], A1[p + 2], B1[p], B1[p + 1], B1[p + 2]);
    const float xj = d2(A2[q], A2[q + 1], A2[q + 2], B2[q], B2[q + 1], B2[q + 2]);
    const float y = d2(A1[p], A1[p + 1], A1[p + 2], B2[q], B2[q + 1], B2[q + 2]);
    const float yj = d2(A2[q], A2[q + 1], A2[q + 2], B1[p], B1[p + 1], B1[p + 2]);
    ad = ad && x <= t2 && xj <= t2;
    ai = ai && y <= t2 && yj <= t2;
    md = fmaxf(md, fmaxf(x, xj));
    mi = fmaxf(mi, fmaxf(y, yj));
    if (k == 0) {
      ex0 = x;
      ex1 = xj;
      ey0 = y;
      ey1 = yj;
    }
  }
  int fl = (ad ? 1 : 0) | (ai ? 2 : 0);
#pragma unroll
  for (int off = 1; off < 4; off <<= 1) {
    md = fmaxf(md, __shfl_xor(md, off));
    mi = fmaxf(mi, __shfl_xor(mi, off));
    fl &= __shfl_xor(fl, off);
  }
  ad = fl & 1;
  ai = fl & 2;
  if (flags & MF_DIR) {
    // sub-lane 0 holds the end points: i = 0 and its partner 20
    const int dl = (int)(lane_id() & ~3u);
    const bool direct = __shfl((int)(fmaxf(ex0, ex1) <= fmaxf(ey0, ey1)), dl) != 0;
    ad = ad && direct;
    ai = ai && !direct;
  }
  D = ad ? (ai ? fminf(md, mi) : md) : mi;
  return ad || ai;
}

// The tile-culled pass with the exact stage fused in; one wave per 64 sorted
// rows (see the top of this file).  With STATS the staged exact stage of the
// other paths runs on the queued pairs instead (one lane per pair), to count
// its tests; with MULTI accepted pairs go to the fibers' bundle slots.
// (five waves per SIMD, 96 registers at most, where that needs no spills;
// the block's LDS allows five blocks per compute unit)
template <int Q, bool STATS, bool MULTI, bool BATCH>
__global__ __launch_bounds__(64 * CW) __attribute__((amdgpu_waves_per_eu(STATS || MULTI ? 4 : 5))) void cull_kernel(CullJob job, Metric mt, MultiOut mo,
                                                       unsigned long long* __restrict__ counters) {
  using FT = typename Frag<Q>::T;
  constexpr int EB = QTraits<Q>::bytes;
  __shared__ __attribute__((aligned(16))) float s_nh[CW][64];  // -Ha: the MFMA C operand
  __shared__ int32_t s_idx[CW][64];                            // input index of each row
  __shared__ float s_len[CW][64];                              // arc length (MF_TN)
  __shared__ int32_t s_sub[CW][BATCH ? 64 : 1];                // subject (a batch)
  __shared__ uint32_t s_sup[CW][64];                           // passing super-tiles
  __shared__ uint32_t s_cand[CW][CROUND];                      // passing tiles
  __shared__ uint32_t s_q[CW][CQ];                             // centroid << 6 | row
  __shared__ unsigned long long s_best[CW][64];                // argmin key of each row
  __shared__ uint32_t s_box[CW][16];                           // union box (16-bit codes)
  __shared__ uint32_t s_hit[CW][STATS ? 64 : 1];               // rows with a survivor (STATS)
  const int lane = (int)(threadIdx.x & 63);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int half = lane >> 5;
  const int l31 = lane & 31;
  const int64_t n = job.n;
  const int64_t wbase = ((int64_t)blockIdx.x * CW + wave) * 64;
  if (wbase >= n) return;  // the whole wave: no block-level synchronisation follows
  const int32_t ntiles = job.ntiles;
  const bool g1 = wbase + 32 < n;  // group 1 holds a row
  StageCounts sc{counters};

  // both groups' permutation entries, then both groups' payloads, in flight
  // together; positions past n are padding rows (never pass, no box)
  FT afr[2];
  int32_t prow[2];
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int64_t p = wbase + g * 32 + l31;
    const int32_t r = job.perm[p < n ? p : n - 1];
    prow[g] = r >= 0 && r < n ? r : 0;  // (always in range; the clamp only guards the reads)
  }
  float2 cst[2] = {make_float2(0.0f, 0.0f), make_float2(0.0f, 0.0f)};  // 1-byte codes
  float4 ext[2] = {make_float4(0.0f, 0.0f, 0.0f, 0.0f), make_float4(0.0f, 0.0f, 0.0f, 0.0f)};
  const bool with_ext = job.pay.ext_on;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    afr[g] = *(const FT*)(job.pay.codes + (int64_t)prow[g] * (16 * EB) + 8 * half * EB);
    if (EB == 1) cst[g] = job.pay.cst[prow[g]];
    if (with_ext) ext[g] = job.pay.ext[prow[g]];
  }
  if (BATCH && !with_ext) {
    // a chunk of at most BATCH_SUBS subjects: the subject of a row from the
    // subjects' first rows (wave-uniform loads), no extra payload word
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      int32_t sb = 0;
      int64_t r0 = 0;
#pragma unroll
      for (int k = 1; k < BATCH_SUBS; ++k) {
        if (k < job.nsub) {
          const int64_t rk = job.subs[k].row0;
          if (prow[g] >= rk) {
            sb = k;
            r0 = rk;
          }
        }
      }
      ext[g].y = __int_as_float(sb);
      ext[g].z = __int_as_float((int32_t)(prow[g] - r0));
    }
  }
  const Frame fr = frame(job.prm, Q);
  const float isf = (float)fr.is;  // a power of two
  const double gam = gamma_acc(KPC);
  // per row: the error bound and -Ha (from the codes, as the fiber kernel
  // computes it, with 2-byte codes); the wave's largest error bound; the
  // codes as order-preserving 16-bit values, lowest and highest over the
  // wave's valid rows (padding rows take the neutral values)
  float emax = 0.0f;
  uint32_t omin[4], omax[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    omin[j] = 0xFFFFFFFFu;
    omax[j] = 0u;
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const bool valid = wbase + g * 32 + l31 < n;
    uint32_t w[4];
    float er, nh;
    if (EB == 2) {
      __builtin_memcpy(w, &afr[g], 16);
      // half 1 holds features 8-15: the slot of 15 is the error bound
      const float eh = half ? __half2float(__ushort_as_half((unsigned short)(w[3] >> 16))) : 0.0f;
      if (half) w[3] &= 0xFFFFu;
      __builtin_memcpy(&afr[g], w, 16);
      er = fmaxf(eh, __shfl_xor(eh, 32));
      double nqp = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double x = (double)(QTraits<Q>::decf((w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu) * isf);
        nqp += x * x;
      }
      const double nq = nqp + __shfl_xor(nqp, 32);  // the same in both halves
      const double ha = (0.5 - gam) * nq * (1.0 - 0x1p-40);  // round towards passing
      nh = er < __builtin_inff() ? __double2float_ru(-ha * fr.s2) : __builtin_inff();
    } else {
      er = cst[g].y;
      nh = cst[g].x;
      // eight 1-byte codes as 16-bit lanes
      uint64_t b8;
      __builtin_memcpy(&b8, &afr[g], 8);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        w[j] = (uint32_t)((b8 >> (16 * j)) & 0xFFu) | ((uint32_t)((b8 >> (16 * j + 8)) & 0xFFu) << 16);
    }
    if (half == 0) {
      // a padding row's C operand is NaN: its products are NaN and never pass
      s_nh[wave][g * 32 + l31] = valid ? nh : __builtin_nanf("");
      s_idx[wave][g * 32 + l31] = valid ? (BATCH ? __float_as_int(ext[g].z) : prow[g]) : 0;
      s_len[wave][g * 32 + l31] = ext[g].x;
      if (BATCH) s_sub[wave][g * 32 + l31] = valid ? __float_as_int(ext[g].y) : 0;
    }
    if (valid) {
      emax = fmaxf(emax, er);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t o = ord_codes<EB>(w[j]);
        omin[j] = pk_min_u16(omin[j], o);
        omax[j] = pk_max_u16(omax[j], o);
      }
    }
  }
  // wave-uniform (scalar) union box: features 0-7 from half 0, 8-15 from
  // half 1, widened by the largest error bound
  float ulo[BOXD], uhi[BOXD];
  union_box<Q>(omin, omax, emax, isf, s_box[wave], ulo, uhi);
  s_best[wave][lane] = NO_KEY;
  if (STATS) s_hit[wave][lane] = 0u;
  wave_lds_sync();

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
  // the fiber record of row `slot` (input index f)
  auto frec = [&](int slot, int32_t f) {
    const float* base = BATCH ? job.subs[s_sub[wave][slot]].fibers : job.fibers;
    return base + (int64_t)f * NF;
  };
  // an accepted pair: into the row's argmin key, or the fiber's bundle slots
  auto fold = [&](int slot, int32_t f, uint32_t c, float v) {
    if (MULTI)
      multi_insert(mo.slots + (int64_t)f * mo.K, mo.K, (uint32_t)mo.bid[c], v, mo.flag);
    else
      atomicMin(&s_best[wave][slot], (unsigned long long)make_key(v, c));
  };
  // C: the exact stage on queue entries [0, cnt)
  auto drain = [&](uint32_t cnt) {
    wave_lds_sync();
    if (STATS && lane == 0) {
      atomicAdd(counters + 0, (unsigned long long)cnt);
      atomicAdd(counters + 4, 1ull);
    }
    if constexpr (STATS) {
      for (uint32_t j0 = 0; j0 < cnt; j0 += 64) {
        const uint32_t j = j0 + lane;
        const bool act = j < cnt;
        const uint32_t e = act ? s_q[wave][j] : 0u;
        const int slot = (int)(e & 63u);
        const uint32_t col = e >> 6;
        const uint32_t c = (uint32_t)job.ccent[col];
        const int32_t f = s_idx[wave][slot];
        const float* ar = frec(slot, f);
        if (act) s_hit[wave][slot] = 1u;
        float D, v;
        const bool ok = exact_pair<true>(ar, job.csort + (size_t)col * CREC, act, D, sc, mt.flags);
        if (ok && variant_value(D, c, s_len[wave][slot], mt, v)) fold(slot, f, c, v);
      }
    } else {
      const int sl = lane & 3;
      for (uint32_t j0 = 0; j0 < cnt; j0 += 16) {
        const uint32_t j = j0 + (uint32_t)(lane >> 2);
        const bool act = j < cnt;
        const uint32_t e = act ? s_q[wave][j] : 0u;  // inactive quads read row 0, column 0
        const int slot = (int)(e & 63u);
        const uint32_t col = e >> 6;
        const uint32_t c = (uint32_t)job.ccent[col];  // (loads with the record)
        const int32_t f = s_idx[wave][slot];
        float D, v;
        const bool ok = quad_pair(frec(slot, f), job.csort + (size_t)col * CREC, sl, D, mt.flags);
        if (sl == 0 && act && ok && variant_value(D, c, s_len[wave][slot], mt, v))
          fold(slot, f, c, v);
      }
    }
    wave_lds_sync();
  };
  uint32_t qn = 0;
  // survivors of one (tile, group) product: every (row, column) at or above
  // the column constant is queued (the caller made room for 1024); padding
  // rows are NaN and never pass
  // (row r of the lane's outputs is row 8 (r / 4) + 4 half + r % 4 of the
  // group: the entry of output r is ebase + 8 (r / 4) + r % 4)
  auto extract = [&](const f32x16& a, int g, uint32_t col, float cbv) {
    const uint32_t ebase = (col << 6) | (uint32_t)(g * 32 + 4 * half);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t e = ebase + (uint32_t)(8 * (r >> 2) + (r & 3));
      const bool p = a[r] >= cbv;
      const uint64_t msk = __ballot(p);
      if (!msk) continue;
      if (p) s_q[wave][qn + bits_below(msk)] = e;
      qn += (uint32_t)__popcll(msk);
    }
  };
  auto cload = [&](uint32_t i, FT& b, float& cb, uint32_t& cn) {
    const uint32_t col = s_cand[wave][i] * 32u + (uint32_t)l31;
    b = *(const FT*)(job.cfeat + (int64_t)col * (KPC * EB) + 8 * half * EB);
    cb = job.cbias[col];
    cn = col;
  };

  // gap^2 of box row `i` of a [TROWS][cnt] struct-of-arrays table against
  // the union box; passes when it does not exceed the stored radius
  // whether box row `i` of a [TROWS][cnt] struct-of-arrays table is near the
  // union box: gap^2 not above the stored radius
  // (32-bit offsets from a wave-uniform row address: the table has at most
  // TROWS * 2^19 entries)
  auto near = [&](const float* __restrict__ box, uint32_t cnt, uint32_t i) {
    float tl[BOXD], th[BOXD];
#pragma unroll
    for (int k = 0; k < BOXD; ++k) {
      tl[k] = (box + (size_t)k * cnt)[i];
      th[k] = (box + (size_t)(BOXD + k) * cnt)[i];
    }
    const float r2 = (box + (size_t)(2 * BOXD) * cnt)[i];
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < BOXD; ++k) {
      const float g = fmaxf(fmaxf(tl[k] - uhi[k], ulo[k] - th[k]), 0.0f);
      s = __builtin_fmaf(g, g, s);
    }
    return !(s > r2);
  };
  // B: the MFMA bound on candidate tiles [0, nc), the columns of the next
  // three loading meanwhile (a ring of three); both groups (group 1 only
  // when it holds a row)
  auto products = [&](uint32_t nc) {
    wave_lds_sync();
    if (STATS && lane == 0)
      atomicAdd(counters + 5, (unsigned long long)nc * (g1 ? 2u : 1u));
    auto step = [&](const FT& b, float cbv, uint32_t col) {
      if (qn > (uint32_t)(CQ - CQ_ROOM)) {
        drain(qn);
        qn = 0;
      }
      {
        const f32x16 a = Frag<Q>::mfma(afr[0], b, negh(0));
        if (wave_any(max16(a) >= cbv)) extract(a, 0, col, cbv);
      }
      if (g1) {
        if (qn > (uint32_t)(CQ - CQ_ROOM)) {
          drain(qn);
          qn = 0;
        }
        const f32x16 a = Frag<Q>::mfma(afr[1], b, negh(1));
        if (wave_any(max16(a) >= cbv)) extract(a, 1, col, cbv);
      }
    };
    FT b0, b1, b2;
    float cb0 = 0.0f, cb1 = 0.0f, cb2 = 0.0f;
    uint32_t cn0 = 0, cn1 = 0, cn2 = 0;
    cload(0, b0, cb0, cn0);
    if (nc > 1) cload(1, b1, cb1, cn1);
    if (nc > 2) cload(2, b2, cb2, cn2);
    for (uint32_t i = 0; i < nc; i += 3) {
      step(b0, cb0, cn0);
      if (i + 3 < nc) cload(i + 3, b0, cb0, cn0);
      if (i + 1 < nc) {
        step(b1, cb1, cn1);
        if (i + 4 < nc) cload(i + 4, b1, cb1, cn1);
      }
      if (i + 2 < nc) {
        step(b2, cb2, cn2);
        if (i + 5 < nc) cload(i + 5, b2, cb2, cn2);
      }
    }
    wave_lds_sync();  // the candidate list is rewritten after this
  };

  // A: super-tiles (8 tiles) against the union box, 64 at a time; the tiles
  // of the passing ones, 8 super-tiles at a time
  const int32_t nsuper = job.nsuper;
  uint32_t nc = 0;
  for (int32_t s0 = 0; s0 < nsuper; s0 += 64) {
    const int32_t st = s0 + lane;
    const bool ps = st < nsuper && near(job.sbox, (uint32_t)nsuper, (uint32_t)st);
    const uint64_t msk = __ballot(ps);
    if (!msk) continue;
    if (ps) s_sup[wave][bits_below(msk)] = (uint32_t)st;
    const uint32_t nsup = (uint32_t)__popcll(msk);
    wave_lds_sync();
    for (uint32_t i0 = 0; i0 < nsup; i0 += 64 / SUPER) {
      const uint32_t i = i0 + (uint32_t)(lane / SUPER);
      const int32_t t = i < nsup ? (int32_t)s_sup[wave][i] * SUPER + (lane % SUPER) : ntiles;
      const bool pt = t < ntiles && near(job.tbox, (uint32_t)ntiles, (uint32_t)t);
      const uint64_t m2 = __ballot(pt);
      if (pt) s_cand[wave][nc + bits_below(m2)] = (uint32_t)t;
      nc += (uint32_t)__popcll(m2);
      if (nc > (uint32_t)(CROUND - 64)) {
        products(nc);
        nc = 0;
      }
    }
    wave_lds_sync();  // s_sup is rewritten by the next round
  }
  if (nc) products(nc);
  if (qn) drain(qn);
  if (STATS) {
    wave_lds_sync();
    const uint64_t hit = __ballot(s_hit[wave][lane] != 0u);
    if (lane == 0 && hit) atomicAdd(counters + 6, (unsigned long long)__popcll(hit));
  }
  // D: results of the rows with an accepted centroid
  if (!MULTI) {
    const unsigned long long best = s_best[wave][lane];
    if (wbase + lane < n && best != NO_KEY) {
      const int32_t f = s_idx[wave][lane];
      if (BATCH) {
        const int64_t o = (int64_t)s_sub[wave][lane] * job.na + job.atlas;
        write_result(best, job.bid, job.out_lab[o] + f, job.out_dst[o] + f, mt.flags);
      } else {
        write_result(best, job.bid, job.labels + f, job.dists + f, mt.flags);
      }
    }
  }
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

// Digit counts of one pass and their scan; the digit totals follow the
// per-block counts in `hist`.
void radix_count(int pass, int64_t n, const uint32_t* kin, uint32_t* hist, hipStream_t s) {
  const int32_t nblocks = (int32_t)((n + RS_IPB - 1) / RS_IPB);
  rs_hist_kernel<<<nblocks, RS_THREADS, 0, s>>>(kin, n, 8 * pass, hist, nblocks);
  rs_scan_rows_kernel<<<RS_BINS, RS_THREADS, 0, s>>>(hist, nblocks,
                                                     hist + (size_t)RS_BINS * nblocks);
}
// Stable sort of n keys (15 bits) into a permutation: vals_b[k] = index of
// the k-th smallest key.  keys_a holds the keys on entry; keys_b, vals_a,
// vals_b and hist (RS_BINS * nblocks + RS_BINS) are scratch.
int radix_sort(int64_t n, uint32_t* keys_a, uint32_t* keys_b, int32_t* vals_a, int32_t* vals_b,
               uint32_t* hist, hipStream_t s) {
  if (n <= 0) return 0;
  const int32_t nblocks = (int32_t)((n + RS_IPB - 1) / RS_IPB);
  uint32_t* tot = hist + (size_t)RS_BINS * nblocks;
  // pass 1: bits 0-7, input order as values; pass 2: bits 8-14
  radix_count(0, n, keys_a, hist, s);
  rs_scatter_kernel<<<nblocks, RS_THREADS, 0, s>>>(keys_a, nullptr, n, 0, hist, tot, nblocks,
                                                   keys_b, vals_a);
  radix_count(1, n, keys_b, hist, s);
  rs_scatter_kernel<<<nblocks, RS_THREADS, 0, s>>>(keys_b, vals_a, n, 8, hist, tot, nblocks,
                                                   nullptr, vals_b);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The fibers' sort (as radix_sort) with the column sets of `cs` computed
// beside its first scatter.
template <int Q>
int sort_with_columns(int64_t n, uint32_t* keys_a, uint32_t* keys_b, int32_t* vals_a,
                      int32_t* perm, uint32_t* hist, const ColSet& cs, hipStream_t s) {
  const int32_t nbs = (int32_t)((n + RS_IPB - 1) / RS_IPB);
  uint32_t* tot = hist + (size_t)RS_BINS * nbs;
  radix_count(0, n, keys_a, hist, s);
  scatter_column_kernel<Q><<<(unsigned)(cs.first[cs.n] + nbs), 256, 0, s>>>(
      keys_a, n, hist, tot, nbs, keys_b, vals_a, cs);
  radix_count(1, n, keys_b, hist, s);
  rs_scatter_kernel<<<nbs, RS_THREADS, 0, s>>>(keys_b, vals_a, n, 8, hist, tot, nbs, nullptr,
                                               perm);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Sort scratch for up to nk keys: keys (two buffers), values (two buffers;
// the second is the permutation) and the digit counts.
int grow_sort(PrefilterBuf& pb, int64_t nk) {
  const int64_t nblocks = (nk + RS_IPB - 1) / RS_IPB;
  int rc = grow(&pb.keys, &pb.keys_bytes, (size_t)nk * 2 * sizeof(uint32_t));
  rc = rc ? rc : grow(&pb.vals, &pb.vals_bytes, (size_t)nk * 2 * sizeof(int32_t));
  rc = rc ? rc : grow(&pb.hist, &pb.hist_bytes, (size_t)RS_BINS * (nblocks + 1) * 4);
  return rc;
}

// Centroid order for up to RANK_MAX centroids by counting ranks: with the
// unique composite keys c = cell << 15 | index (their order is the stable
// order by cell), the sorted position of centroid i is the number of c below
// its own.  rank_count_kernel: block (x, y) counts, for its 256 centroids i,
// the c of centroid tile y (RANK_TILE of them, staged in LDS) below c_i, into
// part[y][i]; rank_place_kernel adds the parts and writes cperm[pos] = i.
// Plain integer sums, so the order is deterministic.
constexpr int RANK_MAX = 16384;
constexpr int RANK_TILE = 256;
__device__ __forceinline__ uint32_t comp_key(const float* __restrict__ cprep, int32_t i,
                                             const PfParams* __restrict__ prm) {
  return (center_cell(cprep + (int64_t)i * CREC, prm) << 15) | (uint32_t)i;
}
__global__ __launch_bounds__(256) void rank_count_kernel(const float* __restrict__ cprep, int32_t m,
                                                         const PfParams* __restrict__ prm,
                                                         uint32_t* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint32_t s_c[RANK_TILE];
  const int tid = (int)threadIdx.x;
  const int32_t j0 = (int32_t)blockIdx.y * RANK_TILE;
  for (int k = tid; k < RANK_TILE; k += 256) {
    const int32_t j = j0 + k;
    s_c[k] = j < m ? comp_key(cprep, j, prm) : 0xFFFFFFFFu;  // past m: above every key
  }
  const int32_t i = (int32_t)blockIdx.x * 256 + tid;
  const uint32_t ci = i < m ? comp_key(cprep, i, prm) : 0u;
  __syncthreads();
  uint32_t cnt = 0;
#pragma unroll 8
  for (int k = 0; k < RANK_TILE; k += 4) {
    const uint4 v = *(const uint4*)&s_c[k];
    cnt += (v.x < ci) + (v.y < ci) + (v.z < ci) + (v.w < ci);
  }
  if (i < m) part[(int64_t)blockIdx.y * m + i] = cnt;
}
__global__ __launch_bounds__(256) void rank_place_kernel(const uint32_t* __restrict__ part,
                                                         int32_t m, int32_t tiles,
                                                         int32_t* __restrict__ cperm) {
  const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (i >= m) return;
  uint32_t pos = 0;
#pragma unroll 8
  for (int32_t y = 0; y < tiles; ++y) pos += part[(int64_t)y * m + i];
  cperm[pos] = i;  // pos < m: the c are distinct
}

// Centroid order: by counting ranks for up to RANK_MAX centroids, else cell
// keys of the prepared records and the radix sort.
int sort_centroids(const float* cprep, int32_t m, const PfParams* prm, PrefilterBuf& pb, int64_t nk,
                   int32_t* cperm, hipStream_t s) {
  if (m <= RANK_MAX) {
    const int32_t tiles = (m + RANK_TILE - 1) / RANK_TILE;
    if (grow(&pb.rank, &pb.rank_bytes, (size_t)tiles * m * sizeof(uint32_t))) return -3;
    uint32_t* part = (uint32_t*)pb.rank;
    rank_count_kernel<<<dim3((unsigned)((m + 255) / 256), (unsigned)tiles), 256, 0, s>>>(
        cprep, m, prm, part);
    rank_place_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(part, m, tiles, cperm);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  uint32_t* keys_a = (uint32_t*)pb.keys;
  int32_t* vals_a = (int32_t*)pb.vals;
  cell_key_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(cprep, m, CREC, prm, keys_a);
  return radix_sort(m, keys_a, keys_a + nk, vals_a, cperm, (uint32_t*)pb.hist, s);
}

// The frame of a prepared atlas (its box, as order-preserving integers) kept
// after its centroid order: saved once, loaded by each call in place of the
// box reduction, with the fiber error slots reset as a fresh frame has them.
__global__ void frame_save_kernel(const PfParams* __restrict__ prm, int* __restrict__ out) {
  const int t = (int)threadIdx.x;
  if (t < 3) {
    out[t] = prm->lo[t];
    out[3 + t] = prm->hi[t];
  }
}
__global__ void frame_load_kernel(PfParams* __restrict__ prm, const int* __restrict__ in) {
  const int t = (int)threadIdx.x;
  if (t < 3) {
    prm->lo[t] = in[t];
    prm->hi[t] = in[3 + t];
  }
  if (t < EMAX_SLOTS) prm->emax_bits[t] = 0u;
}
static_assert(EMAX_SLOTS <= 64, "one 64-thread block resets every slot");

template <int Q>
int cull_launch(const float* fibers, int64_t n, const float* cprep, int32_t m, const int32_t* bid,
                int32_t* labels, float* dists, unsigned long long* counters, Metric mt,
                PrefilterBuf& pb, hipEvent_t* ev, hipStream_t s, const MultiOut* mo,
                const int32_t* cperm_cached) {
  constexpr int EB = QTraits<Q>::bytes;
  const int32_t ncols_pad = (m + 31) / 32 * 32;
  const int32_t ntiles = ncols_pad / 32;
  const int64_t nk = std::max<int64_t>(std::max<int64_t>(n, m), 1);  // sort capacity
  // scratch: fiber payloads (input order), sort state (keys, the fiber
  // permutation), the centroid order, columns and tile boxes
  int rc = grow(&pb.fib_feat, &pb.fib_feat_bytes, (size_t)n * PAY_BYTES);
  rc = rc ? rc : grow_sort(pb, nk);
  rc = rc ? rc : grow(&pb.cperm, &pb.cperm_bytes, (size_t)std::max<int32_t>(m, 1) * 4);
  rc = rc ? rc : grow(&pb.cen_feat, &pb.cen_feat_bytes,
                      (size_t)ncols_pad * (CREC_BYTES + KPC * EB + 2 * sizeof(float)));
  const int32_t nsuper = (ncols_pad + 255) / 256;  // one column block each
  rc = rc ? rc : grow(&pb.tbox, &pb.tbox_bytes,
                      (size_t)TROWS * (ntiles + nsuper) * sizeof(float));
  if (rc) return rc;
  if (!pb.emax && hipMalloc((void**)&pb.emax, sizeof(PfParams)) != hipSuccess) return -3;
  PfParams* prm = (PfParams*)pb.emax;
  const Payload pay = payload_of(pb.fib_feat, n, (mt.flags & MF_TN) != 0);
  // columns: records in column order, codes, constants, centroids
  float* csort = (float*)pb.cen_feat;
  uint8_t* cfeat = (uint8_t*)(csort + (size_t)ncols_pad * CREC);
  float* cbias = (float*)(cfeat + (size_t)ncols_pad * KPC * EB);
  int32_t* ccent = (int32_t*)(cbias + ncols_pad);
  uint32_t* keys_a = (uint32_t*)pb.keys;
  int32_t* vals_a = (int32_t*)pb.vals;
  int32_t* perm = vals_a + nk;
  int32_t* cperm = (int32_t*)pb.cperm;
  // the frame: kept with a prepared atlas (after its centroid order), else
  // the box of the atlas points
  if (cperm_cached)
    frame_load_kernel<<<1, 64, 0, s>>>(prm, (const int*)(cperm_cached + m));
  else if (launch_pf_setup(prm, cprep, m, s))
    return -1;
  // centroids: their order (unless the prepared atlas holds it)
  if (!cperm_cached) {
    rc = sort_centroids(cprep, m, prm, pb, nk, cperm, s);
    if (rc) return rc;
  }
  // fibers: payloads and cells in input order, then the permutation
  {
    const int64_t nb = (n + CF_FIB - 1) / CF_FIB;
    const FiberOut fo{pay, keys_a, mo ? nullptr : labels, mo ? nullptr : dists, nullptr, 0, 0,
                      nullptr, nullptr, 0};
    if (mt.flags & MF_TN) {
      const int64_t g = cf_grid<Q, false, true>();
      cull_fiber_kernel<Q, false, true><<<(unsigned)(nb < g ? nb : g), CF_THREADS, 0, s>>>(
          fibers, n, prm, fo);
    } else {
      const int64_t g = cf_grid<Q, false, false>();
      cull_fiber_kernel<Q, false, false><<<(unsigned)(nb < g ? nb : g), CF_THREADS, 0, s>>>(
          fibers, n, prm, fo);
    }
  }
  // the fibers' sort (as radix_sort), with the sorted columns and their tile
  // boxes launched beside its first scatter
  float* tbox = (float*)pb.tbox;
  float* sbox = tbox + (size_t)TROWS * ntiles;
  {
    ColSet cs{};
    cs.c[0] = ColArgs{cprep, m,     ncols_pad, nsuper, cperm_cached ? cperm_cached : cperm,
                      prm,   cfeat, cbias,     ccent,  csort, tbox, sbox};
    cs.first[0] = 0;
    cs.first[1] = nsuper;
    cs.n = 1;
    if (sort_with_columns<Q>(n, keys_a, keys_a + nk, vals_a, perm, (uint32_t*)pb.hist, cs, s))
      return -1;
  }
  const CullJob job{pay,    perm,  prm,     cfeat,   cbias,   ccent, tbox, sbox, ntiles,
                    nsuper, fibers, n,      csort,   bid,     labels,  dists, nullptr, nullptr,
                    nullptr, 0, 0};
  const MultiOut mout = mo ? *mo : MultiOut{nullptr, 0, nullptr, nullptr};
  const unsigned blocks = (unsigned)((n + 64 * CW - 1) / (64 * CW));
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return -1;
  if (counters)
    mo ? cull_kernel<Q, true, true, false><<<blocks, 64 * CW, 0, s>>>(job, mt, mout, counters)
       : cull_kernel<Q, true, false, false><<<blocks, 64 * CW, 0, s>>>(job, mt, mout, counters);
  else
    mo ? cull_kernel<Q, false, true, false><<<blocks, 64 * CW, 0, s>>>(job, mt, mout, counters)
       : cull_kernel<Q, false, false, false><<<blocks, 64 * CW, 0, s>>>(job, mt, mout, counters);
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// A batch of subjects against prepared atlases, in chunks of consecutive
// subjects of at most CHUNK_ROWS fibers (a subject with more is a chunk of
// its own), so that a chunk's payloads stay in the memory-side cache for the
// gathers of the culled passes: per chunk the payloads and cells of its
// fibers in one launch (one frame over the union of the atlas boxes, set up
// once), one sort of its rows, then per atlas the columns (their constants
// cover the largest fiber error seen so far) and one culled pass over the
// chunk, each row writing its subject's output for that atlas.  The launches
// are captured once per launch shape into a HIP graph and replayed.
constexpr int64_t CHUNK_ROWS = (int64_t)1 << 22;
template <int Q>
int cull_batch_launch(const BatchAtlas* at, int32_t na, const int32_t* const* cperms,
                      const float* const* fibers, const int64_t* nf, int32_t ns,
                      int32_t* const* labels, float* const* dists, int mflags, PrefilterBuf& pb,
                      BatchBuf& bb, hipStream_t s) {
  constexpr int EB = QTraits<Q>::bytes;
  // subjects with fibers, in order, and their outputs; chunks of them, each
  // subject's first row and payload batch counted within its chunk
  struct Chunk {
    int32_t sub0, nsub;
    int64_t rows, blk;
  };
  std::vector<SubDev> subs;
  std::vector<Chunk> chunks;
  std::vector<int32_t*> olab;
  std::vector<float*> odst;
  int64_t rows = 0;  // the largest chunk
  for (int32_t i = 0; i < ns; ++i) {
    if (nf[i] <= 0) continue;
    if (chunks.empty() || (chunks.back().rows > 0 && chunks.back().rows + nf[i] > CHUNK_ROWS))
      chunks.push_back(Chunk{(int32_t)subs.size(), 0, 0, 0});
    Chunk& ch = chunks.back();
    subs.push_back(SubDev{fibers[i], nf[i], ch.rows, ch.blk});
    for (int32_t a = 0; a < na; ++a) {
      olab.push_back(labels[i * na + a]);
      odst.push_back(dists[i * na + a]);
    }
    ++ch.nsub;
    ch.rows += nf[i];
    ch.blk += (nf[i] + CF_FIB - 1) / CF_FIB;
    rows = std::max(rows, ch.rows);
  }
  if (rows == 0) return 0;
  if (rows >= ((int64_t)1 << 31)) return -4;  // sorted rows are indexed with 32 bits
  const int32_t nsub = (int32_t)subs.size();
  int32_t mmax = 1;
  for (int32_t a = 0; a < na; ++a) mmax = std::max(mmax, at[a].m);
  const int64_t nk = std::max<int64_t>(rows, mmax);
  // each atlas its own columns (records, codes, constants, centroids) and
  // tile boxes, so that the columns of several atlases are built together
  std::vector<size_t> col_off(na), box_off(na);
  size_t col_bytes = 0, box_floats = 0;
  for (int32_t a = 0; a < na; ++a) {
    const int64_t cpad = at[a].m > 0 ? ((int64_t)at[a].m + 31) / 32 * 32 : 0;
    col_off[a] = col_bytes;
    col_bytes += ((size_t)cpad * (CREC_BYTES + KPC * EB + 2 * sizeof(float)) + 255) / 256 * 256;
    box_off[a] = box_floats;
    box_floats += (size_t)TROWS * (cpad / 32 + (cpad + 255) / 256);
  }
  // scratch (allocated before any capture)
  int rc = grow(&pb.fib_feat, &pb.fib_feat_bytes, (size_t)rows * PAY_BYTES);
  rc = rc ? rc : grow_sort(pb, nk);
  rc = rc ? rc : grow(&pb.cen_feat, &pb.cen_feat_bytes, std::max<size_t>(col_bytes, 256));
  rc = rc ? rc : grow(&pb.tbox, &pb.tbox_bytes, std::max<size_t>(box_floats, 64) * sizeof(float));
  const size_t tab = (size_t)nsub * sizeof(SubDev) + olab.size() * 2 * sizeof(void*);
  rc = rc ? rc : grow(&bb.citems, &bb.citems_bytes, tab);
  if (rc) return rc;
  if (!pb.emax && hipMalloc((void**)&pb.emax, sizeof(PfParams)) != hipSuccess) return -3;
  // the subject table (uploaded when it changed)
  std::vector<uint64_t> tkey;
  for (const SubDev& d : subs) {
    tkey.push_back((uint64_t)(uintptr_t)d.fibers);
    tkey.push_back((uint64_t)d.n);
  }
  for (size_t k = 0; k < olab.size(); ++k) {
    tkey.push_back((uint64_t)(uintptr_t)olab[k]);
    tkey.push_back((uint64_t)(uintptr_t)odst[k]);
  }
  SubDev* dsubs = (SubDev*)bb.citems;
  int32_t** dlab = (int32_t**)(dsubs + nsub);
  float** ddst = (float**)(dlab + olab.size());
  if (bb.ckey != tkey || bb.citems_tab != bb.citems) {
    std::vector<uint8_t> host(tab);
    memcpy(host.data(), subs.data(), (size_t)nsub * sizeof(SubDev));
    memcpy(host.data() + (size_t)nsub * sizeof(SubDev), olab.data(), olab.size() * sizeof(void*));
    memcpy(host.data() + (size_t)nsub * sizeof(SubDev) + olab.size() * sizeof(void*), odst.data(),
           odst.size() * sizeof(void*));
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(bb.citems, host.data(), tab, hipMemcpyHostToDevice) != hipSuccess)
      return -1;
    bb.ckey = tkey;
    bb.citems_tab = bb.citems;
  }
  PfParams* prm = (PfParams*)pb.emax;
  const Payload pay_ext = payload_of(pb.fib_feat, rows, true);
  const Payload pay_noext = payload_of(pb.fib_feat, rows, false);
  uint32_t* keys_a = (uint32_t*)pb.keys;
  int32_t* vals_a = (int32_t*)pb.vals;
  int32_t* perm = vals_a + nk;
  float* tbox = (float*)pb.tbox;
  const bool tn = (mflags & MF_TN) != 0;
  const int64_t g = tn ? cf_grid<Q, true, true>() : cf_grid<Q, true, false>();
  // atlas a's columns and boxes in its own regions
  auto col_args = [&](int32_t a) {
    const int32_t m = at[a].m;
    const int32_t ncols_pad = (m + 31) / 32 * 32;
    const int32_t ntiles = ncols_pad / 32;
    const int32_t nsuper = (ncols_pad + 255) / 256;
    float* csort = (float*)((uint8_t*)pb.cen_feat + col_off[a]);
    uint8_t* cfeat = (uint8_t*)(csort + (size_t)ncols_pad * CREC);
    float* cbias = (float*)(cfeat + (size_t)ncols_pad * KPC * EB);
    int32_t* ccent = (int32_t*)(cbias + ncols_pad);
    float* tb = tbox + box_off[a];
    return ColArgs{at[a].cprep, m,     ncols_pad, nsuper, cperms[a], prm,
                   cfeat,       cbias, ccent,     csort,  tb,        tb + (size_t)TROWS * ntiles};
  };
  auto enqueue = [&](hipStream_t cs) -> int {
    launch_pf_init(prm, cs);
    for (int32_t a = 0; a < na; ++a) launch_pf_bbox_acc(prm, at[a].cprep, at[a].m, cs);
    for (const Chunk& ch : chunks) {
      SubDev* csubs = dsubs + ch.sub0;
      int32_t* const* clab = dlab + (size_t)ch.sub0 * na;
      float* const* cdst = ddst + (size_t)ch.sub0 * na;
      const Payload pay = tn || ch.nsub > BATCH_SUBS ? pay_ext : pay_noext;
      const FiberOut fo{pay, keys_a, nullptr, nullptr, csubs, ch.nsub, ch.blk, clab, cdst, na};
      const unsigned grid = (unsigned)(ch.blk < g ? ch.blk : g);
      if (tn)
        cull_fiber_kernel<Q, true, true><<<grid, CF_THREADS, 0, cs>>>(nullptr, 0, prm, fo);
      else
        cull_fiber_kernel<Q, true, false><<<grid, CF_THREADS, 0, cs>>>(nullptr, 0, prm, fo);
      // the sort, with the columns of the first COL_MAX atlases beside its
      // first scatter (the columns depend on the chunk through the largest
      // fiber error so far)
      ColSet set{};
      std::vector<bool> in_set(na, false);
      for (int32_t a = 0; a < na && set.n < COL_MAX; ++a) {
        if (at[a].m <= 0) continue;
        set.c[set.n] = col_args(a);
        set.first[set.n + 1] = set.first[set.n] + set.c[set.n].nsuper;
        in_set[a] = true;
        ++set.n;
      }
      if (sort_with_columns<Q>(ch.rows, keys_a, keys_a + nk, vals_a, perm, (uint32_t*)pb.hist,
                               set, cs))
        return -1;
      for (int32_t a = 0; a < na; ++a) {
        if (at[a].m <= 0) continue;  // every output already holds (-1, +inf)
        const ColArgs ca = col_args(a);
        if (!in_set[a]) cull_column_kernel<Q><<<(unsigned)ca.nsuper, 256, 0, cs>>>(ca);
        const int32_t ntiles = ca.ncols_pad / 32;
        const CullJob job{pay,    perm,    prm,      ca.feat,    ca.cb, ca.ccent, ca.tbox,
                          ca.sbox, ntiles, ca.nsuper, nullptr,   ch.rows, ca.csort,
                          at[a].bid, nullptr, nullptr, csubs, clab,  cdst,   na, a, ch.nsub};
        const MultiOut mout{nullptr, 0, nullptr, nullptr};
        cull_kernel<Q, false, false, true>
            <<<(unsigned)((ch.rows + 64 * CW - 1) / (64 * CW)), 64 * CW, 0, cs>>>(
                job, Metric{at[a].cext, mflags}, mout, nullptr);
      }
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
  };
  std::vector<uint64_t> key = {3u, (uint64_t)Q, (uint64_t)na, (uint64_t)mflags, (uint64_t)rows,
                               (uint64_t)(uintptr_t)pb.fib_feat, (uint64_t)(uintptr_t)pb.keys,
                               (uint64_t)(uintptr_t)pb.vals, (uint64_t)(uintptr_t)pb.hist,
                               (uint64_t)(uintptr_t)pb.cen_feat, (uint64_t)(uintptr_t)pb.tbox,
                               (uint64_t)(uintptr_t)pb.emax, (uint64_t)(uintptr_t)bb.citems};
  for (int32_t a = 0; a < na; ++a) {
    key.push_back((uint64_t)(uintptr_t)at[a].cprep);
    key.push_back((uint64_t)at[a].m);
    key.push_back((uint64_t)(uintptr_t)cperms[a]);
  }
  key.insert(key.end(), tkey.begin(), tkey.end());
  return graph_launch(bb, key, s, enqueue);
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

int run_cull_batch(int q, const BatchAtlas* atlases, int32_t n_atlases,
                   const int32_t* const* cperms, const float* const* fibers,
                   const int64_t* n_fibers, int32_t n_subjects, int32_t* const* labels,
                   float* const* dists, int mflags, PrefilterBuf& pb, BatchBuf& bb,
                   hipStream_t s) {
  switch (q) {
    case 0: return cull_batch_launch<Q_BF16>(atlases, n_atlases, cperms, fibers, n_fibers, n_subjects, labels, dists, mflags, pb, bb, s);
    case 1: return cull_batch_launch<Q_F16>(atlases, n_atlases, cperms, fibers, n_fibers, n_subjects, labels, dists, mflags, pb, bb, s);
    case 2: return cull_batch_launch<Q_FP8>(atlases, n_atlases, cperms, fibers, n_fibers, n_subjects, labels, dists, mflags, pb, bb, s);
    default: return -2;
  }
}

int cull_sort_centroids(const float* cprep, int32_t m, int32_t* cperm_out, PrefilterBuf& pb,
                        hipStream_t s) {
  if (m <= 0) return 0;
  int rc = grow_sort(pb, m);
  if (rc) return rc;
  if (!pb.emax && hipMalloc((void**)&pb.emax, sizeof(PfParams)) != hipSuccess) return -3;
  PfParams* prm = (PfParams*)pb.emax;
  if (launch_pf_setup(prm, cprep, m, s)) return -1;
  rc = sort_centroids(cprep, m, prm, pb, m, cperm_out, s);
  if (rc) return rc;
  frame_save_kernel<<<1, 64, 0, s>>>(prm, (int*)(cperm_out + m));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seg
