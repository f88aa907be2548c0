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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "seg_device.hpp"
#include "seg_graph.hpp"
#include "seg_internal.hpp"
#include "seg_pf.hpp"

namespace seg {

__global__ void pf_init_kernel(PfParams* __restrict__ prm) {
  const int t = threadIdx.x;
  if (t < 3) {
    prm->lo[t] = ord(__builtin_inff());
    prm->hi[t] = ord(-__builtin_inff());
  }
  if (t < EMAX_SLOTS) prm->emax_bits[t] = 0u;
}

// Bounding box of the centroid coordinates: the prepared records read as one
// flat array of 16-byte words (coalesced, grid-stride, four words per thread
// in flight at once), each float sorted to its axis by its place in the
// 64-float record (the last float, T2, is not a coordinate); reduced over the
// wave and the block, then one atomic per block and axis.
constexpr int BBOX_BLOCK = 256, BBOX_GRID = 64;
__global__ __launch_bounds__(BBOX_BLOCK) void pf_bbox_kernel(const float* __restrict__ cprep,
                                                             int32_t m,
                                                             PfParams* __restrict__ prm) {
  static_assert(CREC == 64 && NF == 63, "record layout");
  __shared__ float s_red[BBOX_BLOCK / 64][6];
  float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  const int64_t nq = (int64_t)m * (CREC / 4);
  const int64_t stride = (int64_t)gridDim.x * BBOX_BLOCK;
  constexpr int U = 4;  // words per thread and round, all loads in flight together
  for (int64_t q0 = (int64_t)blockIdx.x * BBOX_BLOCK + threadIdx.x; q0 < nq; q0 += U * stride) {
    float4 w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = q0 + u * stride;
      w[u] = q < nq ? *(const float4*)(cprep + 4 * q)
                    : make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""),
                                  __builtin_nanf(""));  // past the end: skipped below
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float v[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
      const int pos0 = (int)((4 * (q0 + u * stride)) & (CREC - 1));
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pos = pos0 + i;
        if (pos < NF && __builtin_isfinite(v[i])) {
          const int d = pos % 3;
          // select by axis without a dynamically indexed register array
          lo[0] = d == 0 ? fminf(lo[0], v[i]) : lo[0];
          hi[0] = d == 0 ? fmaxf(hi[0], v[i]) : hi[0];
          lo[1] = d == 1 ? fminf(lo[1], v[i]) : lo[1];
          hi[1] = d == 1 ? fmaxf(hi[1], v[i]) : hi[1];
          lo[2] = d == 2 ? fminf(lo[2], v[i]) : lo[2];
          hi[2] = d == 2 ? fmaxf(hi[2], v[i]) : hi[2];
        }
      }
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[d] = fminf(lo[d], __shfl_xor(lo[d], off));
      hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], off));
    }
  }
  const int wave = threadIdx.x >> 6;
  if (lane_id() == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      s_red[wave][d] = lo[d];
      s_red[wave][3 + d] = hi[d];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    float r = s_red[0][k];
    for (int w = 1; w < BBOX_BLOCK / 64; ++w) r = k < 3 ? fminf(r, s_red[w][k]) : fmaxf(r, s_red[w][k]);
    if (k < 3)
      atomicMin(&prm->lo[k], ord(r));
    else
      atomicMax(&prm->hi[k - 3], ord(r));
  }
}

// Launch of pf_bbox_kernel (nothing for m <= 0).
inline void launch_pf_bbox(const float* cprep, int32_t m, PfParams* prm, hipStream_t s) {
  if (m <= 0) return;
  const int64_t want = ((int64_t)m * (CREC / 4) + BBOX_BLOCK - 1) / BBOX_BLOCK;
  pf_bbox_kernel<<<(unsigned)(want < BBOX_GRID ? want : BBOX_GRID), BBOX_BLOCK, 0, s>>>(cprep, m,
                                                                                       prm);
}

// One wave per 64 fibers: the wave copies its 64 records (16 KB, contiguous)
// into LDS with coalesced loads, then each lane computes the quantised
// features of its fiber (row-major [n_pad][KP]), the row constant -Ha (MFMA
// C operand) and the wave's largest error, folded into the device maximum
// with one atomic.
template <int Q, int MAPK, int KP>
__global__ __launch_bounds__(64) void pf_fiber_kernel(const float* __restrict__ fibers, int64_t n,
                                                      int64_t n_pad, PfParams* __restrict__ prm,
                                                      uint8_t* __restrict__ feat,
                                                      float* __restrict__ negh) {
  using T = QTraits<Q>;
  __shared__ float s_rec[64 * NF];
  const int lane = (int)threadIdx.x;
  const int64_t f0 = (int64_t)blockIdx.x * 64;
  const int64_t nrec = n - f0 < 64 ? (n - f0 > 0 ? n - f0 : 0) : 64;
  const float* src = fibers + f0 * NF;
  if (nrec == 64) {
    // all 63 coalesced loads in flight at once, then the LDS writes
    float v[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) v[j] = src[j * 64 + lane];
#pragma unroll
    for (int j = 0; j < NF; ++j) s_rec[j * 64 + lane] = v[j];
  } else {
    for (int64_t i = lane; i < nrec * NF; i += 64) s_rec[i] = src[i];
  }
  __syncthreads();
  const int64_t f = f0 + lane;
  float e32 = 0.0f;  // every lane reaches the wave maximum below
  if (f < n_pad)
    fiber_feature_row<Q, MAPK, KP>(s_rec + lane * NF, f, n, prm, feat + f * (KP * T::bytes), negh,
                                   &e32);
  for (int off = 32; off > 0; off >>= 1) e32 = fmaxf(e32, __shfl_xor(e32, off));
  if (lane == 0) atomicMax(&prm->emax_bits[blockIdx.x % EMAX_SLOTS], __float_as_uint(e32));
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
#pragma unroll
    for (int k = 0; k < KP * T::bytes; k += 16) *(uint4*)(row + k) = make_uint4(0, 0, 0, 0);
    cb[col] = __builtin_inff();
    return;
  }
  cb[col] = column_row<Q, MAPK, KP>(cprep + (int64_t)c * CREC, (col % MI::CPC) == 1, prm, row);
}

// ------------------------------------------------------------------ fused kernel

// One subject against one atlas, as the fused kernel sees it.
struct PfJob {
  const uint8_t* ffeat;  // quantised fiber features [n_pad][KP]
  const float* fnegh;    // -Ha per fiber row [n_pad]
  const uint8_t* cfeat;  // quantised column features [ncols_pad][KP]
  const float* cbias;    // cb per column [ncols_pad]
  int32_t ncols_pad;
  const float* fibers;   // the subject's fiber records
  int64_t n;
  const float* cprep;    // prepared centroid records (63 coordinates + T2)
  const int32_t* bid;
  int32_t* labels;
  float* dists;
  Metric mt;
};

// Centroid tiles per LDS chunk for a feature width.
template <int KP> struct Chunk { static constexpr int CH = KP <= 32 ? 8 : (KP <= 48 ? 4 : 2); };

// Rows = fibers (A operand, held in registers for the whole kernel), columns
// = centroid columns (B operand).  Each wave owns GF groups of 32 fibers; the
// four waves of a block share the centroid stream.
//
// Centroid stream: chunks of CH tiles (32 columns each) pass through three
// LDS buffers.  During chunk k every thread holds chunk k+2 in registers
// (loaded from global at the start of the chunk) and writes it to the buffer
// of chunk k-1 at the end; one barrier per chunk then makes it visible.  The
// MFMAs of tile t+1 are issued before the epilogue of tile t (two
// accumulator sets), also across chunk boundaries, so the matrix unit works
// while the VALU reduces.
//
// Per tile and group: KP/16 MFMAs starting from C = -Ha, then the largest of
// the lane's 16 outputs is compared with the column constant cb; the hot loop
// only records which (tile, group) has a lane above it.  After the loop those
// few are recomputed and every (fiber, centroid) above cb is pushed into the
// wave's LDS queue (ballot + prefix count), drained by the exact stage as in
// the plain pass.  With PAIRS, survivors are written to a global list instead
// (diagnostics).
template <int Q, int KP, int GF, int CPC, bool STATS, bool PAIRS>
__device__ __forceinline__ void prefilter_block(const PfJob& job, int64_t block,
                                                unsigned long long* __restrict__ counters,
                                                int32_t* __restrict__ pairs, int64_t cap) {
  const uint8_t* __restrict__ ffeat = job.ffeat;
  const float* __restrict__ fnegh = job.fnegh;
  const uint8_t* __restrict__ cfeat = job.cfeat;
  const float* __restrict__ cbias = job.cbias;
  const int32_t ncols_pad = job.ncols_pad;
  const float* __restrict__ fibers = job.fibers;
  const int64_t n = job.n;
  const float* __restrict__ cprep = job.cprep;
  const int32_t* __restrict__ bid = job.bid;
  int32_t* __restrict__ labels = job.labels;
  float* __restrict__ dists = job.dists;
  using FT = typename Frag<Q>::T;
  constexpr int KS = KP / 16;
  constexpr int EB = QTraits<Q>::bytes;
  constexpr int WAVES = 4;
  constexpr int FPW = GF * 32;
  constexpr int CH = Chunk<KP>::CH;
  constexpr int CCOLS = 32 * CH;  // columns per chunk (<= 256 = one per thread)
  // The queue takes at most 64 entries per push (one per lane) and is drained
  // before a push whenever fewer than 64 places are left.
  constexpr int QCAP = 512;
  static_assert(FPW <= 256, "slot must fit 8 bits");
  static_assert(CCOLS <= 256, "one chunk column per thread");
  static_assert(CH % 2 == 0, "accumulator sets alternate within a chunk");
  __shared__ FT s_feat[3][CH][KS][2][32];
  __shared__ float s_cb[3][CH][32];
  // tiles with a survivor, processed after the centroid loop
  constexpr int HCAP = 256;
  __shared__ uint32_t s_hits[WAVES][HCAP];
  __shared__ uint32_t s_queue[PAIRS ? 1 : WAVES][PAIRS ? 1 : QCAP];
  __shared__ uint64_t s_keys[PAIRS ? 1 : WAVES][PAIRS ? 1 : FPW];
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5;
  const int64_t wbase = (block * WAVES + wave) * FPW;
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
  const int32_t nchunks = ncols_pad / CCOLS;

  // chunk staging: thread tid < CCOLS owns chunk column tid
  FT gfe[KS][2];
  float gcb = 0.0f;
  auto gload = [&](int32_t chunk) {
    if (tid < CCOLS && chunk < nchunks) {
      const int64_t col = (int64_t)chunk * CCOLS + tid;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          gfe[s][h] = *(const FT*)(cfeat + col * (KP * EB) + (s * 16 + 8 * h) * EB);
      gcb = cbias[col];
    }
  };
  auto lstore = [&](int buf, int32_t chunk) {
    if (tid < CCOLS && chunk < nchunks) {
      const int tl = tid >> 5, j = tid & 31;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) s_feat[buf][tl][s][h][j] = gfe[s][h];
      s_cb[buf][tl][j] = gcb;
    }
  };
  gload(0);
  lstore(0, 0);
  gload(1);
  lstore(1, 1);
  __syncthreads();

  // Three stages per tile: the fragment of tile t+2 is read from LDS, the
  // MFMAs of tile t+1 are issued (its fragment was read one step earlier),
  // and the epilogue of tile t runs on the products issued one step earlier.
  FT frag[2][KS];
  float fcb[2];
  auto fetch = [&](int set, int bufx, int tl) {
#pragma unroll
    for (int s = 0; s < KS; ++s) frag[set][s] = s_feat[bufx][tl][s][half][lane & 31];
    fcb[set] = s_cb[bufx][tl][lane & 31];
  };
  f32x16 acc[2][GF];
  float cbc[2];
  auto issue = [&](int set, int fset) {
#pragma unroll
    for (int g = 0; g < GF; ++g) {
      acc[set][g] = Frag<Q>::mfma(afr[g][0], frag[fset][0], negh[g]);
#pragma unroll
      for (int s = 1; s < KS; ++s) acc[set][g] = Frag<Q>::mfma(afr[g][s], frag[fset][s], acc[set][g]);
    }
    cbc[set] = fcb[fset];
  };
  // tile 0 issued, tile 1 fetched (both in chunk 0 since CH >= 2)
  fetch(0, 0, 0);
  issue(0, 0);
  fetch(1, 0, 1);

  // Survivor extraction for one tile, after the centroid loop: the products
  // of every fiber group are recomputed (one more MFMA each; hits are rare)
  // and every (fiber, centroid) at or above cb is pushed.
  uint32_t qn = 0;
  auto extract_tile = [&](int32_t tile) {
    const int32_t col = tile * 32 + (lane & 31);
    FT b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s)
      b[s] = *(const FT*)(cfeat + (int64_t)col * (KP * EB) + (s * 16 + 8 * half) * EB);
    const float cb = cbias[col];
    const uint32_t cent = (uint32_t)(col / CPC);
#pragma unroll
    for (int g = 0; g < GF; ++g) {
      f32x16 a = Frag<Q>::mfma(afr[g][0], b[0], negh[g]);
#pragma unroll
      for (int s = 1; s < KS; ++s) a = Frag<Q>::mfma(afr[g][s], b[s], a);
      if (!wave_any(max16(a) >= cb)) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int slot = g * 32 + out_row(lane, r);
        const bool p = a[r] >= cb && wbase + slot < n;
        const uint64_t msk = __ballot(p);
        if (!msk) continue;
        if (PAIRS) {
          if (p) {
            const unsigned long long kk = atomicAdd(counters, 1ull);
            if ((int64_t)kk < cap) {
              pairs[2 * kk] = (int32_t)(wbase + slot);
              pairs[2 * kk + 1] = (int32_t)cent;
            }
          }
        } else {
          if (qn > (uint32_t)(QCAP - 64)) {
            queue_drain_call<STATS>(wq, qn, fib_base, cprep, sc, job.mt);
            qn = 0;
          }
          queue_push(wq, qn, msk, (cent << 8) | (uint32_t)slot);
        }
      }
    }
  };

  // The hot loop only records which tiles have a lane at or above cb (a
  // wave-uniform list in LDS, in increasing tile order).  If the list fills
  // up, the tiles after the last recorded one are scanned again afterwards.
  uint32_t nh = 0;
  uint32_t* hl = s_hits[wave];
  int buf = 0;
  for (int32_t k = 0; k < nchunks; ++k) {
    gload(k + 2);
    const int nbuf = buf == 2 ? 0 : buf + 1;
    const int fbuf = k + 1 < nchunks ? nbuf : buf;  // past the end: harmless re-reads
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      // tile u+1 was fetched into set (u+1)&1 one step ago: issue it; then
      // fetch tile u+2 into the set just consumed (u&1)
      issue((u + 1) & 1, (u + 1) & 1);
      if (u + 2 < CH)
        fetch(u & 1, buf, u + 2);
      else
        fetch(u & 1, fbuf, u + 2 - CH);
      const int cs = u & 1;
      float mx = max16(acc[cs][0]);
#pragma unroll
      for (int g = 1; g < GF; ++g) mx = __builtin_fmaxf(mx, max16(acc[cs][g]));
      if (wave_any(mx >= cbc[cs])) {
        if (nh < (uint32_t)HCAP && lane == 0) hl[nh] = (uint32_t)(k * CH + u);
        ++nh;
      }
    }
    // chunk k+2 goes into the buffer of chunk k-1 (nobody reads it any more)
    lstore(buf == 0 ? 2 : buf - 1, k + 2);
    __syncthreads();
    buf = nbuf;
  }
  const int32_t ntiles = nchunks * CH;
  const uint32_t nrec = nh < (uint32_t)HCAP ? nh : (uint32_t)HCAP;
  int32_t scan = nh > (uint32_t)HCAP ? (int32_t)hl[HCAP - 1] + 1 : ntiles;
  for (uint32_t i = 0;; ++i) {
    int32_t tile;
    if (i < nrec)
      tile = (int32_t)hl[i];
    else if (scan < ntiles)
      tile = scan++;
    else
      break;
    extract_tile(tile);
  }
  if (PAIRS) return;
  queue_drain_call<STATS>(wq, qn, fib_base, cprep, sc, job.mt);
  for (int k = lane; k < FPW; k += 64) {
    const int64_t f = wbase + k;
    if (f < n) write_result(wq.keys[k], bid, labels + f, dists + f, job.mt.flags);
  }
}

template <int Q, int KP, int GF, int CPC, bool STATS, bool PAIRS>
__global__ __launch_bounds__(256) void prefilter_kernel(PfJob job,
                                                        unsigned long long* __restrict__ counters,
                                                        int32_t* __restrict__ pairs, int64_t cap) {
  prefilter_block<Q, KP, GF, CPC, STATS, PAIRS>(job, blockIdx.x, counters, pairs, cap);
}

// Batch form: one launch over the flattened work list.  Block b runs fiber
// block b - start[j] of job j; jobs are ordered by cost per block (largest
// atlas first), and the hardware dispatches blocks in index order as CUs
// free up, so the costliest items start first and the cheapest fill the
// tail.  (A persistent loop pulling items from a counter needs about 100
// more registers per lane here and runs at half the occupancy.)
template <int Q, int KP, int GF, int CPC>
__global__ __launch_bounds__(256) void prefilter_batch_kernel(const PfJob* __restrict__ jobs,
                                                              const int64_t* __restrict__ job_start,
                                                              int32_t njobs) {
  const int64_t it = blockIdx.x;
  const int32_t j = find_job(job_start, njobs, it);
  prefilter_block<Q, KP, GF, CPC, false, false>(jobs[j], it - job_start[j], nullptr, nullptr, 0);
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

}  // namespace

// Kernel configuration of the sorted, tile-culled form (symmetric maps).
constexpr int CULL_TILE = 8;

namespace {

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
    case 3: c->kp = 16; c->gf = 1; break;
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
               int64_t cap, Metric mt, PrefilterBuf& pb, hipEvent_t* ev, hipStream_t s) {
  using MI = MapInfo<MAPK, KP>;
  constexpr int EB = QTraits<Q>::bytes;
  constexpr int FPB = 4 * GF * 32;  // fibers per block
  const int64_t n_pad = (n + FPB - 1) / FPB * FPB;
  const int32_t ncols = m * MI::CPC;
  constexpr int CC = 32 * Chunk<KP>::CH;  // columns per LDS chunk
  const int32_t ncols_pad = (ncols + CC - 1) / CC * CC;
  int rc = grow(&pb.fib_feat, &pb.fib_feat_bytes, (size_t)n_pad * KP * EB);
  rc = rc ? rc : grow((void**)&pb.fib_h, &pb.fib_h_bytes, (size_t)n_pad * sizeof(float));
  rc = rc ? rc : grow(&pb.cen_feat, &pb.cen_feat_bytes,
                      (size_t)ncols_pad * (KP * EB + sizeof(float)));
  if (rc) return rc;
  if (!pb.emax && hipMalloc((void**)&pb.emax, sizeof(PfParams)) != hipSuccess) return -3;
  PfParams* prm = (PfParams*)pb.emax;
  uint8_t* cfeat = (uint8_t*)pb.cen_feat;
  float* cb = (float*)(cfeat + (size_t)ncols_pad * KP * EB);
  pf_init_kernel<<<1, 64, 0, s>>>(prm);
  launch_pf_bbox(cprep, m, prm, s);
  pf_fiber_kernel<Q, MAPK, KP><<<(unsigned)((n_pad + 63) / 64), 64, 0, s>>>(
      fibers, n, n_pad, prm, (uint8_t*)pb.fib_feat, pb.fib_h);
  pf_column_kernel<Q, MAPK, KP><<<(unsigned)((ncols_pad + 255) / 256), 256, 0, s>>>(
      cprep, m, ncols_pad, prm, cfeat, cb);
  const unsigned blocks = (unsigned)(n_pad / FPB);
  const PfJob job{(const uint8_t*)pb.fib_feat, pb.fib_h, cfeat, cb, ncols_pad, fibers, n, cprep,
                  bid, labels, dists, mt};
  if (pairs) {
    prefilter_kernel<Q, KP, GF, MI::CPC, false, true><<<blocks, 256, 0, s>>>(job, counters, pairs,
                                                                             cap);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return -1;
  if (counters)
    prefilter_kernel<Q, KP, GF, MI::CPC, true, false><<<blocks, 256, 0, s>>>(job, counters,
                                                                             nullptr, 0);
  else
    prefilter_kernel<Q, KP, GF, MI::CPC, false, false><<<blocks, 256, 0, s>>>(job, counters,
                                                                              nullptr, 0);
  if (ev && hipEventRecord(ev[1], s) != hipSuccess) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dispatch(const Cfg& c, const float* fibers, int64_t n, const float* cprep, int32_t m,
             const int32_t* bid, int32_t* labels, float* dists, unsigned long long* counters,
             int32_t* pairs, int64_t cap, Metric mt, PrefilterBuf& pb, hipEvent_t* ev,
             hipStream_t s) {
#define SEG_PF(QQ, MM, KK, GG)                                                                   \
  if (c.q == QQ && c.mapk == MM && c.kp == KK && c.gf == GG)                                     \
    return launch_cfg<QQ, MM, KK, GG>(fibers, n, cprep, m, bid, labels, dists, counters, pairs, \
                                      cap, mt, pb, ev, s);
  SEG_PF(Q_BF16, MAP_SYM, 16, 2)
  SEG_PF(Q_BF16, MAP_SYM, 16, 4)
  SEG_PF(Q_BF16, MAP_SYM, 16, 1)
  SEG_PF(Q_BF16, MAP_SYM, 32, 2)
  SEG_PF(Q_BF16, MAP_SYM, 32, 4)
  SEG_PF(Q_BF16, MAP_SYM, 48, 2)
  SEG_PF(Q_BF16, MAP_SYM, 48, 4)
  SEG_PF(Q_F16, MAP_SYM, 16, 2)
  SEG_PF(Q_F16, MAP_SYM, 16, 4)
  SEG_PF(Q_F16, MAP_SYM, 16, 1)
  SEG_PF(Q_F16, MAP_SYM, 32, 2)
  SEG_PF(Q_F16, MAP_SYM, 32, 4)
  SEG_PF(Q_F16, MAP_SYM, 48, 2)
  SEG_PF(Q_F16, MAP_SYM, 48, 4)
  SEG_PF(Q_FP8, MAP_SYM, 16, 2)
  SEG_PF(Q_FP8, MAP_SYM, 16, 4)
  SEG_PF(Q_FP8, MAP_SYM, 16, 1)
  SEG_PF(Q_FP8, MAP_SYM, 32, 2)
  SEG_PF(Q_FP8, MAP_SYM, 32, 4)
  SEG_PF(Q_FP8, MAP_SYM, 48, 2)
  SEG_PF(Q_FP8, MAP_SYM, 48, 4)
  SEG_PF(Q_BF16, MAP_ORIENTED, 64, 2)
  SEG_PF(Q_BF16, MAP_ORIENTED, 64, 4)
#undef SEG_PF
  return -2;
}

// A batch: every subject against every atlas with one shared frame (origin,
// scale) and one fiber error bound, so each subject's features are computed
// once for all atlases.  Launched as one persistent kernel inside a cached
// HIP graph.
template <int Q, int MAPK, int KP, int GF>
int batch_cfg(int mode, int cfg, const BatchAtlas* at, int32_t na, const float* const* fibers,
              const int64_t* nf, int32_t ns, int32_t* const* labels, float* const* dists,
              int mflags, BatchBuf& bb, hipStream_t s) {
  using MI = MapInfo<MAPK, KP>;
  constexpr int EB = QTraits<Q>::bytes;
  constexpr int FPB = 4 * GF * 32;
  constexpr int CC = 32 * Chunk<KP>::CH;
  constexpr size_t HDR = 512;  // PfParams at the head of the job buffer
  std::vector<uint64_t> key = {2u, (uint64_t)mode, (uint64_t)cfg, (uint64_t)na, (uint64_t)ns,
                               (uint64_t)mflags};
  for (int32_t a = 0; a < na; ++a) {
    key.push_back((uint64_t)(uintptr_t)at[a].cprep);
    key.push_back((uint64_t)at[a].m);
  }
  for (int32_t i = 0; i < ns; ++i) {
    key.push_back((uint64_t)(uintptr_t)fibers[i]);
    key.push_back((uint64_t)nf[i]);
    for (int32_t a = 0; a < na; ++a) {
      key.push_back((uint64_t)(uintptr_t)labels[i * na + a]);
      key.push_back((uint64_t)(uintptr_t)dists[i * na + a]);
    }
  }
  std::vector<int64_t> foff(ns), npad(ns);
  int64_t ftot = 0;
  for (int32_t i = 0; i < ns; ++i) {
    npad[i] = (nf[i] + FPB - 1) / FPB * FPB;
    foff[i] = ftot;
    ftot += npad[i];
  }
  std::vector<int64_t> coff(na);
  std::vector<int32_t> ncp(na);
  int64_t ctot = 0;
  for (int32_t a = 0; a < na; ++a) {
    ncp[a] = (at[a].m * MI::CPC + CC - 1) / CC * CC;
    coff[a] = ctot;
    ctot += ncp[a];
  }
  // jobs: atlases with more columns first (costlier blocks early), then subjects
  std::vector<int32_t> order(na);
  for (int32_t a = 0; a < na; ++a) order[a] = a;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return ncp[x] > ncp[y]; });
  const bool same = bb.exec && bb.key == key;
  uint8_t* items = (uint8_t*)bb.items;
  if (!same) {
    // buffers may be in use by a previous launch on this stream
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    int rc = grow(&bb.fib_feat, &bb.fib_feat_bytes, (size_t)std::max<int64_t>(ftot, 1) * KP * EB);
    rc = rc ? rc : grow((void**)&bb.fib_h, &bb.fib_h_bytes, (size_t)std::max<int64_t>(ftot, 1) * 4);
    rc = rc ? rc : grow(&bb.cen_feat, &bb.cen_feat_bytes,
                        (size_t)std::max<int64_t>(ctot, 1) * (KP * EB + 4));
    if (rc) return rc;
    std::vector<PfJob> jobs;
    std::vector<int64_t> start(1, 0);
    uint8_t* cfeat = (uint8_t*)bb.cen_feat;
    float* cbb = (float*)(cfeat + (size_t)ctot * KP * EB);
    for (int32_t oi = 0; oi < na; ++oi) {
      const int32_t a = order[oi];
      if (at[a].m == 0) continue;
      for (int32_t i = 0; i < ns; ++i) {
        if (nf[i] == 0) continue;
        jobs.push_back(PfJob{(const uint8_t*)bb.fib_feat + (size_t)foff[i] * KP * EB,
                             bb.fib_h + foff[i], cfeat + (size_t)coff[a] * KP * EB,
                             cbb + coff[a], ncp[a], fibers[i], nf[i], at[a].cprep, at[a].bid,
                             labels[i * na + a], dists[i * na + a],
                             Metric{at[a].cext, mflags}});
        start.push_back(start.back() + npad[i] / FPB);
      }
    }
    const size_t need = HDR + jobs.size() * sizeof(PfJob) + start.size() * sizeof(int64_t);
    rc = grow(&bb.items, &bb.items_bytes, need);
    if (rc) return rc;
    items = (uint8_t*)bb.items;
    std::vector<uint8_t> host(need - HDR);
    if (!jobs.empty()) memcpy(host.data(), jobs.data(), jobs.size() * sizeof(PfJob));
    memcpy(host.data() + jobs.size() * sizeof(PfJob), start.data(), start.size() * sizeof(int64_t));
    if (hipMemcpy(items + HDR, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
      return -1;
    bb.key.clear();  // stale until the new graph is captured
    bb.njobs = (int32_t)jobs.size();
  }
  static_assert(sizeof(PfParams) <= HDR, "parameters fit the header of the job buffer");
  PfParams* prm = (PfParams*)items;
  const PfJob* djobs = (const PfJob*)(items + HDR);
  const int64_t* dstart = (const int64_t*)(items + HDR + bb.njobs * sizeof(PfJob));
  const int32_t njobs = bb.njobs;
  int64_t total = 0;  // work items (fiber blocks over all jobs)
  for (int32_t a = 0; a < na; ++a)
    if (at[a].m > 0)
      for (int32_t i = 0; i < ns; ++i) total += npad[i] / FPB;
  auto enqueue = [&](hipStream_t cs) -> int {
    uint8_t* cfeat = (uint8_t*)bb.cen_feat;
    float* cbb = (float*)(cfeat + (size_t)ctot * KP * EB);
    pf_init_kernel<<<1, 64, 0, cs>>>(prm);
    for (int32_t a = 0; a < na; ++a)
      if (at[a].m > 0)
        launch_pf_bbox(at[a].cprep, at[a].m, prm, cs);
    for (int32_t i = 0; i < ns; ++i)
      if (nf[i] > 0)
        pf_fiber_kernel<Q, MAPK, KP><<<(unsigned)(npad[i] / 64), 64, 0, cs>>>(
            fibers[i], nf[i], npad[i], prm, (uint8_t*)bb.fib_feat + (size_t)foff[i] * KP * EB,
            bb.fib_h + foff[i]);
    for (int32_t a = 0; a < na; ++a) {
      if (at[a].m > 0) {
        pf_column_kernel<Q, MAPK, KP><<<(unsigned)((ncp[a] + 255) / 256), 256, 0, cs>>>(
            at[a].cprep, at[a].m, ncp[a], prm, cfeat + (size_t)coff[a] * KP * EB, cbb + coff[a]);
      } else {
        for (int32_t i = 0; i < ns; ++i)
          if (launch_fill_empty(nf[i], labels[i * na + a], dists[i * na + a], cs)) return -1;
      }
    }
    if (njobs > 0 && total > 0)
      prefilter_batch_kernel<Q, KP, GF, MI::CPC><<<(unsigned)total, 256, 0, cs>>>(djobs, dstart,
                                                                                  njobs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  };
  return graph_launch(bb, key, s, enqueue);
}

int batch_dispatch(int mode, int cfg, const Cfg& c, const BatchAtlas* at, int32_t na,
                   const float* const* fibers, const int64_t* nf, int32_t ns,
                   int32_t* const* labels, float* const* dists, int mflags, BatchBuf& bb,
                   hipStream_t s) {
#define SEG_PFB(QQ, MM, KK, GG)                                                             \
  if (c.q == QQ && c.mapk == MM && c.kp == KK && c.gf == GG)                                \
    return batch_cfg<QQ, MM, KK, GG>(mode, cfg, at, na, fibers, nf, ns, labels, dists, mflags, \
                                     bb, s);
  SEG_PFB(Q_BF16, MAP_SYM, 16, 2)
  SEG_PFB(Q_BF16, MAP_SYM, 16, 1)
  SEG_PFB(Q_BF16, MAP_SYM, 32, 2)
  SEG_PFB(Q_F16, MAP_SYM, 16, 2)
  SEG_PFB(Q_F16, MAP_SYM, 16, 1)
  SEG_PFB(Q_F16, MAP_SYM, 32, 2)
  SEG_PFB(Q_FP8, MAP_SYM, 16, 2)
  SEG_PFB(Q_BF16, MAP_ORIENTED, 64, 2)
#undef SEG_PFB
  return -2;
}

}  // namespace

int prefilter_batch(int mode, int cfg, const BatchAtlas* atlases, int32_t n_atlases,
                    const float* const* fibers, const int64_t* n_fibers, int32_t n_subjects,
                    int32_t* const* labels, float* const* dists, int mflags, BatchBuf& bb,
                    hipStream_t s) {
  Cfg c;
  if (resolve(mode, cfg, &c)) return -2;
  return batch_dispatch(mode, cfg, c, atlases, n_atlases, fibers, n_fibers, n_subjects, labels,
                        dists, mflags, bb, s);
}

size_t pf_params_bytes() { return sizeof(PfParams); }

int launch_pf_init(PfParams* prm, hipStream_t s) {
  pf_init_kernel<<<1, 64, 0, s>>>(prm);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pf_bbox_acc(PfParams* prm, const float* cprep, int32_t m, hipStream_t s) {
  launch_pf_bbox(cprep, m, prm, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pf_setup(PfParams* prm, const float* cprep, int32_t m, hipStream_t s) {
  pf_init_kernel<<<1, 64, 0, s>>>(prm);
  if (m > 0) launch_pf_bbox(cprep, m, prm, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int run_prefilter(int mode, int cfg, const float* fibers, int64_t n, const float* cprep,
                  const float4* ccen, int32_t m, const int32_t* bid, int32_t* labels,
                  float* dists, unsigned long long* counters, Metric mt, PrefilterBuf& pb,
                  hipEvent_t* ev, hipStream_t s, const int32_t* cperm) {
  (void)ccen;
  // symmetric maps: the sorted, tile-culled form unless a streaming tile is
  // asked for (or the subject is too large for 32-bit sorted rows)
  if (mode >= 2 && mode <= 4 && (cfg == CULL_TILE || (cfg == 0 && n < ((int64_t)1 << 31))))
    return run_cull(mode - 2, fibers, n, cprep, m, bid, labels, dists, counters, mt, pb, ev, s,
                    nullptr, cperm);
  Cfg c;
  if (resolve(mode, cfg, &c)) return -2;
  return dispatch(c, fibers, n, cprep, m, bid, labels, dists, counters, nullptr, 0, mt, pb, ev,
                  s);
}

int prefilter_pairs(int mode, const float* fibers, int64_t n, const float* cprep,
                    const float4* ccen, int32_t m, int32_t* pairs, int64_t cap,
                    unsigned long long* count, PrefilterBuf& pb, hipStream_t s) {
  (void)ccen;
  Cfg c;
  if (resolve(mode, 0, &c)) return -2;
  return dispatch(c, fibers, n, cprep, m, nullptr, nullptr, nullptr, count, pairs, cap,
                  Metric{nullptr, 0}, pb, nullptr, s);
}

}  // namespace seg
