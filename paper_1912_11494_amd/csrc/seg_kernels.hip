// Segmentation kernels for gfx950: atlas preparation, input validation, the
// dense exact pass and the plain (center-test) pass.
//
// Data layout in HBM:
//   fibers     caller's [N][21][3] float32 (252-byte records, read in place)
//   centroids  caller's [M][21][3] float32
//   cprep      library's [M][64] float32: the 63 coordinates + T2 of the
//              centroid's bundle (256-byte records, one scalar-load burst)
//   ccen       library's [M] float4: center point (x, y, z) + T2, the only
//              centroid data the center test touches (16 bytes / centroid)
//   labels/dists  caller's [N] int32 / float32
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "seg_device.hpp"
#include "seg_graph.hpp"
#include "seg_internal.hpp"

namespace seg {

// ---------------------------------------------------------------- preparation

// One thread per centroid: copy the record, attach T2 of its bundle.  A bundle
// id outside [0, B) gets T2 = -1 (never matches) and raises a flag.  The
// threads also check the B thresholds for NaN (grid-stride over bundles).
__global__ __launch_bounds__(256) void prep_atlas_kernel(const float* __restrict__ cen, int64_t m,
                                                         const int32_t* __restrict__ bid,
                                                         const float* __restrict__ thr, int32_t nb,
                                                         float* __restrict__ cprep,
                                                         float4* __restrict__ ccen,
                                                         int32_t* __restrict__ bid_out,
                                                         float* __restrict__ cext,
                                                         unsigned int* __restrict__ flags) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t b = c; b < nb; b += (int64_t)gridDim.x * blockDim.x)
    if (__builtin_isnan(thr[b])) atomicOr(flags, FLAG_NONFINITE);
  if (c >= m) {
    // padding up to a multiple of 8: a center test that never passes
    if (c < ((m + 7) & ~(int64_t)7)) {
      ccen[c] = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
      bid_out[c] = -1;
    }
    return;
  }
  const float* src = cen + c * NF;
  float* dst = cprep + c * CREC;
  const int32_t b = bid[c];
  float t2 = -1.0f;
  if (b >= 0 && b < nb) {
    t2 = thr2(thr[b]);
  } else {
    atomicOr(flags, FLAG_BUNDLE);
  }
  // the record in registers: every load issued before the first store, and
  // the arc length taken from the registers, not re-read from the copy
  float v[CREC];
#pragma unroll
  for (int k = 0; k < NF; ++k) v[k] = src[k];
  v[NF] = t2;
  bool finite = true;
#pragma unroll
  for (int k = 0; k < NF; ++k) finite = finite && __builtin_isfinite(v[k]);
#pragma unroll
  for (int k = 0; k < CREC; k += 4)
    *(float4*)(dst + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
  if (!finite) atomicOr(flags, FLAG_NONFINITE);
  ccen[c] = make_float4(v[3 * CTR], v[3 * CTR + 1], v[3 * CTR + 2], t2);
  bid_out[c] = b;
  // for the length-normalised metric: arc length and threshold T
  cext[2 * c] = arc_length(v);
  cext[2 * c + 1] = (b >= 0 && b < nb) ? thr[b] : -1.0f;
}

__global__ __launch_bounds__(256) void check_thresholds_kernel(const float* __restrict__ thr,
                                                               int32_t nb,
                                                               unsigned int* __restrict__ flags) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb && __builtin_isnan(thr[b])) atomicOr(flags, FLAG_NONFINITE);
}

// Grid-stride scan of coordinates for NaN / inf (4-byte aligned input).
__global__ __launch_bounds__(256) void check_finite_kernel(const float* __restrict__ v,
                                                           int64_t count,
                                                           unsigned int* __restrict__ flags) {
  bool ok = true;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    ok = ok && __builtin_isfinite(v[i]);
  if (!wave_any(!ok)) return;
  if (lane_id() == 0) atomicOr(flags, FLAG_NONFINITE);
}

__global__ void fill_u64_kernel(unsigned long long* __restrict__ p, int n, unsigned long long v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void fill_empty_kernel(int64_t n, int32_t* __restrict__ labels,
                                                         float* __restrict__ dists) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    labels[i] = -1;
    dists[i] = __builtin_inff();
  }
}

// ---------------------------------------------------------------- dense exact

// Every pair, all 21 points, both orders, no early exit: the exact stage run
// on the whole N x M product.  Each lane keeps FPL fibers (63 floats each) in
// registers; the centroid record is wave-uniform and arrives through scalar
// loads, so the inner loop is pure VALU work (3 differences, 1 product,
// 2 FMAs and a max per point distance).  The argmin stays in registers: the
// centroid loop runs in increasing index order and a strictly smaller D
// replaces the best, so equal distances keep the lower index.
template <int FPL, bool VAR>
__global__ __launch_bounds__(256) void dense_kernel(const float* __restrict__ fibers, int64_t n,
                                                    const float* __restrict__ cprep, int32_t m,
                                                    const int32_t* __restrict__ bid,
                                                    int32_t* __restrict__ labels,
                                                    float* __restrict__ dists, Metric mt) {
  const int64_t base = ((int64_t)blockIdx.x * blockDim.x) * FPL + threadIdx.x;
  float a[FPL][NF];
  float best[FPL];
  int32_t bc[FPL];
  float ls[FPL];  // arc lengths (metric variants only)
  uint64_t bkey[FPL];
#pragma unroll
  for (int k = 0; k < FPL; ++k) {
    const int64_t f = base + (int64_t)k * blockDim.x;
    const float* src = fibers + (f < n ? f : 0) * NF;
#pragma unroll
    for (int j = 0; j < NF; ++j) a[k][j] = src[j];
    best[k] = 0.0f;
    bc[k] = -1;
    bkey[k] = NO_KEY;
    ls[k] = VAR && (mt.flags & MF_TN) ? arc_length(a[k]) : 0.0f;
  }
  for (int32_t c = 0; c < m; ++c) {
    const float* b = cprep + (size_t)c * CREC;
    const float t2 = b[NF];
#pragma unroll
    for (int k = 0; k < FPL; ++k) {
      float mc = d2(a[k][3 * CTR], a[k][3 * CTR + 1], a[k][3 * CTR + 2], b[3 * CTR],
                    b[3 * CTR + 1], b[3 * CTR + 2]);
      float md = mc, mi = mc;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (i == CTR) continue;
        const int j = NP - 1 - i;
        float x = d2(a[k][3 * i], a[k][3 * i + 1], a[k][3 * i + 2], b[3 * i], b[3 * i + 1],
                     b[3 * i + 2]);
        float y = d2(a[k][3 * i], a[k][3 * i + 1], a[k][3 * i + 2], b[3 * j], b[3 * j + 1],
                     b[3 * j + 2]);
        md = fmaxf(md, x);
        mi = fmaxf(mi, y);
      }
      if (!VAR) {
        const float D = fminf(md, mi);
        const bool take = D <= t2 && (bc[k] < 0 || D < best[k]);
        best[k] = take ? D : best[k];
        bc[k] = take ? c : bc[k];
      } else {
        float D = fminf(md, mi);
        if (mt.flags & MF_DIR) {
          const float x0 = d2(a[k][0], a[k][1], a[k][2], b[0], b[1], b[2]);
          const float x1 = d2(a[k][60], a[k][61], a[k][62], b[60], b[61], b[62]);
          const float y0 = d2(a[k][0], a[k][1], a[k][2], b[60], b[61], b[62]);
          const float y1 = d2(a[k][60], a[k][61], a[k][62], b[0], b[1], b[2]);
          D = fmaxf(x0, x1) <= fmaxf(y0, y1) ? md : mi;
        }
        float v;
        if (D <= t2 && variant_value(D, (uint32_t)c, ls[k], mt, v)) {
          const uint64_t key = make_key(v, (uint32_t)c);
          bkey[k] = key < bkey[k] ? key : bkey[k];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < FPL; ++k) {
    const int64_t f = base + (int64_t)k * blockDim.x;
    if (f < n) {
      uint64_t key = VAR ? bkey[k] : (bc[k] < 0 ? NO_KEY : make_key(best[k], (uint32_t)bc[k]));
      write_result(key, bid, labels + f, dists + f, VAR ? mt.flags : 0);
    }
  }
}

// ---------------------------------------------------------------- plain pass

// The paper's test1 on every pair, fused with the rest of the method.
// Each wave owns 64 * FPL consecutive fibers (lane l, slot k*64 + l) and keeps
// their center points in registers.  For every centroid (wave-uniform, a
// 16-byte scalar load of center + T2) each lane evaluates the center distance
// of its FPL fibers.  Survivors are rare; when a wave has any, it appends
// them to its LDS queue with a ballot + prefix count.  A nearly full queue is
// drained by running tests 2-4 and the full metric with one queued pair per
// lane (exact_pair); accepted pairs are merged into per-fiber 64-bit
// (D, centroid) keys in LDS with an atomic minimum, which makes the result
// independent of drain order.  Memory stays O(N + M): no N x M buffer exists.
// One subject against one atlas, as the plain pass sees it.
struct PlainJob {
  const float* fibers;
  int64_t n;
  const float4* ccen;
  const float* cprep;
  int32_t m;
  const int32_t* bid;
  int32_t* labels;
  float* dists;
  Metric mt;
};

template <int FPL, int QCAP, bool STATS>
__device__ __forceinline__ void plain_block(const PlainJob& job, int64_t block,
                                            unsigned long long* __restrict__ counters) {
  const float* __restrict__ fibers = job.fibers;
  const int64_t n = job.n;
  const float4* __restrict__ ccen = job.ccen;
  const float* __restrict__ cprep = job.cprep;
  const int32_t m = job.m;
  const int32_t* __restrict__ bid = job.bid;
  int32_t* __restrict__ labels = job.labels;
  float* __restrict__ dists = job.dists;
  static_assert(64 * FPL <= 256, "slot must fit 8 bits");
  static_assert(QCAP >= 2 * 64 * FPL, "queue must hold two centroids' worth");
  constexpr int WAVES = 4;
  __shared__ uint32_t s_queue[WAVES][QCAP];
  __shared__ uint64_t s_keys[WAVES][64 * FPL];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;
  const int64_t wbase = (block * WAVES + wave) * (64 * FPL);
  WaveQueue wq{s_queue[wave], s_keys[wave]};
  StageCounts sc{counters};

  float ax[FPL], ay[FPL], az[FPL];
#pragma unroll
  for (int k = 0; k < FPL; ++k) {
    const int64_t f = wbase + k * 64 + lane;
    if (f < n) {
      const float* p = fibers + f * NF + 3 * CTR;
      ax[k] = p[0];
      ay[k] = p[1];
      az[k] = p[2];
    } else {
      // a NaN center fails every comparison, so padding lanes never survive
      ax[k] = ay[k] = az[k] = __builtin_nanf("");
    }
    wq.keys[k * 64 + lane] = NO_KEY;
  }
  const float* fib_base = fibers + (wbase < n ? wbase : 0) * NF;

  // Centroids in groups of 4 (one 64-byte scalar burst); ccen is padded to a
  // multiple of 8 with entries that never pass.  The next group is loaded
  // while the current one is evaluated.
  const int32_t m4 = (m + 3) & ~3;
  uint32_t qn = 0;
  float4 n0 = ccen[0], n1 = ccen[1], n2 = ccen[2], n3 = ccen[3];
  for (int32_t c0 = 0; c0 < m4; c0 += 4) {
    const float4 q[4] = {n0, n1, n2, n3};
    const int32_t cn = c0 + 4 < m4 ? c0 + 4 : c0;
    n0 = ccen[cn];
    n1 = ccen[cn + 1];
    n2 = ccen[cn + 2];
    n3 = ccen[cn + 3];
    uint64_t msk[4][FPL];
    uint64_t any = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int k = 0; k < FPL; ++k) {
        msk[u][k] = __ballot(d2(ax[k], ay[k], az[k], q[u].x, q[u].y, q[u].z) <= q[u].w);
        any |= msk[u][k];
      }
    }
    if (any) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t c = (uint32_t)(c0 + u);
#pragma unroll
        for (int k = 0; k < FPL; ++k)
          if (msk[u][k]) queue_push(wq, qn, msk[u][k], (c << 8) | (uint32_t)(k * 64 + lane));
        if (qn > (uint32_t)(QCAP - 64 * FPL)) {
          queue_drain<STATS>(wq, qn, fib_base, cprep, sc, job.mt);
          qn = 0;
        }
      }
    }
  }
  queue_drain<STATS>(wq, qn, fib_base, cprep, sc, job.mt);

#pragma unroll
  for (int k = 0; k < FPL; ++k) {
    const int64_t f = wbase + k * 64 + lane;
    if (f < n) write_result(wq.keys[k * 64 + lane], bid, labels + f, dists + f, job.mt.flags);
  }
}

template <int FPL, int QCAP, bool STATS>
__global__ __launch_bounds__(256) void plain_kernel(PlainJob job,
                                                    unsigned long long* __restrict__ counters) {
  plain_block<FPL, QCAP, STATS>(job, blockIdx.x, counters);
}

// Batch form: one launch over the flattened work list (see
// prefilter_batch_kernel); jobs are ordered by atlas size, largest first.
template <int FPL, int QCAP>
__global__ __launch_bounds__(256) void plain_batch_kernel(const PlainJob* __restrict__ jobs,
                                                          const int64_t* __restrict__ job_start,
                                                          int32_t njobs) {
  const int64_t it = blockIdx.x;
  const int32_t j = find_job(job_start, njobs, it);
  plain_block<FPL, QCAP, false>(jobs[j], it - job_start[j], nullptr);
}

// Survivors of the center test as (fiber, centroid) pairs (diagnostics).
__global__ __launch_bounds__(256) void plain_pairs_kernel(const float* __restrict__ fibers,
                                                          int64_t n,
                                                          const float4* __restrict__ ccen,
                                                          int32_t m, int32_t* __restrict__ pairs,
                                                          int64_t cap,
                                                          unsigned long long* __restrict__ count) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const float* p = fibers + f * NF + 3 * CTR;
  const float x = p[0], y = p[1], z = p[2];
  for (int32_t c = 0; c < m; ++c) {
    const float4 q = ccen[c];
    if (d2(x, y, z, q.x, q.y, q.z) <= q.w) {
      unsigned long long k = atomicAdd(count, 1ull);
      if ((int64_t)k < cap) {
        pairs[2 * k] = (int32_t)f;
        pairs[2 * k + 1] = c;
      }
    }
  }
}

// ---------------------------------------------------------------- launchers

int launch_prep_atlas(const float* cen, int64_t m, const int32_t* bid, const float* thr,
                      int32_t nb, float* cprep, float4* ccen, int32_t* bid_out, float* cext,
                      unsigned int* flags, hipStream_t s) {
  if (m > 0) {
    const int64_t mp = (m + 7) & ~(int64_t)7;
    // one wave per block: each lane reads a 252-byte record on its own, so the
    // work is spread over as many CUs as there are waves
    prep_atlas_kernel<<<(unsigned)((mp + 63) / 64), 64, 0, s>>>(cen, m, bid, thr, nb, cprep, ccen,
                                                                bid_out, cext, flags);
  }
  else if (nb > 0)  // (prep_atlas_kernel checks the thresholds when it runs)
    check_thresholds_kernel<<<(nb + 255) / 256, 256, 0, s>>>(thr, nb, flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_check_finite(const float* v, int64_t count, unsigned int* flags, hipStream_t s) {
  if (count <= 0) return 0;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  check_finite_kernel<<<(unsigned)blocks, 256, 0, s>>>(v, count, flags);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s) {
  if (n > 0) fill_u64_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n, v);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill_empty(int64_t n, int32_t* labels, float* dists, hipStream_t s) {
  if (n > 0) fill_empty_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, labels, dists);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_dense(const float* fibers, int64_t n, const float* cprep, int32_t m,
                 const int32_t* bid, int32_t* labels, float* dists, int cfg, Metric mt,
                 hipStream_t s) {
  // cfg 1: one fiber per lane; cfg 2: two fibers per lane
  const int fpl = cfg == 2 ? 2 : 1;
  const int64_t per_block = 256 * fpl;
  const unsigned blocks = (unsigned)((n + per_block - 1) / per_block);
  if (mt.flags)
    dense_kernel<1, true><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(fibers, n, cprep, m, bid,
                                                                      labels, dists, mt);
  else if (fpl == 2)
    dense_kernel<2, false><<<blocks, 256, 0, s>>>(fibers, n, cprep, m, bid, labels, dists, mt);
  else
    dense_kernel<1, false><<<blocks, 256, 0, s>>>(fibers, n, cprep, m, bid, labels, dists, mt);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int FPL>
static void plain_launch(const float* fibers, int64_t n, const float4* ccen, const float* cprep,
                         int32_t m, const int32_t* bid, int32_t* labels, float* dists,
                         unsigned long long* counters, Metric mt, hipStream_t s) {
  constexpr int per_block = 4 * 64 * FPL;
  const unsigned blocks = (unsigned)((n + per_block - 1) / per_block);
  constexpr int QCAP = 512;
  const PlainJob job{fibers, n, ccen, cprep, m, bid, labels, dists, mt};
  if (counters)
    plain_kernel<FPL, QCAP, true><<<blocks, 256, 0, s>>>(job, counters);
  else
    plain_kernel<FPL, QCAP, false><<<blocks, 256, 0, s>>>(job, counters);
}

int plain_default_cfg(int64_t n) {
  // enough waves to fill 256 CUs x 4 SIMDs several times over
  const int64_t want_waves = 256 * 4 * 8;
  if (n >= want_waves * 64 * 4) return 4;
  if (n >= want_waves * 64 * 2) return 2;
  return 1;
}

int launch_plain(const float* fibers, int64_t n, const float4* ccen, const float* cprep,
                 int32_t m, const int32_t* bid, int32_t* labels, float* dists,
                 unsigned long long* counters, int cfg, Metric mt, hipStream_t s) {
  if (cfg <= 0) cfg = plain_default_cfg(n);
  switch (cfg) {
    case 1: plain_launch<1>(fibers, n, ccen, cprep, m, bid, labels, dists, counters, mt, s); break;
    case 2: plain_launch<2>(fibers, n, ccen, cprep, m, bid, labels, dists, counters, mt, s); break;
    case 4: plain_launch<4>(fibers, n, ccen, cprep, m, bid, labels, dists, counters, mt, s); break;
    default: return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

namespace {

int grow_buf(void** p, size_t* have, size_t want) {
  if (want <= *have) return 0;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  if (hipMalloc(p, want) != hipSuccess) return -3;
  *have = want;
  return 0;
}

template <int FPL>
int plain_batch_cfg(int cfg, const BatchAtlas* at, int32_t na, const float* const* fibers,
                    const int64_t* nf, int32_t ns, int32_t* const* labels, float* const* dists,
                    int mflags, BatchBuf& bb, hipStream_t s) {
  constexpr int QCAP = 512;
  constexpr int64_t FPB = 4 * 64 * FPL;
  std::vector<uint64_t> key = {1u, (uint64_t)cfg, (uint64_t)na, (uint64_t)ns, (uint64_t)mflags};
  for (int32_t a = 0; a < na; ++a) {
    key.push_back((uint64_t)(uintptr_t)at[a].ccen);
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
  if (!(bb.exec && bb.key == key)) {
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    std::vector<int32_t> order(na);
    for (int32_t a = 0; a < na; ++a) order[a] = a;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return at[x].m > at[y].m; });
    std::vector<PlainJob> jobs;
    std::vector<int64_t> start(1, 0);
    for (int32_t oi = 0; oi < na; ++oi) {
      const int32_t a = order[oi];
      if (at[a].m == 0) continue;
      for (int32_t i = 0; i < ns; ++i) {
        if (nf[i] == 0) continue;
        jobs.push_back(PlainJob{fibers[i], nf[i], at[a].ccen, at[a].cprep, at[a].m, at[a].bid,
                                labels[i * na + a], dists[i * na + a],
                                Metric{at[a].cext, mflags}});
        start.push_back(start.back() + (nf[i] + FPB - 1) / FPB);
      }
    }
    const size_t need = 256 + jobs.size() * sizeof(PlainJob) + start.size() * sizeof(int64_t);
    int rc = grow_buf(&bb.items, &bb.items_bytes, need);
    if (rc) return rc;
    std::vector<uint8_t> host(need - 256);
    if (!jobs.empty()) memcpy(host.data(), jobs.data(), jobs.size() * sizeof(PlainJob));
    memcpy(host.data() + jobs.size() * sizeof(PlainJob), start.data(),
           start.size() * sizeof(int64_t));
    if (hipMemcpy((uint8_t*)bb.items + 256, host.data(), host.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
      return -1;
    bb.key.clear();
    bb.njobs = (int32_t)jobs.size();
  }
  const PlainJob* djobs = (const PlainJob*)((uint8_t*)bb.items + 256);
  const int64_t* dstart = (const int64_t*)((uint8_t*)bb.items + 256 + bb.njobs * sizeof(PlainJob));
  const int32_t njobs = bb.njobs;
  int64_t total = 0;  // work items (fiber blocks over all jobs)
  for (int32_t a = 0; a < na; ++a)
    if (at[a].m > 0)
      for (int32_t i = 0; i < ns; ++i) total += (nf[i] + FPB - 1) / FPB;
  auto enqueue = [&](hipStream_t cs) -> int {
    for (int32_t a = 0; a < na; ++a)
      if (at[a].m == 0)
        for (int32_t i = 0; i < ns; ++i)
          if (launch_fill_empty(nf[i], labels[i * na + a], dists[i * na + a], cs)) return -1;
    if (njobs > 0 && total > 0)
      plain_batch_kernel<FPL, QCAP><<<(unsigned)total, 256, 0, cs>>>(djobs, dstart, njobs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  };
  return graph_launch(bb, key, s, enqueue);
}

}  // namespace

int plain_batch(int cfg, const BatchAtlas* atlases, int32_t n_atlases, const float* const* fibers,
                const int64_t* n_fibers, int32_t n_subjects, int32_t* const* labels,
                float* const* dists, int mflags, BatchBuf& bb, hipStream_t s) {
  switch (cfg) {
    case 0:
    case 4:
      return plain_batch_cfg<4>(cfg, atlases, n_atlases, fibers, n_fibers, n_subjects, labels,
                                dists, mflags, bb, s);
    case 1:
      return plain_batch_cfg<1>(cfg, atlases, n_atlases, fibers, n_fibers, n_subjects, labels,
                                dists, mflags, bb, s);
    case 2:
      return plain_batch_cfg<2>(cfg, atlases, n_atlases, fibers, n_fibers, n_subjects, labels,
                                dists, mflags, bb, s);
    default:
      return -2;
  }
}

int launch_plain_pairs(const float* fibers, int64_t n, const float4* ccen, int32_t m,
                       int32_t* pairs, int64_t cap, unsigned long long* count, hipStream_t s) {
  plain_pairs_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(fibers, n, ccen, m, pairs, cap,
                                                                 count);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace seg
