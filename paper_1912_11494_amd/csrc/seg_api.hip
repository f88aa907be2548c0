// C ABI of libseg.so: argument checks, scratch, validation and launches.
// The operation and its arithmetic contract are documented in include/seg.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <tuple>
#include <vector>

#include "seg.h"
#include "seg_internal.hpp"

namespace {

thread_local std::string t_err;

int fail(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SEG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
  } while (0)

constexpr int64_t kMaxCentroids = (int64_t)1 << 24;  // queue entries hold 24-bit indices

int64_t pad8(int64_t m) { return (m + 7) & ~(int64_t)7; }

// Prepared atlas data in device memory.
struct AtlasBuf {
  float* cprep = nullptr;   // [m_pad][64]
  float4* ccen = nullptr;   // [m_pad]
  int32_t* bid = nullptr;   // [m_pad]
  float* cext = nullptr;    // [m_pad][2]: arc length, threshold T
  int32_t* cperm = nullptr; // [m_pad + 8]: tile-culled centroid order (a prepared atlas),
                            // then its frame at [m, m + 6)
  bool cperm_ok = false;    // cperm holds this atlas's order
  int64_t cap = 0;          // capacity in centroids
  int64_t m = 0;

  int reserve(int64_t mp) {
    cperm_ok = false;
    if (mp <= cap) return 0;
    release();
    HIP_TRY(hipMalloc(&cprep, (size_t)mp * seg::CREC_BYTES));
    HIP_TRY(hipMalloc(&ccen, (size_t)mp * sizeof(float4)));
    HIP_TRY(hipMalloc(&bid, (size_t)mp * sizeof(int32_t)));
    HIP_TRY(hipMalloc(&cext, (size_t)mp * 2 * sizeof(float)));
    HIP_TRY(hipMalloc(&cperm, (size_t)(mp + 8) * sizeof(int32_t)));
    cap = mp;
    return 0;
  }
  void release() {
    if (cprep) (void)hipFree(cprep);
    if (ccen) (void)hipFree(ccen);
    if (bid) (void)hipFree(bid);
    if (cext) (void)hipFree(cext);
    if (cperm) (void)hipFree(cperm);
    cprep = nullptr;
    ccen = nullptr;
    bid = nullptr;
    cext = nullptr;
    cperm = nullptr;
    cperm_ok = false;
    cap = 0;
  }
  const int32_t* order() const { return cperm_ok ? cperm : nullptr; }
};

// Per (device, stream) scratch: atlas copy for one-shot calls, flags, counters.
struct Scratch {
  int device = 0;
  hipStream_t stream = nullptr;
  AtlasBuf atlas;
  unsigned long long* flags = nullptr;     // [1]
  unsigned long long* counters = nullptr;  // [NCOUNTERS]
  seg::PrefilterBuf pre;
  seg::BatchBuf batch;
  void* mslots = nullptr;  // several labels: per-fiber bundle slots
  size_t mslots_bytes = 0;
  bool mslots_zero = false;  // every slot is 0 (each completed call leaves it so)
  void* mscan = nullptr;   // several labels: scan partials
  size_t mscan_bytes = 0;

  int init() {
    if (!flags) HIP_TRY(hipMalloc(&flags, sizeof(unsigned long long)));
    if (!counters) HIP_TRY(hipMalloc(&counters, seg::NCOUNTERS * sizeof(unsigned long long)));
    return 0;
  }
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Scratch*> g_scratch;

int get_scratch(hipStream_t s, Scratch** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, s);
  auto it = g_scratch.find(key);
  if (it == g_scratch.end()) {
    Scratch* sc = new Scratch();
    sc->device = dev;
    sc->stream = s;
    int rc = sc->init();
    if (rc) {
      delete sc;
      return rc;
    }
    it = g_scratch.emplace(key, sc).first;
  }
  *out = it->second;
  return 0;
}

// Tuned tile per (mode, floor(log2 N), floor(log2 M)).
struct Tuned {
  int tile;
  float ms;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Tuned> g_tuned;

int ilog2(int64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
}

int tuned_tile(int mode, int64_t n, int64_t m) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(std::make_tuple(mode, ilog2(n), ilog2(m)));
  return it == g_tuned.end() ? 0 : it->second.tile;
}

// Kernel configurations of a mode (see the launchers).
std::vector<int> mode_tiles(int mode) {
  switch (mode) {
    case SEG_DENSE: return {1, 2};
    case SEG_PLAIN: return {1, 2, 4};
    case SEG_PREFILTER_BF16_ORIENTED: return {1, 2};
    default: return {1, 3, 4, 6, 8};  // symmetric prefilters (K, fiber groups; 8: culled)
  }
}

// State for seg_query_stats.
thread_local unsigned long long* t_stats_counters = nullptr;
thread_local hipStream_t t_stats_stream = nullptr;
thread_local int64_t t_stats_pairs = 0;
thread_local int64_t t_stats_n = 0;
thread_local int32_t* t_stats_labels = nullptr;
thread_local int t_stats_mode = 0;
thread_local bool t_stats_culled = false;

bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

int check_mode(int mode) {
  switch (mode) {
    case SEG_DENSE:
    case SEG_PLAIN:
    case SEG_PREFILTER_BF16:
    case SEG_PREFILTER_FP16:
    case SEG_PREFILTER_FP8:
    case SEG_PREFILTER_BF16_ORIENTED:
      return 0;
    default:
      return fail(SEG_EMODE, "unknown mode " + std::to_string(mode));
  }
}

int check_metric(int flags) {
  if (flags & ~(SEG_METRIC_LENGTH_NORM | SEG_METRIC_DIRECTION))
    return fail(SEG_EINVAL, "unknown metric flag");
  return 0;
}

int check_atlas_args(const float* centroids, int64_t m, const int32_t* bid, const float* thr,
                     int32_t nb) {
  if (m < 0) return fail(SEG_EINVAL, "n_centroids < 0");
  if (m >= kMaxCentroids) return fail(SEG_ERANGE, "n_centroids must be below 2^24");
  if (m > 0 && nb <= 0) return fail(SEG_EINVAL, "n_bundles must be positive when centroids exist");
  if (m > 0 && (!centroids || !bid)) return fail(SEG_EINVAL, "null centroid or bundle-id pointer");
  if (nb > 0 && !thr) return fail(SEG_EINVAL, "null threshold pointer");
  if (!aligned4(centroids) || !aligned4(bid) || !aligned4(thr))
    return fail(SEG_EINVAL, "atlas pointers must be 4-byte aligned");
  return 0;
}

// Prepare an atlas into `ab` on stream s; flags collects validation bits.
int prepare_atlas(AtlasBuf& ab, const float* centroids, int64_t m, const int32_t* bid,
                  const float* thr, int32_t nb, unsigned long long* flags, hipStream_t s) {
  int rc = ab.reserve(pad8(m > 0 ? m : 1));
  if (rc) return rc;
  ab.m = m;
  if (seg::launch_prep_atlas(centroids, m, bid, thr, nb, ab.cprep, ab.ccen, ab.bid, ab.cext,
                             (unsigned int*)flags, s))
    return hip_fail(hipGetLastError(), "prep_atlas launch");
  return 0;
}

int read_flags(unsigned long long* flags, hipStream_t s, unsigned long long* out) {
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(out, flags, sizeof(*out), hipMemcpyDeviceToHost));
  return 0;
}

int flags_error(unsigned long long f) {
  if (f & seg::FLAG_BUNDLE) return fail(SEG_EBUNDLE, "a centroid bundle id is outside [0, n_bundles)");
  if (f & seg::FLAG_NONFINITE) return fail(SEG_ENONFINITE, "non-finite coordinate or NaN threshold");
  return 0;
}

seg_options resolve(const seg_options* opt) {
  seg_options o;
  seg_default_options(&o);
  if (opt) o = *opt;
  return o;
}

// Launch the per-pair path of `mode` for one subject against a prepared atlas.
// `counter_buf` holds NCOUNTERS words; `pre` is the prefilter scratch (null:
// the prefilter modes are refused).
int run_mode(const seg_options& o, const AtlasBuf& ab, unsigned long long* counter_buf,
             seg::PrefilterBuf* pre, const float* fibers, int64_t n, int32_t* labels,
             float* dists, hipStream_t s) {
  unsigned long long* counters = o.collect_stats ? counter_buf : nullptr;
  if (counters && seg::launch_fill_u64(counters, seg::NCOUNTERS, 0ull, s))
    return hip_fail(hipGetLastError(), "counter reset");
  const int32_t m = (int32_t)ab.m;
  hipEvent_t* ev = (hipEvent_t*)o.profile_events;
  const int tile = o.tile ? o.tile : tuned_tile(o.mode, n, m);
  const seg::Metric mt{ab.cext, o.metric};
  int rc = 0;
  switch (o.mode) {
    case SEG_DENSE:
      if (ev) HIP_TRY(hipEventRecord(ev[0], s));
      rc = seg::launch_dense(fibers, n, ab.cprep, m, ab.bid, labels, dists, tile, mt, s);
      if (ev && !rc) HIP_TRY(hipEventRecord(ev[1], s));
      break;
    case SEG_PLAIN:
      if (ev) HIP_TRY(hipEventRecord(ev[0], s));
      rc = seg::launch_plain(fibers, n, ab.ccen, ab.cprep, m, ab.bid, labels, dists, counters,
                             tile, mt, s);
      if (ev && !rc) HIP_TRY(hipEventRecord(ev[1], s));
      break;
    default:
      if (!pre) return fail(SEG_EMODE, "this entry point runs the dense and plain modes only");
      rc = seg::run_prefilter(o.mode, tile, fibers, n, ab.cprep, ab.ccen, m, ab.bid, labels,
                              dists, counters, mt, *pre, ev, s, ab.order());
      if (rc == -3) return fail(SEG_ENOMEM, "prefilter scratch allocation failed");
      break;
  }
  if (rc == -2) return fail(SEG_EMODE, "unknown tile configuration " + std::to_string(tile));
  if (rc == -4) return fail(SEG_ERANGE, "the tile-culled form takes fewer than 2^31 fibers");
  if (rc) return hip_fail(hipGetLastError(), "kernel launch");
  if (o.collect_stats) {
    t_stats_counters = counters;
    t_stats_stream = s;
    t_stats_pairs = n * ab.m;
    t_stats_n = n;
    t_stats_labels = labels;
    t_stats_mode = o.mode;
    t_stats_culled = o.mode >= SEG_PREFILTER_BF16 && o.mode <= SEG_PREFILTER_FP8 &&
                     (tile == 8 || (tile == 0 && n < ((int64_t)1 << 31)));
  }
  return 0;
}

}  // namespace

// ---- scratch of the entry point that allocates nothing (seg_segment_noalloc)
//
// A fixed array in device memory: the validation flag, the statistics
// counters and the prepared atlas (records, centers, bundle ids, arc length
// and threshold) of up to SEG_NOALLOC_MAX_CENTROIDS centroids.  Every device
// the library runs on holds its own copy from module load until the process
// ends.  In host code the array's name is not a device address: host code
// takes each device's address once from hipGetSymbolAddress and uses only
// that.  Calls that overlap on one device share the array and race.
namespace {
constexpr int64_t kNaMaxM = SEG_NOALLOC_MAX_CENTROIDS;  // a multiple of 8
constexpr size_t kNaFlags = 0;                          // 8 bytes
constexpr size_t kNaCounters = 256;                     // NCOUNTERS words
constexpr size_t kNaCprep = 512;
constexpr size_t kNaCcen = kNaCprep + (size_t)kNaMaxM * seg::CREC_BYTES;
constexpr size_t kNaBid = kNaCcen + (size_t)kNaMaxM * sizeof(float4);
constexpr size_t kNaCext = kNaBid + (size_t)kNaMaxM * sizeof(int32_t);
constexpr size_t kNaBytes = kNaCext + (size_t)kNaMaxM * 2 * sizeof(float);
static_assert(kNaMaxM % 8 == 0, "padded atlas fits");
static_assert(seg::NCOUNTERS * sizeof(unsigned long long) <= kNaCprep - kNaCounters, "counters fit");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kNaDevices = 64;
std::mutex g_na_mu;
unsigned char* g_na_ptr[kNaDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call there (with that device current) and kept.
int noalloc_scratch(unsigned char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaDevices) return fail(SEG_ERANGE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SEG_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_na_ptr[dev] = (unsigned char*)p;
  }
  *out = g_na_ptr[dev];
  return 0;
}

}  // namespace

struct seg_atlas {
  int device = 0;
  AtlasBuf buf;
  int32_t n_bundles = 0;
};

extern "C" {

void seg_default_options(seg_options* opt) {
  if (!opt) return;
  opt->mode = SEG_PLAIN;
  opt->validate = 0;
  opt->tile = 0;
  opt->collect_stats = 0;
  opt->profile_events = nullptr;
  opt->metric = 0;
}

const char* seg_last_error(void) { return t_err.c_str(); }

int seg_version(void) { return SEG_VERSION; }

int seg_segment(const float* fibers, int64_t n, const float* centroids, int64_t m,
                const int32_t* bid, const float* thr, int32_t nb, int32_t* labels, float* dists,
                const seg_options* opt, void* stream) {
  t_err.clear();
  const seg_options o = resolve(opt);
  int rc = check_mode(o.mode);
  if (!rc) rc = check_metric(o.metric);
  if (rc) return rc;
  if (n < 0) return fail(SEG_EINVAL, "n_fibers < 0");
  rc = check_atlas_args(centroids, m, bid, thr, nb);
  if (rc) return rc;
  if (n > 0 && (!fibers || !labels || !dists)) return fail(SEG_EINVAL, "null fiber/output pointer");
  if (!aligned4(fibers) || !aligned4(labels) || !aligned4(dists))
    return fail(SEG_EINVAL, "fiber/output pointers must be 4-byte aligned");
  if (n == 0) return SEG_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch* sc = nullptr;
  rc = get_scratch(s, &sc);
  if (rc) return rc;
  if (o.validate && seg::launch_fill_u64(sc->flags, 1, 0ull, s))
    return hip_fail(hipGetLastError(), "flag reset");
  if (m == 0) {
    if (o.validate) {
      if (seg::launch_check_finite(fibers, n * 63, (unsigned int*)sc->flags, s))
        return hip_fail(hipGetLastError(), "validation launch");
      unsigned long long f = 0;
      rc = read_flags(sc->flags, s, &f);
      if (rc) return rc;
      rc = flags_error(f);
      if (rc) return rc;
    }
    if (seg::launch_fill_empty(n, labels, dists, s)) return hip_fail(hipGetLastError(), "fill");
    return SEG_OK;
  }
  rc = prepare_atlas(sc->atlas, centroids, m, bid, thr, nb, sc->flags, s);
  if (rc) return rc;
  if (o.validate) {
    if (seg::launch_check_finite(fibers, n * 63, (unsigned int*)sc->flags, s))
      return hip_fail(hipGetLastError(), "validation launch");
    unsigned long long f = 0;
    rc = read_flags(sc->flags, s, &f);
    if (rc) return rc;
    rc = flags_error(f);
    if (rc) return rc;
  }
  return run_mode(o, sc->atlas, sc->counters, &sc->pre, fibers, n, labels, dists, s);
}

int seg_segment_noalloc(const float* fibers, int64_t n, const float* centroids, int64_t m,
                        const int32_t* bid, const float* thr, int32_t nb, int32_t* labels,
                        float* dists, const seg_options* opt, void* stream) {
  t_err.clear();
  const seg_options o = resolve(opt);
  int rc = check_mode(o.mode);
  if (!rc) rc = check_metric(o.metric);
  if (rc) return rc;
  if (o.mode != SEG_DENSE && o.mode != SEG_PLAIN)
    return fail(SEG_EMODE, "seg_segment_noalloc runs the dense and plain modes");
  if (n < 0) return fail(SEG_EINVAL, "n_fibers < 0");
  rc = check_atlas_args(centroids, m, bid, thr, nb);
  if (rc) return rc;
  if (m > kNaMaxM)
    return fail(SEG_ERANGE, "seg_segment_noalloc takes at most " + std::to_string(kNaMaxM) +
                                " centroids");
  if (n > 0 && (!fibers || !labels || !dists)) return fail(SEG_EINVAL, "null fiber/output pointer");
  if (!aligned4(fibers) || !aligned4(labels) || !aligned4(dists))
    return fail(SEG_EINVAL, "fiber/output pointers must be 4-byte aligned");
  if (n == 0) return SEG_OK;
  hipStream_t s = (hipStream_t)stream;
  unsigned char* base = nullptr;
  rc = noalloc_scratch(&base);
  if (rc) return rc;
  unsigned long long* flags = (unsigned long long*)(base + kNaFlags);
  unsigned long long* counters = (unsigned long long*)(base + kNaCounters);
  // a view of the array as a prepared atlas (never released)
  AtlasBuf ab;
  ab.cprep = (float*)(base + kNaCprep);
  ab.ccen = (float4*)(base + kNaCcen);
  ab.bid = (int32_t*)(base + kNaBid);
  ab.cext = (float*)(base + kNaCext);
  ab.cap = kNaMaxM;
  ab.m = m;
  if (o.validate && seg::launch_fill_u64(flags, 1, 0ull, s))
    return hip_fail(hipGetLastError(), "flag reset");
  if (m > 0 && seg::launch_prep_atlas(centroids, m, bid, thr, nb, ab.cprep, ab.ccen, ab.bid,
                                      ab.cext, (unsigned int*)flags, s))
    return hip_fail(hipGetLastError(), "prep_atlas launch");
  if (o.validate) {
    if (seg::launch_check_finite(fibers, n * 63, (unsigned int*)flags, s))
      return hip_fail(hipGetLastError(), "validation launch");
    unsigned long long f = 0;
    rc = read_flags(flags, s, &f);
    if (rc) return rc;
    rc = flags_error(f);
    if (rc) return rc;
  }
  if (m == 0) {
    if (seg::launch_fill_empty(n, labels, dists, s)) return hip_fail(hipGetLastError(), "fill");
    return SEG_OK;
  }
  return run_mode(o, ab, counters, nullptr, fibers, n, labels, dists, s);
}

int seg_atlas_create(const float* centroids, int64_t m, const int32_t* bid, const float* thr,
                     int32_t nb, void* stream, seg_atlas** out) {
  t_err.clear();
  if (!out) return fail(SEG_EINVAL, "null output handle");
  *out = nullptr;
  int rc = check_atlas_args(centroids, m, bid, thr, nb);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Scratch* sc = nullptr;
  rc = get_scratch(s, &sc);
  if (rc) return rc;
  seg_atlas* a = new seg_atlas();
  HIP_TRY(hipGetDevice(&a->device));
  a->n_bundles = nb;
  if (seg::launch_fill_u64(sc->flags, 1, 0ull, s)) {
    delete a;
    return hip_fail(hipGetLastError(), "flag reset");
  }
  rc = prepare_atlas(a->buf, centroids, m, bid, thr, nb, sc->flags, s);
  // the tile-culled centroid order depends only on the atlas: sorted once
  // here, and complete before the handle is returned (read_flags waits)
  if (!rc && m > 0) {
    const int r = seg::cull_sort_centroids(a->buf.cprep, (int32_t)m, a->buf.cperm, sc->pre, s);
    if (r == -3) rc = fail(SEG_ENOMEM, "prefilter scratch allocation failed");
    else if (r) rc = hip_fail(hipGetLastError(), "centroid order launch");
  }
  unsigned long long f = 0;
  if (!rc) rc = read_flags(sc->flags, s, &f);
  if (!rc) rc = flags_error(f);
  if (rc) {
    a->buf.release();
    delete a;
    return rc;
  }
  a->buf.cperm_ok = m > 0;
  *out = a;
  return SEG_OK;
}

void seg_atlas_destroy(seg_atlas* a) {
  if (!a) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(a->device);
  a->buf.release();
  (void)hipSetDevice(prev);
  delete a;
}

int64_t seg_atlas_size(const seg_atlas* a) { return a ? a->buf.m : -1; }

int seg_segment_atlas(const seg_atlas* a, const float* fibers, int64_t n, int32_t* labels,
                      float* dists, const seg_options* opt, void* stream) {
  t_err.clear();
  if (!a) return fail(SEG_EINVAL, "null atlas");
  const seg_options o = resolve(opt);
  int rc = check_mode(o.mode);
  if (!rc) rc = check_metric(o.metric);
  if (rc) return rc;
  if (n < 0) return fail(SEG_EINVAL, "n_fibers < 0");
  if (n > 0 && (!fibers || !labels || !dists)) return fail(SEG_EINVAL, "null fiber/output pointer");
  if (!aligned4(fibers) || !aligned4(labels) || !aligned4(dists))
    return fail(SEG_EINVAL, "fiber/output pointers must be 4-byte aligned");
  if (n == 0) return SEG_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch* sc = nullptr;
  rc = get_scratch(s, &sc);
  if (rc) return rc;
  if (a->buf.m == 0) {
    if (seg::launch_fill_empty(n, labels, dists, s)) return hip_fail(hipGetLastError(), "fill");
    return SEG_OK;
  }
  if (o.validate) {
    if (seg::launch_fill_u64(sc->flags, 1, 0ull, s) ||
        seg::launch_check_finite(fibers, n * 63, (unsigned int*)sc->flags, s))
      return hip_fail(hipGetLastError(), "validation launch");
    unsigned long long f = 0;
    rc = read_flags(sc->flags, s, &f);
    if (rc) return rc;
    rc = flags_error(f);
    if (rc) return rc;
  }
  return run_mode(o, a->buf, sc->counters, &sc->pre, fibers, n, labels, dists, s);
}

int seg_segment_multi(const seg_atlas* a, const float* fibers, int64_t n, int32_t max_per_fiber,
                      int64_t* offsets, int32_t* bundles, float* dists, int64_t capacity,
                      int64_t* total, int64_t* bundle_counts, const seg_options* opt,
                      void* stream) {
  t_err.clear();
  if (!a) return fail(SEG_EINVAL, "null atlas");
  if (!total) return fail(SEG_EINVAL, "null total pointer");
  *total = 0;
  const seg_options o = resolve(opt);
  int rc = check_mode(o.mode);
  if (!rc) rc = check_metric(o.metric);
  if (rc) return rc;
  if (o.mode != SEG_PREFILTER_BF16 && o.mode != SEG_PREFILTER_FP16 && o.mode != SEG_PREFILTER_FP8)
    return fail(SEG_EMODE, "several labels per fiber use the tile-culled prefilter (bf16, fp16, fp8)");
  if (o.tile != 0 && o.tile != 8)
    return fail(SEG_EMODE, "several labels per fiber use the tile-culled form (tile 0 or 8)");
  if (max_per_fiber < 1 || max_per_fiber > 16) return fail(SEG_EINVAL, "max_per_fiber must be 1..16");
  if (n < 0 || capacity < 0) return fail(SEG_EINVAL, "negative fiber count or capacity");
  if (n >= ((int64_t)1 << 31)) return fail(SEG_ERANGE, "several labels need fewer than 2^31 fibers");
  if (!offsets || (n > 0 && !fibers) || (capacity > 0 && (!bundles || !dists)))
    return fail(SEG_EINVAL, "null fiber/offset/entry pointer");
  if (!aligned4(fibers) || !aligned4(bundles) || !aligned4(dists) || ((uintptr_t)offsets & 7u) ||
      ((uintptr_t)bundle_counts & 7u))
    return fail(SEG_EINVAL, "misaligned pointer");
  hipStream_t s = (hipStream_t)stream;
  Scratch* sc = nullptr;
  rc = get_scratch(s, &sc);
  if (rc) return rc;
  if (o.validate && n > 0) {
    if (seg::launch_fill_u64(sc->flags, 1, 0ull, s) ||
        seg::launch_check_finite(fibers, n * 63, (unsigned int*)sc->flags, s))
      return hip_fail(hipGetLastError(), "validation launch");
    unsigned long long f = 0;
    rc = read_flags(sc->flags, s, &f);
    if (rc) return rc;
    rc = flags_error(f);
    if (rc) return rc;
  }
  const size_t sbytes = (size_t)(n > 0 ? n : 1) * max_per_fiber * sizeof(unsigned long long);
  if (sbytes > sc->mslots_bytes) {
    if (sc->mslots) (void)hipFree(sc->mslots);
    sc->mslots = nullptr;
    sc->mslots_bytes = 0;
    if (hipMalloc(&sc->mslots, sbytes) != hipSuccess)
      return fail(SEG_ENOMEM, "several-label slot allocation failed");
    sc->mslots_bytes = sbytes;
    sc->mslots_zero = false;
  }
  unsigned long long* slots = (unsigned long long*)sc->mslots;
  // the collection clears the slots it reads, so only a new table (or one
  // left by a failed launch) needs a full clear
  if (!sc->mslots_zero &&
      seg::launch_fill_zero_u64(slots, (int64_t)(sc->mslots_bytes / sizeof(unsigned long long)), s))
    return hip_fail(hipGetLastError(), "slot reset");
  sc->mslots_zero = false;
  if (seg::launch_fill_u64(sc->flags, 1, 0ull, s)) return hip_fail(hipGetLastError(), "flag reset");
  unsigned long long* counters = o.collect_stats ? sc->counters : nullptr;
  if (counters && seg::launch_fill_u64(counters, seg::NCOUNTERS, 0ull, s))
    return hip_fail(hipGetLastError(), "counter reset");
  if (n > 0 && a->buf.m > 0) {
    const seg::Metric mt{a->buf.cext, o.metric};
    const seg::MultiOut mo{slots, max_per_fiber, a->buf.bid, (unsigned int*)sc->flags};
    rc = seg::run_cull(o.mode - SEG_PREFILTER_BF16, fibers, n, a->buf.cprep, (int32_t)a->buf.m,
                       a->buf.bid, nullptr, nullptr, counters, mt, sc->pre,
                       (hipEvent_t*)o.profile_events, s, &mo, a->buf.order());
    if (rc == -3) return fail(SEG_ENOMEM, "prefilter scratch allocation failed");
    if (rc) return hip_fail(hipGetLastError(), "kernel launch");
  }
  rc = seg::multi_collect(slots, max_per_fiber, n, offsets, bundles, dists, capacity,
                          bundle_counts, a->n_bundles, o.metric, &sc->mscan, &sc->mscan_bytes, s);
  if (rc == -3) return fail(SEG_ENOMEM, "scan scratch allocation failed");
  if (rc) return hip_fail(hipGetLastError(), "several-label collection launch");
  sc->mslots_zero = true;
  if (o.collect_stats) {
    t_stats_counters = counters;
    t_stats_stream = s;
    t_stats_pairs = n * a->buf.m;
    t_stats_n = n;
    t_stats_labels = nullptr;
    t_stats_mode = o.mode;
    t_stats_culled = true;
  }
  unsigned long long f = 0;
  rc = read_flags(sc->flags, s, &f);
  if (rc) return rc;
  int64_t tot = 0;
  HIP_TRY(hipMemcpy(&tot, offsets + n, sizeof(tot), hipMemcpyDeviceToHost));
  *total = tot;
  if (f & seg::FLAG_MULTI)
    return fail(SEG_ERANGE, "a fiber passes more bundles than max_per_fiber");
  if (tot > capacity)
    return fail(SEG_ECAPACITY, "more label entries (" + std::to_string(tot) + ") than capacity");
  return SEG_OK;
}

int seg_resample(const float* points, int64_t n_points, const int64_t* offsets, int64_t n,
                 float* fibers, int32_t validate, void* stream) {
  t_err.clear();
  if (n < 0 || n_points < 0) return fail(SEG_EINVAL, "negative streamline or point count");
  if (n == 0) return SEG_OK;
  if (!offsets || !fibers || (n_points > 0 && !points))
    return fail(SEG_EINVAL, "null points/offsets/fibers pointer");
  if (!aligned4(points) || !aligned4(fibers) || ((uintptr_t)offsets & 7u))
    return fail(SEG_EINVAL, "points/fibers must be 4-byte and offsets 8-byte aligned");
  if (n_points > ((int64_t)1 << 60)) return fail(SEG_ERANGE, "n_points too large");
  hipStream_t s = (hipStream_t)stream;
  Scratch* sc = nullptr;
  int rc = get_scratch(s, &sc);
  if (rc) return rc;
  unsigned int* flags = nullptr;
  if (validate) {
    if (seg::launch_fill_u64(sc->flags, 1, 0ull, s)) return hip_fail(hipGetLastError(), "flag reset");
    flags = (unsigned int*)sc->flags;
  }
  if (validate && n_points > 0 && seg::launch_check_finite(points, n_points * 3, flags, s))
    return hip_fail(hipGetLastError(), "validation launch");
  if (seg::launch_resample(points, n_points, offsets, n, fibers, flags, s))
    return hip_fail(hipGetLastError(), "resample launch");
  if (validate) {
    unsigned long long f = 0;
    rc = read_flags(sc->flags, s, &f);
    if (rc) return rc;
    if (f & seg::FLAG_OFFSETS)
      return fail(SEG_EOFFSETS, "a streamline is empty or its offsets leave [0, n_points]");
    if (f & seg::FLAG_NONFINITE) return fail(SEG_ENONFINITE, "non-finite streamline coordinate");
  }
  return SEG_OK;
}

int seg_segment_streamlines(const seg_atlas* a, const float* points, int64_t n_points,
                            const int64_t* offsets, int64_t n, float* fibers, int32_t* labels,
                            float* dists, const seg_options* opt, void* stream) {
  t_err.clear();
  if (!a) return fail(SEG_EINVAL, "null atlas");
  const seg_options o = resolve(opt);
  int rc = check_mode(o.mode);
  if (!rc) rc = check_metric(o.metric);
  if (rc) return rc;
  rc = seg_resample(points, n_points, offsets, n, fibers, o.validate, stream);
  if (rc) return rc;
  return seg_segment_atlas(a, fibers, n, labels, dists, &o, stream);
}

int seg_segment_batch(const seg_atlas* const* atlases, int32_t n_atlases, const float* const* fibers,
                      const int64_t* n_fibers, int32_t n_subjects, int32_t* const* labels,
                      float* const* dists, const seg_options* opt, void* stream) {
  t_err.clear();
  if (n_atlases < 0 || n_subjects < 0) return fail(SEG_EINVAL, "negative batch size");
  if ((n_atlases > 0 && !atlases) || (n_subjects > 0 && (!fibers || !n_fibers)) ||
      (n_atlases > 0 && n_subjects > 0 && (!labels || !dists)))
    return fail(SEG_EINVAL, "null batch array");
  const seg_options o = resolve(opt);
  int rc = check_mode(o.mode);
  if (!rc) rc = check_metric(o.metric);
  if (rc) return rc;
  for (int32_t a = 0; a < n_atlases; ++a)
    if (!atlases[a]) return fail(SEG_EINVAL, "null atlas in batch");
  for (int32_t i = 0; i < n_subjects; ++i) {
    if (n_fibers[i] < 0) return fail(SEG_EINVAL, "negative subject size");
    if (n_fibers[i] > 0 && !fibers[i]) return fail(SEG_EINVAL, "null subject pointer");
    for (int32_t a = 0; a < n_atlases; ++a)
      if (n_fibers[i] > 0 && (!labels[i * n_atlases + a] || !dists[i * n_atlases + a]))
        return fail(SEG_EINVAL, "null batch output pointer");
  }
  hipStream_t s = (hipStream_t)stream;
  Scratch* sc = nullptr;
  rc = get_scratch(s, &sc);
  if (rc) return rc;
  std::vector<seg::BatchAtlas> bav;
  for (int32_t a = 0; a < n_atlases; ++a)
    bav.push_back(seg::BatchAtlas{atlases[a]->buf.cprep, atlases[a]->buf.ccen,
                                  atlases[a]->buf.bid, atlases[a]->buf.cext,
                                  (int32_t)atlases[a]->buf.m});
  int64_t nmax = 0, mmax = 0;
  for (int32_t i = 0; i < n_subjects; ++i) nmax = n_fibers[i] > nmax ? n_fibers[i] : nmax;
  for (const auto& a : bav) mmax = a.m > mmax ? a.m : mmax;
  const int tile = o.tile ? o.tile : tuned_tile(o.mode, nmax, mmax);
  const bool culled = o.mode >= SEG_PREFILTER_BF16 && o.mode <= SEG_PREFILTER_FP8 &&
                      (tile == 0 || tile == 8) && nmax < ((int64_t)1 << 31);
  if (culled) {
    // the sorted, tile-culled form: every subject's fibers sorted together
    // once, then one culled pass per atlas over all of them
    std::vector<const int32_t*> cperms;
    for (int32_t a = 0; a < n_atlases; ++a) {
      if (bav[a].m > 0 && !atlases[a]->buf.order())
        return fail(SEG_EINVAL, "a batch atlas lacks its centroid order");
      cperms.push_back(atlases[a]->buf.order());
    }
    rc = seg::run_cull_batch(o.mode - SEG_PREFILTER_BF16, bav.data(), n_atlases, cperms.data(),
                             fibers, n_fibers, n_subjects, labels, dists, o.metric, sc->pre,
                             sc->batch, s);
    if (rc == -3) return fail(SEG_ENOMEM, "batch scratch allocation failed");
    if (rc == -4) return fail(SEG_ERANGE, "the tile-culled batch takes fewer than 2^31 fibers");
    if (rc) return hip_fail(hipGetLastError(), "batch launch");
    return SEG_OK;
  }
  // plain, the oriented map and streaming tiles: one launch of the fused kernel
  // over a flattened list of (subject, atlas, fiber block) items, costliest
  // atlas first, in a cached HIP graph
  if (n_atlases == 0 || n_subjects == 0) return SEG_OK;
  if (o.mode == SEG_PLAIN)
    rc = seg::plain_batch(tile, bav.data(), n_atlases, fibers, n_fibers, n_subjects, labels, dists,
                          o.metric, sc->batch, s);
  else if (o.mode >= SEG_PREFILTER_BF16 && o.mode <= SEG_PREFILTER_BF16_ORIENTED)
    rc = seg::prefilter_batch(o.mode, tile, bav.data(), n_atlases, fibers, n_fibers, n_subjects,
                              labels, dists, o.metric, sc->batch, s);
  else
    rc = -2;  // the dense pass has no batched form
  if (rc == -2) return fail(SEG_EMODE, "mode not supported by the batch path");
  if (rc == -3) return fail(SEG_ENOMEM, "batch scratch allocation failed");
  if (rc) return hip_fail(hipGetLastError(), "batch launch");
  return SEG_OK;
}

int seg_autotune(const seg_atlas* a, const float* fibers, int64_t n, int32_t mode, int32_t reps,
                 int32_t* best_tile, float* best_ms, void* stream) {
  t_err.clear();
  if (!a || !fibers || n <= 0) return fail(SEG_EINVAL, "autotune needs an atlas and fibers");
  int rc = check_mode(mode);
  if (rc) return rc;
  if (reps <= 0) reps = 3;
  hipStream_t s = (hipStream_t)stream;
  int32_t* labels = nullptr;
  float* dists = nullptr;
  HIP_TRY(hipMalloc(&labels, (size_t)n * sizeof(int32_t)));
  if (hipMalloc(&dists, (size_t)n * sizeof(float)) != hipSuccess) {
    (void)hipFree(labels);
    return fail(SEG_ENOMEM, "autotune output allocation failed");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int best = 0;
  float best_t = 0.0f;
  for (int tile : mode_tiles(mode)) {
    seg_options o;
    seg_default_options(&o);
    o.mode = mode;
    o.tile = tile;
    rc = seg_segment_atlas(a, fibers, n, labels, dists, &o, stream);
    if (rc) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && !rc; ++r) rc = seg_segment_atlas(a, fibers, n, labels, dists, &o, stream);
    (void)hipEventRecord(e1, s);
    if (rc) break;
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (best == 0 || ms < best_t) {
      best = tile;
      best_t = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(labels);
  (void)hipFree(dists);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple((int)mode, ilog2(n), ilog2(a->buf.m))] = Tuned{best, best_t};
  }
  if (best_tile) *best_tile = best;
  if (best_ms) *best_ms = best_t;
  return SEG_OK;
}

int seg_tune_save(const char* path) {
  if (!path) return fail(SEG_EINVAL, "null path");
  FILE* f = fopen(path, "w");
  if (!f) return fail(SEG_EINVAL, std::string("cannot write ") + path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : g_tuned)
    fprintf(f, "%d %d %d %d %.6f\n", std::get<0>(kv.first), std::get<1>(kv.first),
            std::get<2>(kv.first), kv.second.tile, kv.second.ms);
  fclose(f);
  return SEG_OK;
}

int seg_tune_load(const char* path) {
  if (!path) return fail(SEG_EINVAL, "null path");
  FILE* f = fopen(path, "r");
  if (!f) return fail(SEG_EINVAL, std::string("cannot read ") + path);
  int mode, ln, lm, tile;
  float ms;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  while (fscanf(f, "%d %d %d %d %f", &mode, &ln, &lm, &tile, &ms) == 5)
    g_tuned[std::make_tuple(mode, ln, lm)] = Tuned{tile, ms};
  fclose(f);
  return SEG_OK;
}

void seg_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
}

int seg_filter_pairs(const float* fibers, int64_t n, const float* centroids, int64_t m,
                     const int32_t* bid, const float* thr, int32_t nb, int32_t mode,
                     int32_t* pairs, int64_t capacity, int64_t* count, void* stream) {
  t_err.clear();
  int rc = check_mode(mode);
  if (rc) return rc;
  if (!count) return fail(SEG_EINVAL, "null count");
  *count = 0;
  if (n < 0 || capacity < 0) return fail(SEG_EINVAL, "negative size");
  rc = check_atlas_args(centroids, m, bid, thr, nb);
  if (rc) return rc;
  if (n == 0 || m == 0) return SEG_OK;
  if (!fibers || (capacity > 0 && !pairs)) return fail(SEG_EINVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  Scratch* sc = nullptr;
  rc = get_scratch(s, &sc);
  if (rc) return rc;
  rc = prepare_atlas(sc->atlas, centroids, m, bid, thr, nb, sc->flags, s);
  if (rc) return rc;
  if (seg::launch_fill_u64(sc->counters, 1, 0ull, s)) return hip_fail(hipGetLastError(), "reset");
  if (mode == SEG_PLAIN || mode == SEG_DENSE) {
    rc = seg::launch_plain_pairs(fibers, n, sc->atlas.ccen, (int32_t)m, pairs, capacity,
                                 sc->counters, s);
  } else {
    rc = seg::prefilter_pairs(mode, fibers, n, sc->atlas.cprep, sc->atlas.ccen, (int32_t)m, pairs,
                              capacity, sc->counters, sc->pre, s);
    if (rc == -3) return fail(SEG_ENOMEM, "prefilter scratch allocation failed");
  }
  if (rc == -2) return fail(SEG_EMODE, "mode has no filter");
  if (rc) return hip_fail(hipGetLastError(), "filter launch");
  unsigned long long c = 0;
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(&c, sc->counters, sizeof(c), hipMemcpyDeviceToHost));
  *count = (int64_t)c;
  return SEG_OK;
}

int64_t seg_scratch_bytes(void* stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(std::make_pair(dev, (hipStream_t)stream));
  if (it == g_scratch.end()) return 0;
  const Scratch& sc = *it->second;
  const seg::PrefilterBuf& p = sc.pre;
  const seg::BatchBuf& b = sc.batch;
  int64_t t = (int64_t)sizeof(unsigned long long) * (1 + seg::NCOUNTERS);
  t += sc.atlas.cap * (int64_t)(seg::CREC_BYTES + sizeof(float4) + 2 * sizeof(int32_t) +
                                2 * sizeof(float));
  t += (int64_t)(p.fib_feat_bytes + p.cen_feat_bytes + p.fib_h_bytes + p.tbox_bytes +
                 p.keys_bytes + p.vals_bytes + p.hist_bytes + p.cperm_bytes + p.rank_bytes);
  if (p.emax) t += (int64_t)seg::pf_params_bytes();
  t += (int64_t)(b.items_bytes + b.fib_feat_bytes + b.fib_h_bytes + b.cen_feat_bytes +
                 b.citems_bytes);
  t += (int64_t)(sc.mslots_bytes + sc.mscan_bytes);
  return t;
}

int seg_query_stats(seg_stats* out) {
  if (!out) return fail(SEG_EINVAL, "null output");
  if (!t_stats_counters) return fail(SEG_EINVAL, "no call with collect_stats = 1 on this thread");
  unsigned long long c[seg::NCOUNTERS];
  HIP_TRY(hipStreamSynchronize(t_stats_stream));
  HIP_TRY(hipMemcpy(c, t_stats_counters, sizeof(c), hipMemcpyDeviceToHost));
  out->pairs = t_stats_pairs;
  out->filter_pass = t_stats_mode == SEG_DENSE ? t_stats_pairs : (int64_t)c[0];
  out->test2_pass = (int64_t)c[1];
  out->test3_pass = (int64_t)c[2];
  out->accepted = (int64_t)c[3];
  out->drains = (int64_t)c[4];
  out->bound_pairs = t_stats_culled ? (int64_t)c[5] * 1024 : t_stats_pairs;
  out->survivor_rows = t_stats_culled ? (int64_t)c[6] : -1;
  out->labelled = -1;
  return SEG_OK;
}

}  // extern "C"
