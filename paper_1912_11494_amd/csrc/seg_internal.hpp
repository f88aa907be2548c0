// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "seg_device.hpp"

namespace seg {

constexpr unsigned int FLAG_BUNDLE = 1u;
constexpr unsigned int FLAG_NONFINITE = 2u;
constexpr unsigned int FLAG_OFFSETS = 4u;

// Number of 64-bit statistics counters (see StageCounts).
constexpr int NCOUNTERS = 8;
constexpr size_t CREC_BYTES = 64 * sizeof(float);

// Library-owned prefilter scratch (per device and stream), grown on demand.
struct PrefilterBuf {
  void* fib_feat = nullptr;   // quantised fiber features
  size_t fib_feat_bytes = 0;
  void* cen_feat = nullptr;   // quantised centroid features + biases
  size_t cen_feat_bytes = 0;
  float* fib_h = nullptr;     // per-fiber bound terms
  size_t fib_h_bytes = 0;
  unsigned int* emax = nullptr;  // device max of the fiber quantisation error
  // sorted, tile-culled form (seg_cull.hip)
  void* tbox = nullptr;   // feature boxes and radii of centroid tiles
  size_t tbox_bytes = 0;
  void* keys = nullptr;   // sort keys, two buffers
  size_t keys_bytes = 0;
  void* vals = nullptr;   // sort values, two buffers (the fiber permutation)
  size_t vals_bytes = 0;
  void* hist = nullptr;   // digit counts per block + digit offsets
  size_t hist_bytes = 0;
  void* cperm = nullptr;  // sorted column -> centroid
  size_t cperm_bytes = 0;
  void* rank = nullptr;   // partial rank counts of the centroid order
  size_t rank_bytes = 0;
};

struct PfParams;

// Library-owned batch scratch: the device job list and the last captured HIP
// graph with the launch shape it was captured for.
struct BatchBuf {
  void* items = nullptr;  // job descriptors + prefix sums of work items
  size_t items_bytes = 0;
  void* fib_feat = nullptr;  // quantised features of every subject of the batch
  size_t fib_feat_bytes = 0;
  float* fib_h = nullptr;
  size_t fib_h_bytes = 0;
  void* cen_feat = nullptr;  // column features + constants of every atlas
  size_t cen_feat_bytes = 0;
  hipStream_t cap = nullptr;  // private stream for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> key;  // launch shape of `exec`
  int32_t njobs = 0;          // jobs in the uploaded list
  // the tile-culled batch: subject table and output pointers on the device
  void* citems = nullptr;
  size_t citems_bytes = 0;
  std::vector<uint64_t> ckey;    // what `citems` holds
  void* citems_tab = nullptr;    // the buffer `ckey` was uploaded to
};

// A prepared atlas as the batch path sees it.
struct BatchAtlas {
  const float* cprep;
  const float4* ccen;
  const int32_t* bid;
  const float* cext;  // per centroid: arc length, threshold (metric variants)
  int32_t m;
};

int launch_prep_atlas(const float* cen, int64_t m, const int32_t* bid, const float* thr,
                      int32_t nb, float* cprep, float4* ccen, int32_t* bid_out, float* cext,
                      unsigned int* flags, hipStream_t s);
int launch_check_finite(const float* v, int64_t count, unsigned int* flags, hipStream_t s);
// seg_multi.hip: slot rows -> sorted rows, CSR offsets, entries and bundle
// counts (see seg_segment_multi); flags is the device word of multi_insert
int multi_collect(unsigned long long* slots, int32_t K, int64_t n, int64_t* offsets,
                  int32_t* bundles, float* dists, int64_t capacity, int64_t* bundle_counts,
                  int32_t nb, int mflags, void** scan_buf, size_t* scan_bytes, hipStream_t s);
int launch_fill_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
// seg_resample.hip: raw streamlines (CSR) to [n][21][3]; flags may be null
int launch_resample(const float* pts, int64_t npts, const int64_t* off, int64_t n, float* out,
                    unsigned int* flags, hipStream_t s);
int launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t s);
int launch_fill_empty(int64_t n, int32_t* labels, float* dists, hipStream_t s);
int launch_dense(const float* fibers, int64_t n, const float* cprep, int32_t m,
                 const int32_t* bid, int32_t* labels, float* dists, int cfg, Metric mt,
                 hipStream_t s);
int plain_default_cfg(int64_t n);
int launch_plain(const float* fibers, int64_t n, const float4* ccen, const float* cprep,
                 int32_t m, const int32_t* bid, int32_t* labels, float* dists,
                 unsigned long long* counters, int cfg, Metric mt, hipStream_t s);
int launch_plain_pairs(const float* fibers, int64_t n, const float4* ccen, int32_t m,
                       int32_t* pairs, int64_t cap, unsigned long long* count, hipStream_t s);

// Prefilter modes (seg_prefilter.hip).  Return 0, -1 on a HIP error, -2 on an
// unsupported mode or tile, -3 on a failed allocation.
// `cperm`, when not null, is the atlas's sorted column order computed once by
// cull_sort_centroids, followed by its frame (the tile-culled form then skips
// that sort and the box reduction).
int run_prefilter(int mode, int cfg, const float* fibers, int64_t n, const float* cprep,
                  const float4* ccen, int32_t m, const int32_t* bid, int32_t* labels,
                  float* dists, unsigned long long* counters, Metric mt, PrefilterBuf& pb,
                  hipEvent_t* ev, hipStream_t s, const int32_t* cperm = nullptr);
// Frame set-up shared by the prefilter forms: reset the parameters and take
// the bounding box of the atlas points (seg_prefilter.hip).
int launch_pf_setup(PfParams* prm, const float* cprep, int32_t m, hipStream_t s);
// The same in parts: reset, then widen the box by the points of one atlas
// (several atlases share a frame this way).
int launch_pf_init(PfParams* prm, hipStream_t s);
size_t pf_params_bytes();
int launch_pf_bbox_acc(PfParams* prm, const float* cprep, int32_t m, hipStream_t s);

// Sorted, tile-culled prefilter (seg_cull.hip); q: 0 bf16, 1 fp16, 2 fp8.
// Returns as run_prefilter, and -4 for 2^31 fibers or more.
int run_cull(int q, const float* fibers, int64_t n, const float* cprep, int32_t m,
             const int32_t* bid, int32_t* labels, float* dists, unsigned long long* counters,
             Metric mt, PrefilterBuf& pb, hipEvent_t* ev, hipStream_t s, const MultiOut* mo = nullptr,
             const int32_t* cperm = nullptr);
// The tile-culled form for a batch: every subject's fibers sorted together,
// then one culled pass per atlas (seg_cull.hip).  cperms[a] is atlas a's
// centroid order (cull_sort_centroids).  Returns as run_cull.
int run_cull_batch(int q, const BatchAtlas* atlases, int32_t n_atlases,
                   const int32_t* const* cperms, const float* const* fibers,
                   const int64_t* n_fibers, int32_t n_subjects, int32_t* const* labels,
                   float* const* dists, int mflags, PrefilterBuf& pb, BatchBuf& bb,
                   hipStream_t s);
// The tile-culled form's centroid order for a prepared atlas: centroids
// sorted by the cell of their center point in the atlas's frame (the same for
// every subject and quantisation), written to cperm_out [m], and the frame
// itself (six words) after it, at cperm_out [m, m + 6): cperm_out holds
// m + 6 entries.  run_cull reads the frame there when given the order.
int cull_sort_centroids(const float* cprep, int32_t m, int32_t* cperm_out, PrefilterBuf& pb,
                        hipStream_t s);

int prefilter_pairs(int mode, const float* fibers, int64_t n, const float* cprep,
                    const float4* ccen, int32_t m, int32_t* pairs, int64_t cap,
                    unsigned long long* count, PrefilterBuf& pb, hipStream_t s);

// Per-mode batch launches (seg_prefilter.hip / seg_kernels.hip): size the
// buffers, upload the job list (synchronising `s` when the launch shape
// changes) and run the whole batch as one cached HIP graph (seg_graph.hpp).
int prefilter_batch(int mode, int cfg, const BatchAtlas* atlases, int32_t n_atlases,
                    const float* const* fibers, const int64_t* n_fibers, int32_t n_subjects,
                    int32_t* const* labels, float* const* dists, int mflags, BatchBuf& bb,
                    hipStream_t s);
int plain_batch(int cfg, const BatchAtlas* atlases, int32_t n_atlases, const float* const* fibers,
                const int64_t* n_fibers, int32_t n_subjects, int32_t* const* labels,
                float* const* dists, int mflags, BatchBuf& bb, hipStream_t s);

}  // namespace seg
