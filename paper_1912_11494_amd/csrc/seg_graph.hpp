// Capture-once / replay-many launch of a batch through a HIP graph.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "seg_internal.hpp"

namespace seg {

// Replays the cached graph when `key` matches the shape it was captured for;
// otherwise captures `enqueue(stream)` on the private stream, instantiates it
// and launches it on `s`.  Nothing inside the graph is a memset node (device
// counters are cleared by a kernel).
template <class F>
int graph_launch(BatchBuf& bb, const std::vector<uint64_t>& key, hipStream_t s, F&& enqueue) {
  if (bb.exec && bb.key == key) return hipGraphLaunch(bb.exec, s) == hipSuccess ? 0 : -1;
  if (bb.exec) {
    (void)hipGraphExecDestroy(bb.exec);
    bb.exec = nullptr;
  }
  if (bb.graph) {
    (void)hipGraphDestroy(bb.graph);
    bb.graph = nullptr;
  }
  if (!bb.cap && hipStreamCreateWithFlags(&bb.cap, hipStreamNonBlocking) != hipSuccess) return -1;
  if (hipStreamBeginCapture(bb.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return -1;
  int rc = enqueue(bb.cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(bb.cap, &g);
  if (rc || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : -1;
  }
  if (hipGraphInstantiate(&bb.exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    bb.exec = nullptr;
    return -1;
  }
  bb.graph = g;
  bb.key = key;
  return hipGraphLaunch(bb.exec, s) == hipSuccess ? 0 : -1;
}

}  // namespace seg
