// hipGraph capture of the solvers' check blocks (k sweeps + residual + readback).
//
// A block is recorded once on a context-owned stream (the caller's stream may be the
// legacy null stream, which cannot be captured) and replayed with one hipGraphLaunch on
// the caller's stream. Blocks only contain kernels and a device-to-host copy into pinned
// memory; buffers are cleared by fill kernels, never by memset nodes.
#pragma once

#include <utility>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

struct GraphKey {
  int kind;
  const void* a;
  const void* b;
  const void* c;
  int parity;
  int k;
  int T;
  double tol;
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && a == o.a && b == o.b && c == o.c && parity == o.parity &&
           k == o.k && T == o.T && tol == o.tol;
  }
};

struct GraphCache {
  std::vector<std::pair<GraphKey, hipGraphExec_t>> entries;
  hipStream_t capture_stream = nullptr;

  hipGraphExec_t find(const GraphKey& key) const {
    for (const auto& e : entries)
      if (e.first == key) return e.second;
    return nullptr;
  }
  void put(const GraphKey& key, hipGraphExec_t g) {
    if (entries.size() >= 16) {
      (void)hipGraphExecDestroy(entries.front().second);
      entries.erase(entries.begin());
    }
    entries.emplace_back(key, g);
  }
  void clear() {
    for (auto& e : entries) (void)hipGraphExecDestroy(e.second);
    entries.clear();
  }
  ~GraphCache() {
    clear();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
};

// Run `enqueue(stream)` as a captured graph on `s` (recording it on first use), or directly
// on `s` when graphs are off. `enqueue` must only enqueue asynchronous work.
template <class F>
int run_block(gabp_ctx* c, GraphCache& cache, hipStream_t s, const GraphKey& key, F&& enqueue) {
  if (!c->opt.use_graphs) return enqueue(s);
  hipGraphExec_t exec = cache.find(key);
  if (!exec) {
    if (!cache.capture_stream)
      GABP_HIP(hipStreamCreateWithFlags(&cache.capture_stream, hipStreamNonBlocking));
    GABP_HIP(hipStreamBeginCapture(cache.capture_stream, hipStreamCaptureModeThreadLocal));
    const int st = enqueue(cache.capture_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cache.capture_stream, &graph);
    if (st != GABP_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate");
    cache.put(key, exec);
  }
  GABP_HIP(hipGraphLaunch(exec, s));
  return GABP_OK;
}

}  // namespace gabp
