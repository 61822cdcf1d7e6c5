// The lp_graph handle: device-resident graph (compressed or plain CSR) plus
// the host-side sizes every launcher needs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "lp_device.h"
#include "prims.h"

struct lp_graph {
  int32_t n = 0;
  uint64_t two_m = 0;
  int32_t compressed = 0;
  int32_t weighted = 0;     // edge weights stored
  int32_t intervals = 0;    // compressed with interval encoding
  int64_t total_vwgt = 0;   // sum of vertex weights
  int64_t max_wdeg = 0;     // max over u of the summed weight of u's edges
  int64_t max_deg = 0;
  uint64_t nbytes = 0;      // compressed adjacency bytes (without padding)
  int device = 0;
  // compressed form
  uint64_t* offs = nullptr;   // n + 1 byte offsets
  uint8_t* bytes = nullptr;   // nbytes + kBytePad
  // plain form
  uint64_t* xadj = nullptr;   // n + 1
  int32_t* adjncy = nullptr;  // two_m
  int32_t* adjwgt = nullptr;  // two_m or null
  int32_t* vwgt = nullptr;    // n or null (unit)
  // disjoint union of several graphs (lp_batch_create); nbatch == 0 otherwise
  int32_t nbatch = 0;
  int32_t* gid = nullptr;     // n: graph of each vertex
  int32_t* gbase = nullptr;   // nbatch + 1: first vertex of each graph
  int32_t* deg = nullptr;     // n: degrees (first-edge headers restart per graph)
  std::vector<int32_t> vbase; // host copy of gbase
  // handles made inside a call (coarse graphs, batches) take their buffers from
  // the library's memory cache on that call's stream and release them in its order
  bool stream_mem = false;
  hipStream_t mem_stream = nullptr;
  // degree buckets, tiles and hub pieces for the default thresholds, built on
  // first use (a derived, result-free cache; the graph itself never changes)
  mutable void* plan = nullptr;
  void (*plan_free)(void*) = nullptr;
  mutable std::mutex plan_mu;
  // degree-ordered copy for the rating kernels (reorder.h), built on first use
  mutable std::atomic<int32_t> cluster_calls{0};  // lp_cluster(_ex) calls on this handle
  mutable void* reord = nullptr;
  mutable void (*reord_free)(void*) = nullptr;
  mutable std::mutex reord_mu;

  lp::GraphView view() const {
    lp::GraphView v;
    v.n = n;
    v.weighted = weighted;
    v.intervals = intervals;
    v.two_m = two_m;
    v.offs = offs;
    v.bytes = bytes;
    v.xadj = xadj;
    v.adjncy = adjncy;
    v.adjwgt = adjwgt;
    v.vwgt = vwgt;
    return v;
  }
};

namespace lp {

// Device buffer of a handle (see stream_mem).
inline hipError_t graph_alloc(const lp_graph* g, void** p, size_t bytes) {
  if (!bytes) bytes = 1;
  if (!g->stream_mem) return hipMalloc(p, bytes);
  *p = cache_alloc(bytes, g->mem_stream);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

// Readable padding after the compressed bytes, so that cooperative window
// loads may run past the last record.
constexpr size_t kBytePad = 8192;

// Degrees deg[u] (int32) of any handle; fe[u] optional first-edge IDs.
lp_status compute_degrees(const lp_graph* g, int32_t* deg, hipStream_t s);

// Max of deg over u (for launch sizing); host result.
lp_status reduce_max_i32(const int32_t* a, int64_t n, int32_t* out_host, Scratch& sc);

}  // namespace lp
