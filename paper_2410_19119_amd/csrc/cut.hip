// Edge cut of a clustering (Section I: the partitioning objective): the total
// weight of the edges whose endpoints carry different labels. Every edge is
// visited by the same lane / tile / piece decoders as the rating kernels
// (with the graph's cached plan), each counting the weights of its edges that
// leave their vertex's cluster; the sum counts every cut edge twice.
#include "graph.h"

#include <mutex>

namespace lp {
lp_status visit_edges_cut(const lp_graph* g, const int32_t* labels, unsigned long long* cut, hipStream_t s);
lp_status visit_edges_cut_noalloc(const lp_graph* g, const int32_t* labels, unsigned long long* cut,
                                  uint32_t* counters, hipStream_t s);
}

using namespace lp;

// Scratch of lp_edge_cut_noalloc, one copy per device for the life of the
// process: word 0 accumulates the weights of the cut edges, words 16..31 hold
// the 32 uint32 counters of the edge visit (a flag and the hand-out counters
// of the tile and piece kernels). Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress.
constexpr int kCutScratchWords = 32;
static __device__ __align__(256) unsigned long long scratch[kCutScratchWords];

namespace {

__global__ void k_cut_scratch_clear(unsigned long long* ws) {
  for (int i = threadIdx.x; i < kCutScratchWords; i += blockDim.x) ws[i] = 0;
}

__global__ void k_cut_finish(const unsigned long long* ws, int64_t* cut_out) { *cut_out = (int64_t)(ws[0] / 2); }

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
lp_status cut_scratch(unsigned long long** out) {
  int dev = -1;
  LP_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return LP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    LP_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return LP_EDEVICE;
    g_scratch_ptr[dev] = (unsigned long long*)p;
  }
  *out = g_scratch_ptr[dev];
  return LP_OK;
}

}  // namespace

extern "C" lp_status lp_edge_cut(const lp_graph* g, const int32_t* labels, int64_t* cut_out, void* stream) {
  clear_error();
  if (!g || !cut_out || (!labels && g->n > 0)) return LP_EINVAL;
  *cut_out = 0;
  if (g->n == 0) return LP_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  unsigned long long* acc = sc.alloc<unsigned long long>(1);
  if (!acc) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long), s));
  LP_CHECK(visit_edges_cut(g, labels, acc, s));
  unsigned long long h = 0;
  LP_CHECK_HIP(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  *cut_out = (int64_t)(h / 2);
  return LP_OK;
}

extern "C" lp_status lp_edge_cut_noalloc(const lp_graph* g, const int32_t* labels, int64_t* cut_dev, void* stream) {
  clear_error();
  if (!g || !cut_dev || (!labels && g->n > 0)) return LP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* ws = nullptr;
  LP_CHECK(cut_scratch(&ws));
  hipLaunchKernelGGL(k_cut_scratch_clear, dim3(1), dim3(64), 0, s, ws);
  LP_CHECK_LAUNCH();
  LP_CHECK(visit_edges_cut_noalloc(g, labels, ws, (uint32_t*)(ws + 16), s));
  hipLaunchKernelGGL(k_cut_finish, dim3(1), dim3(1), 0, s, ws, cut_dev);
  return last_error();
}
