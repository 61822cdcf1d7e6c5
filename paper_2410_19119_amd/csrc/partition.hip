// Uncoarsening slice of the multilevel scheme (Section II-A of the paper):
// the initial partition of the coarsest graph and the projection of blocks
// from a quotient graph to the graph it was contracted from. Refinement is
// lp_refine (the LP rounds of cluster.hip started from the blocks).
#include "graph.h"

namespace lp {
namespace {

// Contiguous-weight initial partition with unit weights: P_u = u, c(V) = n.
__global__ void k_ip_unit(int32_t n, int32_t k, int32_t* labels) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    labels[u] = (int32_t)((uint64_t)k * (uint64_t)u / (uint64_t)n);
}

__global__ void k_widen(const int32_t* vwgt, int32_t n, uint64_t* out) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    out[u] = (uint64_t)vwgt[u];
}

// Weighted: P_u from an exclusive scan; k * P_u < k * c(V) < 2^63 (checked
// on the host), so the quotient is exact in 64 bits.
__global__ void k_ip_weighted(const uint64_t* prefix, int32_t n, int32_t k, uint64_t total, int32_t* labels) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    labels[u] = (int32_t)((uint64_t)k * prefix[u] / total);
}

__global__ void k_project(int32_t n, const int32_t* map, int32_t coarse_n, const int32_t* coarse, int32_t* out) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = map[u];
    out[u] = (uint32_t)a < (uint32_t)coarse_n ? coarse[a] : -1;
  }
}

}  // namespace
}  // namespace lp

using namespace lp;

extern "C" lp_status lp_initial_partition(const lp_graph* g, int32_t k, int32_t* labels, void* stream) {
  clear_error();
  if (!g || g->nbatch || k < 1 || (!labels && g->n > 0)) return LP_EINVAL;
  const int32_t n = g->n;
  if (n == 0) return LP_OK;
  const uint64_t total = (uint64_t)g->total_vwgt;
  if (total == 0 || total > (uint64_t)INT64_MAX / (uint64_t)k) return LP_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = grid_for(n, 256, 65536);
  if (!g->vwgt) {
    hipLaunchKernelGGL(k_ip_unit, dim3(grid), dim3(256), 0, s, n, k, labels);
    return last_error();
  }
  Scratch sc(s);
  uint64_t* pre = sc.alloc<uint64_t>(n);
  if (!pre) return LP_ENOMEM;
  hipLaunchKernelGGL(k_widen, dim3(grid), dim3(256), 0, s, g->vwgt, n, pre);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u64(pre, pre, n, nullptr, sc));
  hipLaunchKernelGGL(k_ip_weighted, dim3(grid), dim3(256), 0, s, pre, n, k, total, labels);
  return last_error();
}

extern "C" lp_status lp_project(int32_t n, const int32_t* map, int32_t coarse_n, const int32_t* coarse_labels,
                                int32_t* labels, void* stream) {
  clear_error();
  if (n < 0 || coarse_n < 0 || (n > 0 && (!map || !labels || (coarse_n > 0 && !coarse_labels)))) return LP_EINVAL;
  if (n == 0) return LP_OK;
  hipLaunchKernelGGL(k_project, dim3(grid_for(n, 256, 65536)), dim3(256), 0, (hipStream_t)stream, n, map, coarse_n,
                     coarse_labels, labels);
  return last_error();
}
