// Degree-ordered copy of a graph for the rating kernels (built once per
// handle, on first use, and kept with it).
//
// Rating gathers one label per edge at a random vertex ID. Most edges of a
// power-law graph end at a few high-degree vertices; numbered by descending
// degree, their labels share cache lines, so far fewer lines are fetched per
// round. The copy renumbers vertices only inside the library: its labels are
// the original cluster IDs, proposals are written at the original vertex and
// acceptance, the cut and contraction run on the original graph, so every
// result equals that of a run on the original numbering.
//
// New vertex i is original vertex orig[i]: vertices in order of descending
// degree, equal degrees by ascending ID. Each neighbourhood is renumbered
// through pos = orig^-1 and sorted by (new ID, weight): equal original
// neighbours keep their weight order, because the sort is stable and the
// original neighbourhoods are sorted by (ID, weight).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "graph.h"
#include "lp.h"
#include "prims.h"
#include "reorder.h"

namespace lp {
namespace {

__global__ void k_ro_keys(int32_t n, const int32_t* deg, int32_t maxd, uint64_t* key, uint32_t* val) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    key[u] = (uint64_t)(uint32_t)(maxd - deg[u]);
    val[u] = (uint32_t)u;
  }
}

__global__ void k_ro_maps(int32_t n, const uint32_t* sorted, const int32_t* deg, const int32_t* vwgt, int32_t* orig,
                          int32_t* pos, uint64_t* ndeg, int32_t* nvwgt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = (int32_t)sorted[i];
    orig[i] = u;
    pos[u] = (int32_t)i;
    ndeg[i] = (uint64_t)(uint32_t)deg[u];
    if (nvwgt) nvwgt[i] = vwgt[u];
  }
}

// One wavefront per new vertex: its neighbours renumbered, keyed by
// (new vertex, new neighbour) at the vertex's new edge range.
__global__ __launch_bounds__(256) void k_ro_edges(int32_t n, const int32_t* orig, const int32_t* pos,
                                                  const uint64_t* xadj, const int32_t* adj, const int32_t* wgt,
                                                  const uint64_t* nxadj, int nbits, uint64_t* key, uint32_t* val) {
  const int lane = threadIdx.x % kWave;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = w0; i < n; i += nw) {
    const int32_t u = orig[i];
    const uint64_t a = xadj[u], d = xadj[u + 1] - a, o = nxadj[i];
    for (uint64_t e = (uint64_t)lane; e < d; e += kWave) {
      key[o + e] = ((uint64_t)i << nbits) | (uint64_t)(uint32_t)pos[adj[a + e]];
      val[o + e] = wgt ? (uint32_t)wgt[a + e] : 0u;
    }
  }
}

__global__ void k_ro_split(uint64_t m, const uint64_t* key, const uint32_t* val, uint64_t mask, int32_t* adj,
                           int32_t* wgt) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (uint64_t)gridDim.x * blockDim.x) {
    adj[j] = (int32_t)(key[j] & mask);
    if (wgt) wgt[j] = (int32_t)val[j];
  }
}

void ro_delete(void* p) {
  Reorder* r = (Reorder*)p;
  if (!r) return;
  (void)hipDeviceSynchronize();
  if (r->g) lp_graph_free(r->g);
  (void)hipFree(r->orig);
  (void)hipFree(r->pos);
  delete r;
}

int bitlen64(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

lp_status build(const lp_graph* g, hipStream_t s, Reorder* R) {
  const int32_t n = g->n;
  const uint64_t m = g->two_m;
  Scratch sc(s);
  int32_t* deg = sc.alloc<int32_t>(n);
  uint64_t* k1 = sc.alloc<uint64_t>(n);
  uint64_t* k2 = sc.alloc<uint64_t>(n);
  uint32_t* v1 = sc.alloc<uint32_t>(n);
  uint32_t* v2 = sc.alloc<uint32_t>(n);
  uint32_t* cnt = sc.alloc<uint32_t>(1);
  uint64_t* nxadj = sc.alloc<uint64_t>((size_t)n + 1);
  int32_t* nvwgt = g->vwgt ? sc.alloc<int32_t>(n) : nullptr;
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMalloc((void**)&R->orig, (size_t)n * sizeof(int32_t)));
  LP_CHECK_HIP(hipMalloc((void**)&R->pos, (size_t)n * sizeof(int32_t)));
  LP_CHECK(compute_degrees(g, deg, s));
  const uint32_t nh = (uint32_t)n;
  LP_CHECK_HIP(hipMemcpyAsync(cnt, &nh, sizeof(uint32_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_ro_keys, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, deg, (int32_t)g->max_deg, k1, v1);
  LP_CHECK_LAUNCH();
  uint64_t* ks;
  uint32_t* vs;
  LP_CHECK(radix_sort_pairs(k1, v1, k2, v2, cnt, n, std::max(1, bitlen64((uint64_t)g->max_deg)), &ks, &vs, sc));
  hipLaunchKernelGGL(k_ro_maps, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, vs, deg, g->vwgt, R->orig, R->pos,
                     nxadj, nvwgt);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u64(nxadj, nxadj, (int64_t)n + 1, nullptr, sc));
  // the original CSR, then every edge keyed by (new vertex, new neighbour)
  uint64_t* xadj = sc.alloc<uint64_t>((size_t)n + 1);
  int32_t* adj = sc.alloc<int32_t>(m);
  int32_t* wgt = g->weighted ? sc.alloc<int32_t>(m) : nullptr;
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK(lp_decompress(g, xadj, adj, wgt, nullptr, s));
  uint64_t* e1 = sc.alloc<uint64_t>(m);
  uint64_t* e2 = sc.alloc<uint64_t>(m);
  uint32_t* w1 = sc.alloc<uint32_t>(m);
  uint32_t* w2 = sc.alloc<uint32_t>(m);
  uint32_t* mcnt = sc.alloc<uint32_t>(1);
  if (sc.failed) return LP_ENOMEM;
  const int nbits = std::max(1, bitlen64((uint64_t)(n - 1)));
  hipLaunchKernelGGL(k_ro_edges, dim3(grid_for((int64_t)n * kWave, 256, 65536)), dim3(256), 0, s, n, R->orig, R->pos,
                     xadj, adj, wgt, nxadj, nbits, e1, w1);
  LP_CHECK_LAUNCH();
  const uint32_t mh = (uint32_t)m;
  LP_CHECK_HIP(hipMemcpyAsync(mcnt, &mh, sizeof(uint32_t), hipMemcpyHostToDevice, s));
  LP_CHECK(radix_sort_pairs(e1, w1, e2, w2, mcnt, (int64_t)m, 2 * nbits, &ks, &vs, sc));
  hipLaunchKernelGGL(k_ro_split, dim3(grid_for((int64_t)m, 256, 1 << 20)), dim3(256), 0, s, m, ks, vs,
                     (1ull << nbits) - 1ull, adj, wgt);
  LP_CHECK_LAUNCH();
  if (g->compressed)
    LP_CHECK(lp_compress_ex(n, nxadj, adj, wgt, nvwgt, g->intervals ? LP_COMPRESS_INTERVALS : 0, s, &R->g));
  else
    LP_CHECK(lp_graph_from_csr(n, nxadj, adj, wgt, nvwgt, s, &R->g));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  return LP_OK;
}

}  // namespace

bool reorder_applies(const lp_graph* g) {
  return g->nbatch == 0 && g->n >= 2 && g->two_m <= 0xFFFFFFFFull && 2 * bitlen64((uint64_t)(g->n - 1)) <= 64;
}

lp_status get_reorder(const lp_graph* g, hipStream_t s, const Reorder** out) {
  std::lock_guard<std::mutex> lock(g->reord_mu);
  if (!g->reord) {
    Reorder* R = new Reorder();
    const lp_status st = build(g, s, R);
    if (st != LP_OK) {
      ro_delete(R);
      return st;
    }
    g->reord = R;
    g->reord_free = ro_delete;
    // the one-time buffers of the build are large; the cache keeps none of them
    cache_trim_all();
  }
  *out = (const Reorder*)g->reord;
  return LP_OK;
}

const Reorder* existing_reorder(const lp_graph* g) {
  std::lock_guard<std::mutex> lock(g->reord_mu);
  return (const Reorder*)g->reord;
}

}  // namespace lp
