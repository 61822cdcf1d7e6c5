// Batches of graphs: the disjoint union of G resident graphs as one handle,
// so that one launch of every rating, acceptance and apply kernel serves all
// of them. Vertex IDs of graph g are shifted by its first vertex vbase[g];
// the compressed records are copied unchanged (each record is coded relative
// to its own vertex, so a shift of all IDs leaves the bytes valid), with byte
// offsets rebased. The first-edge headers restart in every graph, so the
// union keeps explicit degrees. Each graph keeps its own cap and seed, and
// its tie-break keys use labels local to the graph (Section IV-A rules apply
// per graph), which makes every graph's labels exactly those of a run alone.
#include <string.h>

#include <algorithm>
#include <vector>

#include "graph.h"

namespace lp {
namespace {

struct BatchSrc {
  const uint64_t* const* offs;    // per graph (compressed)
  const uint8_t* const* bytes;    // per graph (compressed)
  const uint64_t* const* xadj;    // per graph (plain)
  const int32_t* const* vwgt;     // per graph or null
  const int32_t* vbase;           // G + 1
  const uint64_t* bbase;          // G + 1: byte (compressed) or edge (plain) base
  const uint64_t* two_m;          // G: directed edges of each graph
  int32_t G;
};

__device__ __forceinline__ int32_t graph_of(const int32_t* vbase, int32_t G, int32_t u) {
  int32_t lo = 0, hi = G;  // vbase[lo] <= u < vbase[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (vbase[mid] <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t header_at(const uint8_t* b, uint64_t pos) {
  uint64_t x = 0;
  int shift = 0;
  while (true) {
    const uint32_t c = b[pos++];
    x |= (uint64_t)(c & 0x7F) << shift;
    if (!(c & 0x80)) return x;
    shift += 7;
  }
}

// Per union vertex: rebased offset, degree, graph, weight.
__global__ void k_batch_vertices(BatchSrc src, int32_t n, bool comp, uint64_t* offs, uint64_t* xadj, int32_t* deg,
                                 int32_t* gid, int32_t* vwgt) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = graph_of(src.vbase, src.G, (int32_t)u);
    const int32_t lu = (int32_t)u - src.vbase[g];
    const int32_t ng = src.vbase[g + 1] - src.vbase[g];
    if (comp) {
      const uint64_t* o = src.offs[g];
      offs[u] = src.bbase[g] + o[lu];
      const uint64_t a = header_at(src.bytes[g], o[lu]);
      const uint64_t b = lu + 1 < ng ? header_at(src.bytes[g], o[lu + 1]) : src.two_m[g];
      deg[u] = (int32_t)(b - a);
    } else {
      const uint64_t* x = src.xadj[g];
      xadj[u] = src.bbase[g] + x[lu];
      deg[u] = (int32_t)(x[lu + 1] - x[lu]);
    }
    gid[u] = g;
    if (vwgt) vwgt[u] = src.vwgt[g] ? src.vwgt[g][lu] : 1;
  }
}

// Plain unions: neighbour IDs shifted by their graph's first vertex.
__global__ void k_batch_shift(const int32_t* const* adj, const uint64_t* ebase, const int32_t* vbase, int32_t G,
                              uint64_t m, int32_t* out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; (uint64_t)e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = G;  // ebase[lo] <= e < ebase[hi]
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (ebase[mid] <= (uint64_t)e) lo = mid;
      else hi = mid;
    }
    out[e] = adj[lo][(uint64_t)e - ebase[lo]] + vbase[lo];
  }
}

__global__ void k_set_u64(uint64_t* p, uint64_t v) { *p = v; }

// Labels of a batch run: global cluster IDs -> IDs local to each graph,
// written to one array (out) or to the graph's own array (outs[g]).
__global__ void k_batch_localize(const int32_t* lab, const int32_t* gid, const int32_t* gbase, int32_t n,
                                 int32_t* out, int32_t* const* outs) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = gid[u];
    const int32_t v = lab[u] - gbase[g];
    if (out) out[u] = v;
    else outs[g][u - gbase[g]] = v;
  }
}

}  // namespace

lp_status batch_localize(const lp_graph* b, const int32_t* lab, int32_t* out, int32_t* const* outs_dev,
                         hipStream_t s) {
  if (b->n == 0) return LP_OK;
  hipLaunchKernelGGL(k_batch_localize, dim3(grid_for(b->n, 256, 65536)), dim3(256), 0, s, lab, b->gid, b->gbase, b->n,
                     out, outs_dev);
  return last_error();
}

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_batch_create(int32_t G, const lp_graph* const* gs, void* stream, lp_graph** out) {
  clear_error();
  if (!out || G < 1 || !gs) return LP_EINVAL;
  *out = nullptr;
  for (int32_t i = 0; i < G; ++i)
    if (!gs[i] || gs[i]->nbatch) return LP_EINVAL;
  const bool comp = gs[0]->compressed, weighted = gs[0]->weighted, itv = gs[0]->intervals;
  for (int32_t i = 0; i < G; ++i)
    if ((bool)gs[i]->compressed != comp || (bool)gs[i]->weighted != weighted || (bool)gs[i]->intervals != itv)
      return LP_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> vbase(G + 1);
  std::vector<uint64_t> bbase(G + 1), two_m(G);
  int64_t n = 0;
  uint64_t m = 0, nb = 0;
  bool any_vwgt = false;
  int64_t max_wdeg = 0, max_deg = 0, total = 0;
  for (int32_t i = 0; i < G; ++i) {
    const lp_graph* g = gs[i];
    vbase[i] = (int32_t)n;
    bbase[i] = comp ? nb : m;
    two_m[i] = g->two_m;
    n += g->n;
    m += g->two_m;
    nb += g->nbytes;
    any_vwgt |= g->vwgt != nullptr;
    max_wdeg = std::max(max_wdeg, g->max_wdeg);
    max_deg = std::max(max_deg, g->max_deg);
    total += g->total_vwgt;
    if (n > 0x7FFFFFFF) return LP_EUNSUPPORTED;
  }
  vbase[G] = (int32_t)n;
  bbase[G] = comp ? nb : m;

  lp_graph* b = new lp_graph();
  (void)hipGetDevice(&b->device);
  b->n = (int32_t)n;
  b->two_m = m;
  b->compressed = comp;
  b->weighted = weighted;
  b->intervals = itv;
  b->total_vwgt = total;
  b->max_wdeg = max_wdeg;
  b->max_deg = max_deg;
  b->nbytes = comp ? nb : 0;
  b->nbatch = G;
  b->vbase = vbase;
  b->stream_mem = true;
  b->mem_stream = s;
  lp_status st = LP_OK;
  Scratch sc(s);
  std::vector<const void*> all;  // per-graph pointer tables (live until the final synchronisation)
  do {
    auto dmalloc = [&](void** p, size_t bytes) {
      if (st == LP_OK && graph_alloc(b, p, bytes) != hipSuccess) st = LP_ENOMEM;
    };
    dmalloc((void**)&b->gid, (size_t)n * sizeof(int32_t));
    dmalloc((void**)&b->deg, (size_t)n * sizeof(int32_t));
    dmalloc((void**)&b->gbase, (size_t)(G + 1) * sizeof(int32_t));
    if (any_vwgt) dmalloc((void**)&b->vwgt, (size_t)n * sizeof(int32_t));
    if (comp) {
      dmalloc((void**)&b->offs, (size_t)(n + 1) * sizeof(uint64_t));
      dmalloc((void**)&b->bytes, nb + kBytePad);
    } else {
      dmalloc((void**)&b->xadj, (size_t)(n + 1) * sizeof(uint64_t));
      dmalloc((void**)&b->adjncy, (size_t)m * sizeof(int32_t));
      if (weighted) dmalloc((void**)&b->adjwgt, (size_t)m * sizeof(int32_t));
    }
    if (st) break;
    // per-graph pointer tables
    std::vector<const void*> p_offs(G), p_bytes(G), p_xadj(G), p_vwgt(G), p_adj(G);
    for (int32_t i = 0; i < G; ++i) {
      p_offs[i] = gs[i]->offs;
      p_bytes[i] = gs[i]->bytes;
      p_xadj[i] = gs[i]->xadj;
      p_vwgt[i] = gs[i]->vwgt;
      p_adj[i] = gs[i]->adjncy;
    }
    const void** d_ptr = sc.alloc<const void*>((size_t)5 * G);
    int32_t* d_vbase = b->gbase;
    uint64_t* d_bbase = sc.alloc<uint64_t>((size_t)G + 1);
    uint64_t* d_two_m = sc.alloc<uint64_t>((size_t)G);
    if (sc.failed) {
      st = LP_ENOMEM;
      break;
    }
    for (auto* v : {&p_offs, &p_bytes, &p_xadj, &p_vwgt, &p_adj}) all.insert(all.end(), v->begin(), v->end());
    if (hipMemcpyAsync(d_ptr, all.data(), all.size() * sizeof(void*), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_vbase, vbase.data(), (G + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_bbase, bbase.data(), (G + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_two_m, two_m.data(), G * sizeof(uint64_t), hipMemcpyHostToDevice, s) != hipSuccess) {
      st = LP_EDEVICE;
      break;
    }
    BatchSrc src{(const uint64_t* const*)d_ptr, (const uint8_t* const*)(d_ptr + G),
                 (const uint64_t* const*)(d_ptr + 2 * G), (const int32_t* const*)(d_ptr + 3 * G), d_vbase, d_bbase,
                 d_two_m, G};
    if (n > 0) {
      hipLaunchKernelGGL(k_batch_vertices, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, src, (int32_t)n, comp,
                         b->offs, b->xadj, b->deg, b->gid, b->vwgt);
      if ((st = last_error())) break;
    }
    if (comp) {
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, b->offs + n, nb);
      if ((st = last_error())) break;
      for (int32_t i = 0; i < G && !st; ++i)
        if (gs[i]->nbytes &&
            hipMemcpyAsync(b->bytes + bbase[i], gs[i]->bytes, gs[i]->nbytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
          st = LP_EDEVICE;
      if (!st && hipMemsetAsync(b->bytes + nb, 0, kBytePad, s) != hipSuccess) st = LP_EDEVICE;
    } else {
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, b->xadj + n, m);
      if ((st = last_error())) break;
      if (m > 0) {
        hipLaunchKernelGGL(k_batch_shift, dim3(grid_for((int64_t)m, 256, 65536)), dim3(256), 0, s,
                           (const int32_t* const*)(d_ptr + 4 * G), d_bbase, d_vbase, G, m, b->adjncy);
        if ((st = last_error())) break;
      }
      for (int32_t i = 0; i < G && weighted && !st; ++i)
        if (gs[i]->two_m && hipMemcpyAsync(b->adjwgt + bbase[i], gs[i]->adjwgt, gs[i]->two_m * sizeof(int32_t),
                                           hipMemcpyDeviceToDevice, s) != hipSuccess)
          st = LP_EDEVICE;
    }
  } while (0);
  if (st == LP_OK && hipStreamSynchronize(s) != hipSuccess) st = LP_EDEVICE;
  if (st != LP_OK) {
    lp_graph_free(b);
    return st;
  }
  *out = b;
  return LP_OK;
}

extern "C" lp_status lp_batch_info(const lp_graph* b, int32_t* G, int32_t* vbase) {
  clear_error();
  if (!b) return LP_EINVAL;
  if (G) *G = b->nbatch;
  if (vbase && b->nbatch) memcpy(vbase, b->vbase.data(), (b->vbase.size()) * sizeof(int32_t));
  return LP_OK;
}
