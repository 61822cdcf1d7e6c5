// Cluster contraction (Section IV-B) and the edge cut (Section I).
//
// Contraction: nonempty labels are ranked (coarse IDs in increasing label
// order), members are grouped per coarse vertex, and each coarse
// neighbourhood is aggregated in an LDS table, sorted in LDS and written to a
// staging area; a prefix sum over the coarse degrees places the
// neighbourhoods in the final CSR. Following the paper's two-phase
// aggregation (Section IV-B1), light clusters (small total member degree)
// are aggregated by one wavefront or one workgroup each; heavy clusters by a
// workgroup that sweeps the coarse-ID range in LDS-sized windows.
#include <algorithm>

#include "decode.h"
#include "graph.h"

namespace lp {

namespace {

constexpr uint32_t kErrLabel = 1, kErrOverflow = 2, kErrFormat = 4;

__global__ void k_check_mark(const int32_t* C, int32_t n, uint32_t* flags, uint32_t* err) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = C[u];
    if (c < 0 || c >= n) atomicOr(err, kErrLabel);
    else flags[c] = 1;
  }
}

__global__ void k_map(const int32_t* C, int32_t n, const uint32_t* id, const int32_t* deg, const int32_t* vwgt,
                      int32_t* map, uint32_t* cnt, unsigned long long* vw, unsigned long long* dsum) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = (int32_t)id[C[u]];
    map[u] = a;
    atomicAdd(&cnt[a], 1u);
    atomicAdd(&vw[a], (unsigned long long)(vwgt ? vwgt[u] : 1));
    if (deg[u]) atomicAdd(&dsum[a], (unsigned long long)deg[u]);
  }
}

__global__ void k_members(const int32_t* map, int32_t n, const uint32_t* mstart, uint32_t* cursor, int32_t* members) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = map[u];
    members[mstart[a] + atomicAdd(&cursor[a], 1u)] = (int32_t)u;
  }
}

// Staging capacity of a coarse vertex and its aggregation class.
__global__ void k_cclass(const unsigned long long* dsum, const unsigned long long* vw, int32_t nc, uint64_t* tcap,
                         uint8_t* cls, int32_t* vwgt_out, uint32_t* err, uint32_t t_wave, uint32_t t_block) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nc; a += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t d = dsum[a];
    tcap[a] = std::min<uint64_t>(d, (uint64_t)nc - 1);
    cls[a] = d == 0 ? 0 : (d <= t_wave ? 1 : (d <= t_block ? 2 : 3));
    const unsigned long long w = vw[a];
    if (w > 0x7FFFFFFFull) atomicOr(err, kErrOverflow);
    vwgt_out[a] = (int32_t)w;
  }
}

__global__ void k_class_list(const uint8_t* cls, int32_t nc, uint32_t* counters, int32_t* lists, int32_t stride) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nc; a += (int64_t)gridDim.x * blockDim.x) {
    const int c = cls[a];
    if (c == 0) continue;
    const uint32_t slot = atomicAdd(&counters[c], 1u);
    lists[(int64_t)(c - 1) * stride + slot] = (int32_t)a;
  }
}

template <int NT>
struct CSmem {
  DecodeSmem<NT> dec;
  int32_t scan[NT / kWave > 0 ? NT / kWave : 1];
  uint32_t distinct;
  uint32_t overflow;
};

__device__ __forceinline__ uint32_t ceil_log2(uint32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

// Inserts coarse edge (b, w) with a reservation guard: at most `limit`
// distinct keys are admitted, further new keys set sm.overflow.
template <int NT>
__device__ __forceinline__ void c_insert(int32_t* keys, int64_t* vals, uint32_t mask, uint32_t shift, int32_t b,
                                         int64_t w, uint32_t limit, CSmem<NT>& sm) {
  uint32_t h = slot_hash((uint32_t)b) >> shift;
  bool reserved = false;
  while (true) {
    const int32_t k = keys[h];
    if (k == b) {
      atomicAdd((unsigned long long*)&vals[h], (unsigned long long)w);
      return;
    }
    if (k == kEmpty) {
      if (!reserved) {
        if (atomicAdd(&sm.distinct, 1u) >= limit) {
          sm.overflow = 1;
          return;
        }
        reserved = true;
      }
      const int32_t old = atomicCAS(&keys[h], kEmpty, b);
      if (old == kEmpty || old == b) {
        atomicAdd((unsigned long long*)&vals[h], (unsigned long long)w);
        return;
      }
    }
    h = (h + 1) & mask;
  }
}

// Walks all members of coarse vertex a and calls f(b, w) for every fine
// edge leaving the cluster (b = coarse ID of the other endpoint).
template <int NT, bool COMP, typename F>
__device__ __forceinline__ bool for_cluster_edges(const GraphView& g, const int32_t* map, const int32_t* deg,
                                                  const int32_t* members, uint32_t m0, uint32_t m1, int32_t a,
                                                  CSmem<NT>& sm, F&& f) {
  const int tid = group_tid<NT>();
  bool ok = true;
  for (uint32_t m = m0; m < m1; ++m) {
    const int32_t u = members[m];
    const uint32_t d = (uint32_t)deg[u];
    if (d == 0) continue;
    auto body = [&](uint32_t, int32_t v, int32_t w) {
      const int32_t b = map[v];
      if (b != a) f(b, (int64_t)w);
    };
    if constexpr (COMP) {
      const Nbh h = nbh_locate(g, u, d);
      for (uint32_t ch = 0; ch < h.nchunks; ++ch) {
        uint64_t pos = nbh_chunk_pos(g, h, ch);
        const uint32_t first = ch * LP_CHUNK_LEN;
        const uint32_t cnt = (h.nchunks > 1) ? min((uint32_t)LP_CHUNK_LEN, d - first) : d;
        int32_t pv, pw;
        ok &= group_decode<NT>(g.bytes, pos, u, cnt, g.weighted, true, pv, pw, sm.dec, body);
      }
    } else {
      const uint64_t b0 = g.xadj[u];
      for (uint32_t k = tid; k < d; k += NT) body(k, g.adjncy[b0 + k], g.adjwgt ? g.adjwgt[b0 + k] : 1);
    }
  }
  return ok;
}

// Bitonic sort of (keys, vals)[0..cap) by key in LDS; cap is a power of two.
template <int NT>
__device__ __forceinline__ void lds_bitonic(int32_t* keys, int64_t* vals, uint32_t cap) {
  const int tid = group_tid<NT>();
  for (uint32_t k = 2; k <= cap; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < cap; i += NT) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const int32_t ki = keys[i], kj = keys[ixj];
          if ((ki > kj) == up) {
            keys[i] = kj;
            keys[ixj] = ki;
            const int64_t t = vals[i];
            vals[i] = vals[ixj];
            vals[ixj] = t;
          }
        }
      }
      group_sync<NT>();
    }
  }
}

// Sorts the table, then appends its k entries to the staging area at out.
// Returns k (group-uniform).
template <int NT>
__device__ __forceinline__ uint32_t flush_sorted(int32_t* keys, int64_t* vals, uint32_t cap, int32_t* ob, int64_t* ow,
                                                 uint32_t* err, CSmem<NT>& sm) {
  const int tid = group_tid<NT>();
  for (uint32_t i = tid; i < cap; i += NT)
    if (keys[i] == kEmpty) keys[i] = 0x7FFFFFFF;
  group_sync<NT>();
  lds_bitonic<NT>(keys, vals, cap);
  uint32_t mine = 0;
  for (uint32_t i = tid; i < cap; i += NT) mine += keys[i] != 0x7FFFFFFF;
  int32_t tot;
  (void)block_incl_scan_add<NT, int32_t>((int32_t)mine, sm.scan, &tot);
  for (uint32_t i = tid; i < (uint32_t)tot; i += NT) {
    ob[i] = keys[i];
    ow[i] = vals[i];
    if (vals[i] > 0x7FFFFFFFll) atomicOr(err, kErrOverflow);
  }
  group_sync<NT>();
  return (uint32_t)tot;
}

struct CArgs {
  GraphView g;
  const int32_t* map;
  const int32_t* deg;
  const int32_t* members;
  const uint32_t* mstart;
  const uint64_t* tbase;
  const uint64_t* tcap;
  int32_t* tb;       // staging: coarse neighbour
  int64_t* tw;       // staging: weight
  uint64_t* cdeg;    // coarse degree per coarse vertex
  uint32_t* err;
  int32_t nc;
};

// Light clusters: one group per coarse vertex, table capacity >= 2 * dsum.
template <int NT, bool COMP>
__global__ __launch_bounds__(NT == kWave ? 256 : NT) void k_contract_light(CArgs A, const int32_t* list, int32_t cnt,
                                                                           uint32_t tmax) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  constexpr int G = (NT == kWave) ? 4 : 1;
  const int gi = (NT == kWave) ? (int)(threadIdx.x / kWave) : 0;
  const int tid = group_tid<NT>();
  const size_t per = ((size_t)tmax * 12 + sizeof(CSmem<NT>) + 15) & ~size_t(15);
  uint8_t* base = smem_raw + gi * per;
  int64_t* vals = (int64_t*)base;
  int32_t* keys = (int32_t*)(base + (size_t)tmax * 8);
  CSmem<NT>& sm = *(CSmem<NT>*)(base + (size_t)tmax * 12);
  for (int64_t it = (int64_t)blockIdx.x * G + gi; it < cnt; it += (int64_t)gridDim.x * G) {
    const int32_t a = list[it];
    const uint32_t want = (uint32_t)std::min<uint64_t>(A.tcap[a], tmax / 2);
    const uint32_t logc = max(6u, ceil_log2(2 * max(want, 1u)));
    const uint32_t cap = 1u << logc, mask = cap - 1, shift = 32 - logc;
    for (uint32_t s = tid; s < cap; s += NT) {
      keys[s] = kEmpty;
      vals[s] = 0;
    }
    if (tid == 0) {
      sm.distinct = 0;
      sm.overflow = 0;
    }
    group_sync<NT>();
    bool ok = for_cluster_edges<NT, COMP>(A.g, A.map, A.deg, A.members, A.mstart[a], A.mstart[a + 1], a, sm,
                                          [&](int32_t b, int64_t w) {
                                            c_insert<NT>(keys, vals, mask, shift, b, w, cap, sm);
                                          });
    group_sync<NT>();
    if (!ok && tid == 0) atomicOr(A.err, kErrFormat);
    const uint32_t k = flush_sorted<NT>(keys, vals, cap, A.tb + A.tbase[a], A.tw + A.tbase[a], A.err, sm);
    if (tid == 0) A.cdeg[a] = k;
    group_sync<NT>();
  }
}

// Heavy clusters: one workgroup per coarse vertex. The coarse-ID range is
// swept in windows; each window's edges are aggregated in LDS, sorted and
// appended, so the neighbourhood comes out sorted. A window whose distinct
// count exceeds the table is split in two and retried.
template <bool COMP>
__global__ __launch_bounds__(kBlockThreads) void k_contract_heavy(CArgs A, const int32_t* list, int32_t cnt,
                                                                  uint32_t tcap) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  constexpr int NT = kBlockThreads;
  int64_t* vals = (int64_t*)smem_raw;
  int32_t* keys = (int32_t*)(smem_raw + (size_t)tcap * 8);
  CSmem<NT>& sm = *(CSmem<NT>*)(smem_raw + (size_t)tcap * 12);
  const int tid = threadIdx.x;
  const uint32_t mask = tcap - 1, shift = 32 - ceil_log2(tcap);
  const uint32_t limit = tcap / 2;
  for (int64_t it = blockIdx.x; it < cnt; it += gridDim.x) {
    const int32_t a = list[it];
    const uint64_t nc = (uint64_t)A.nc;
    // initial window width: expected distinct per window about limit / 2
    const uint64_t dist = std::max<uint64_t>(A.tcap[a], 1);
    uint64_t width = std::max<uint64_t>(1, (nc * (uint64_t)(limit / 2) + dist - 1) / dist);
    uint64_t lo = 0;
    uint64_t written = 0;
    int32_t* ob = A.tb + A.tbase[a];
    int64_t* ow = A.tw + A.tbase[a];
    while (lo < nc) {
      const uint64_t hi = std::min<uint64_t>(nc, lo + width);
      for (uint32_t s = tid; s < tcap; s += NT) {
        keys[s] = kEmpty;
        vals[s] = 0;
      }
      if (tid == 0) {
        sm.distinct = 0;
        sm.overflow = 0;
      }
      __syncthreads();
      bool ok = for_cluster_edges<NT, COMP>(A.g, A.map, A.deg, A.members, A.mstart[a], A.mstart[a + 1], a, sm,
                                            [&](int32_t b, int64_t w) {
                                              if ((uint64_t)b >= lo && (uint64_t)b < hi)
                                                c_insert<NT>(keys, vals, mask, shift, b, w, limit, sm);
                                            });
      __syncthreads();
      if (!ok && tid == 0) atomicOr(A.err, kErrFormat);
      if (sm.overflow && hi - lo > 1) {
        width = std::max<uint64_t>(1, (hi - lo) / 2);
        __syncthreads();
        continue;
      }
      const uint32_t k = flush_sorted<NT>(keys, vals, tcap, ob + written, ow + written, A.err, sm);
      written += k;
      lo = hi;
      // widen again if the window was sparse
      if (k < limit / 4 && width < nc) width *= 2;
      __syncthreads();
    }
    if (tid == 0) A.cdeg[a] = written;
    __syncthreads();
  }
}

// Final placement of the staged neighbourhoods (wave per coarse vertex).
__global__ __launch_bounds__(256) void k_contract_place(const uint64_t* cx, const uint64_t* tbase, const int32_t* tb,
                                                        const int64_t* tw, int32_t nc, int32_t* adjncy,
                                                        int32_t* adjwgt) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t a = wid; a < nc; a += nw) {
    const uint64_t o = cx[a], d = cx[a + 1] - o, t = tbase[a];
    for (uint64_t i = lane; i < d; i += kWave) {
      adjncy[o + i] = tb[t + i];
      adjwgt[o + i] = (int32_t)tw[t + i];
    }
  }
}

// Edge cut: wave per vertex, weight of edges to other clusters.
template <bool COMP>
__global__ __launch_bounds__(256) void k_cut(GraphView g, const int32_t* C, const int32_t* deg,
                                             unsigned long long* acc, uint32_t* err) {
  __shared__ DecodeSmem<kWave> dsm[4];
  __shared__ int64_t red[4];
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int64_t sum = 0;
  for (int64_t u = wid; u < g.n; u += nw) {
    const uint32_t d = (uint32_t)deg[u];
    if (d == 0) continue;
    const int32_t cu = C[u];
    auto body = [&](uint32_t, int32_t v, int32_t wt) {
      if (C[v] != cu) sum += wt;
    };
    if constexpr (COMP) {
      const Nbh h = nbh_locate(g, (int32_t)u, d);
      for (uint32_t ch = 0; ch < h.nchunks; ++ch) {
        uint64_t pos = nbh_chunk_pos(g, h, ch);
        const uint32_t first = ch * LP_CHUNK_LEN;
        const uint32_t cnt = (h.nchunks > 1) ? min((uint32_t)LP_CHUNK_LEN, d - first) : d;
        int32_t pv, pw;
        if (!group_decode<kWave>(g.bytes, pos, (int32_t)u, cnt, g.weighted, true, pv, pw, dsm[w], body) && lane == 0)
          atomicOr(err, kErrFormat);
      }
    } else {
      const uint64_t b = g.xadj[u];
      for (uint32_t k = lane; k < d; k += kWave) body(k, g.adjncy[b + k], g.adjwgt ? g.adjwgt[b + k] : 1);
    }
  }
  sum = wave_reduce_add(sum);
  if (lane == 0) red[w] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t t = red[0] + red[1] + red[2] + red[3];
    if (t) atomicAdd(acc, (unsigned long long)t);
  }
}

__global__ __launch_bounds__(256) void k_wdeg(const uint64_t* xadj, const int32_t* adjwgt, int32_t n,
                                              unsigned long long* max_wdeg, unsigned long long* max_deg) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t u = wid; u < n; u += nw) {
    const uint64_t b = xadj[u], e = xadj[u + 1];
    int64_t s = 0;
    for (uint64_t k = b + lane; k < e; k += kWave) s += adjwgt[k];
    s = wave_reduce_add(s);
    if (lane == 0) {
      atomicMax(max_wdeg, (unsigned long long)s);
      atomicMax(max_deg, (unsigned long long)(e - b));
    }
  }
}

__global__ void k_fill_u32(uint32_t* a, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

template <typename F>
lp_status set_lds(F* kern, size_t bytes) {
  LP_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return LP_OK;
}

constexpr uint32_t kCWave = 256;     // total member degree handled by one wavefront
constexpr uint32_t kCBlock = 4096;   // ... by one workgroup
constexpr uint32_t kCHeavyTable = 8192;

template <bool COMP>
lp_status contract_aggregate(CArgs A, const int32_t* lists, int32_t stride, const uint32_t* ccount, hipStream_t s) {
  // wave class
  if (ccount[1] > 0) {
    const uint32_t tmax = 2 * kCWave;
    const size_t per = ((size_t)tmax * 12 + sizeof(CSmem<kWave>) + 15) & ~size_t(15);
    auto k = k_contract_light<kWave, COMP>;
    LP_CHECK(set_lds(k, per * 4));
    hipLaunchKernelGGL(k, dim3(grid_for(ccount[1], 4, 1u << 20)), dim3(256), per * 4, s, A, lists, (int32_t)ccount[1],
                       tmax);
    LP_CHECK_LAUNCH();
  }
  if (ccount[2] > 0) {
    const uint32_t tmax = 2 * kCBlock;
    const size_t per = ((size_t)tmax * 12 + sizeof(CSmem<kBlockThreads>) + 15) & ~size_t(15);
    auto k = k_contract_light<kBlockThreads, COMP>;
    LP_CHECK(set_lds(k, per));
    hipLaunchKernelGGL(k, dim3(grid_for(ccount[2], 1, 1u << 20)), dim3(kBlockThreads), per, s, A, lists + stride,
                       (int32_t)ccount[2], tmax);
    LP_CHECK_LAUNCH();
  }
  if (ccount[3] > 0) {
    const size_t bytes = (size_t)kCHeavyTable * 12 + sizeof(CSmem<kBlockThreads>);
    auto k = k_contract_heavy<COMP>;
    LP_CHECK(set_lds(k, bytes));
    hipLaunchKernelGGL(k, dim3(grid_for(ccount[3], 1, 1u << 20)), dim3(kBlockThreads), bytes, s, A,
                       lists + 2 * (int64_t)stride, (int32_t)ccount[3], kCHeavyTable);
    LP_CHECK_LAUNCH();
  }
  return LP_OK;
}

}  // namespace

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_contract(const lp_graph* g, const int32_t* labels, int32_t* map_out, void* stream,
                                 lp_graph** coarse_out) {
  clear_error();
  if (!g || !coarse_out || (!labels && g->n > 0)) return LP_EINVAL;
  *coarse_out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const int32_t n = g->n;
  Scratch sc(s);
  struct Ctl {
    uint32_t err;
    uint32_t nc;
    uint32_t ccount[4];
    uint64_t two_mc;
    uint64_t tsum;
  };
  Ctl* ctl = sc.alloc<Ctl>(1);
  int32_t* deg = sc.alloc<int32_t>(n);
  uint32_t* flags = sc.alloc<uint32_t>(n);
  int32_t* map = map_out ? map_out : sc.alloc<int32_t>(n);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(ctl, 0, sizeof(Ctl), s));
  lp_graph* cg = new lp_graph();
  (void)hipGetDevice(&cg->device);
  lp_status st = LP_OK;
  do {
    if (n == 0) {
      if (hipMalloc((void**)&cg->xadj, sizeof(uint64_t)) != hipSuccess) { st = LP_ENOMEM; break; }
      if (hipMemsetAsync(cg->xadj, 0, sizeof(uint64_t), s) != hipSuccess) { st = LP_EDEVICE; break; }
      break;
    }
    st = compute_degrees(g, deg, s);
    if (st) break;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, flags, (int64_t)n, 0u);
    hipLaunchKernelGGL(k_check_mark, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, labels, n, flags, &ctl->err);
    st = last_error();
    if (st) break;
    st = scan_exclusive_u32(flags, flags, n, &ctl->nc, sc);
    if (st) break;
    Ctl h;
    if (hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = LP_EDEVICE; break; }
    if (h.err) { st = LP_EINVAL; break; }
    const int32_t nc = (int32_t)h.nc;
    cg->n = nc;
    uint32_t* cnt = sc.alloc<uint32_t>((size_t)nc + 1);
    uint32_t* cursor = sc.alloc<uint32_t>(nc);
    unsigned long long* vw = sc.alloc<unsigned long long>(nc);
    unsigned long long* dsum = sc.alloc<unsigned long long>(nc);
    int32_t* members = sc.alloc<int32_t>(n);
    uint64_t* tcap = sc.alloc<uint64_t>(nc);
    uint64_t* tbase = sc.alloc<uint64_t>(nc);
    uint64_t* cdeg = sc.alloc<uint64_t>((size_t)nc + 1);
    uint8_t* cls = sc.alloc<uint8_t>(nc);
    int32_t* lists = sc.alloc<int32_t>((size_t)3 * nc);
    if (sc.failed) { st = LP_ENOMEM; break; }
    if (hipMalloc((void**)&cg->vwgt, (size_t)nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&cg->xadj, ((size_t)nc + 1) * sizeof(uint64_t)) != hipSuccess) { st = LP_ENOMEM; break; }
    (void)hipMemsetAsync(cnt, 0, ((size_t)nc + 1) * sizeof(uint32_t), s);
    (void)hipMemsetAsync(cursor, 0, (size_t)nc * sizeof(uint32_t), s);
    (void)hipMemsetAsync(vw, 0, (size_t)nc * 8, s);
    (void)hipMemsetAsync(dsum, 0, (size_t)nc * 8, s);
    hipLaunchKernelGGL(k_map, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, labels, n, flags, deg, g->vwgt, map, cnt,
                       vw, dsum);
    st = last_error();
    if (st) break;
    st = scan_exclusive_u32(cnt, cnt, (int64_t)nc + 1, nullptr, sc);
    if (st) break;
    hipLaunchKernelGGL(k_members, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, map, n, cnt, cursor, members);
    hipLaunchKernelGGL(k_cclass, dim3(grid_for(nc, 256, 65536)), dim3(256), 0, s, dsum, vw, nc, tcap, cls, cg->vwgt,
                       &ctl->err, kCWave, kCBlock);
    hipLaunchKernelGGL(k_class_list, dim3(grid_for(nc, 256, 65536)), dim3(256), 0, s, cls, nc, ctl->ccount - 0, lists,
                       nc);
    st = last_error();
    if (st) break;
    st = scan_exclusive_u64(tcap, tbase, nc, &ctl->tsum, sc);
    if (st) break;
    if (hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = LP_EDEVICE; break; }
    if (h.err) { st = LP_EOVERFLOW; break; }
    int32_t* tb = sc.alloc<int32_t>(h.tsum);
    int64_t* tw = sc.alloc<int64_t>(h.tsum);
    if (sc.failed) { st = LP_ENOMEM; break; }
    (void)hipMemsetAsync(cdeg, 0, ((size_t)nc + 1) * sizeof(uint64_t), s);
    CArgs A;
    A.g = g->view();
    A.map = map;
    A.deg = deg;
    A.members = members;
    A.mstart = cnt;
    A.tbase = tbase;
    A.tcap = tcap;
    A.tb = tb;
    A.tw = tw;
    A.cdeg = cdeg;
    A.err = &ctl->err;
    A.nc = nc;
    uint32_t cc[4] = {0, h.ccount[1], h.ccount[2], h.ccount[3]};
    st = g->compressed ? contract_aggregate<true>(A, lists, nc, cc, s) : contract_aggregate<false>(A, lists, nc, cc, s);
    if (st) break;
    st = scan_exclusive_u64(cdeg, cg->xadj, (int64_t)nc + 1, &ctl->two_mc, sc);
    if (st) break;
    if (hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = LP_EDEVICE; break; }
    if (h.err & kErrFormat) { st = LP_EINVAL; break; }
    if (h.err) { st = LP_EOVERFLOW; break; }
    cg->two_m = h.two_mc;
    cg->weighted = 1;
    if (hipMalloc((void**)&cg->adjncy, (h.two_mc ? h.two_mc : 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&cg->adjwgt, (h.two_mc ? h.two_mc : 1) * sizeof(int32_t)) != hipSuccess) { st = LP_ENOMEM; break; }
    hipLaunchKernelGGL(k_contract_place, dim3(grid_for((int64_t)nc * kWave, 256, 65536)), dim3(256), 0, s, cg->xadj,
                       tbase, tb, tw, nc, cg->adjncy, cg->adjwgt);
    st = last_error();
    if (st) break;
  } while (0);
  if (st == LP_OK && hipStreamSynchronize(s) != hipSuccess) st = LP_EDEVICE;
  if (st != LP_OK) {
    lp_graph_free(cg);
    return st;
  }
  // coarse metadata used by later calls: total weight, degree maxima
  {
    Scratch sc2(s);
    unsigned long long* mx = sc2.alloc<unsigned long long>(2);
    if (!mx) {
      lp_graph_free(cg);
      return LP_ENOMEM;
    }
    unsigned long long hm[2] = {0, 0};
    if (hipMemsetAsync(mx, 0, 16, s) == hipSuccess && cg->n > 0)
      hipLaunchKernelGGL(k_wdeg, dim3(grid_for((int64_t)cg->n * kWave, 256, 65536)), dim3(256), 0, s, cg->xadj,
                         cg->adjwgt, cg->n, mx, mx + 1);
    if (hipMemcpyAsync(hm, mx, 16, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      lp_graph_free(cg);
      return LP_EDEVICE;
    }
    cg->max_wdeg = (int64_t)hm[0];
    cg->max_deg = (int64_t)hm[1];
    cg->total_vwgt = g->total_vwgt;
  }
  *coarse_out = cg;
  return LP_OK;
}

extern "C" lp_status lp_edge_cut(const lp_graph* g, const int32_t* labels, int64_t* cut_out, void* stream) {
  clear_error();
  if (!g || !cut_out || (!labels && g->n > 0)) return LP_EINVAL;
  *cut_out = 0;
  if (g->n == 0) return LP_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  int32_t* deg = sc.alloc<int32_t>(g->n);
  struct Acc {
    unsigned long long sum;
    uint32_t err, pad;
  };
  Acc* acc = sc.alloc<Acc>(1);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(acc, 0, sizeof(Acc), s));
  LP_CHECK(compute_degrees(g, deg, s));
  const unsigned grid = grid_for((int64_t)g->n * kWave, 256, 16384);
  if (g->compressed)
    hipLaunchKernelGGL(k_cut<true>, dim3(grid), dim3(256), 0, s, g->view(), labels, deg, &acc->sum, &acc->err);
  else
    hipLaunchKernelGGL(k_cut<false>, dim3(grid), dim3(256), 0, s, g->view(), labels, deg, &acc->sum, &acc->err);
  LP_CHECK_LAUNCH();
  Acc h;
  LP_CHECK_HIP(hipMemcpyAsync(&h, acc, sizeof(Acc), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  if (h.err) return LP_EINVAL;
  *cut_out = (int64_t)(h.sum / 2);
  return LP_OK;
}
