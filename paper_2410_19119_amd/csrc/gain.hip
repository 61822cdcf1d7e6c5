// Sparse gain table (Section V of the paper; layout in gain.h), the public
// lp_gain_table handle, and the table-driven selection step that lp_refine
// uses instead of re-rating every neighbourhood in each round.
#include "decode.h"
#include "gain.h"

namespace lp {

lp_status plan_degrees(const lp_graph* g, const int32_t** deg, hipStream_t s);

namespace {

constexpr int kGtLaneMax = 16;  // vertices up to this degree are filled / selected by one lane
constexpr int kGtWaves = 4;     // wavefronts per 256-thread workgroup
constexpr int32_t kGtEmpty = -1;

template <typename V>
struct GtView {
  int32_t n, k;
  const uint64_t* off;
  const uint8_t* dense;
  int32_t* key;
  V* val;
  uint32_t* flag;
  int32_t* list;
  uint32_t* cnt;
};

template <typename V>
GtView<V> view_of(const GainTable& t) {
  return GtView<V>{t.g->n, t.k, t.off, t.dense, t.key, (V*)t.val, t.flag, t.list, t.cnt};
}

// Home slot of block b in a hash slice of L = 2^s slots (the top s bits of a
// multiplicative hash).
__device__ __forceinline__ uint32_t gt_hash(int32_t b, uint32_t L) {
  return ((uint32_t)b * 0x9E3779B1u) >> (33u - (uint32_t)__ffs(L));
}

__device__ __forceinline__ void gt_atomic_add(int32_t* p, int32_t w) { atomicAdd(p, w); }
__device__ __forceinline__ void gt_atomic_add(int64_t* p, int64_t w) {
  atomicAdd((unsigned long long*)p, (unsigned long long)w);
}

// Slot of block b in u's slice, inserting it if `insert`; -1 if absent (or,
// when inserting, if the slice has no free slot left).
template <typename V>
__device__ int64_t gt_slot(const GtView<V>& t, int32_t u, int32_t b, bool insert) {
  const uint64_t base = t.off[u];
  if (t.dense[u]) return (int64_t)(base + (uint32_t)b);
  const uint32_t L = (uint32_t)(t.off[u + 1] - base);
  uint32_t h = gt_hash(b, L);
  for (uint32_t p = 0; p < L; ++p) {
    const uint64_t s = base + h;
    const int32_t kk = t.key[s];
    if (kk == b) return (int64_t)s;
    if (kk == kGtEmpty) {
      if (!insert) return -1;
      const int32_t old = atomicCAS(&t.key[s], kGtEmpty, b);
      if (old == kGtEmpty || old == b) return (int64_t)s;
    }
    h = (h + 1) & (L - 1);
  }
  return -1;
}

template <typename V>
__device__ __forceinline__ bool gt_add(const GtView<V>& t, int32_t u, int32_t b, V w) {
  const int64_t s = gt_slot(t, u, b, true);
  if (s < 0) return false;
  gt_atomic_add(&t.val[s], w);
  return true;
}

template <typename V>
__device__ __forceinline__ V gt_get(const GtView<V>& t, int32_t u, int32_t b) {
  const int64_t s = gt_slot(t, u, b, false);
  return s < 0 ? (V)0 : t.val[s];
}

// Every neighbour (v, w) of u, for one wavefront: chunk c of a chunked
// neighbourhood, or all of it (c < 0). Plain graphs are cut into the same
// 1000-edge pieces above the chunking threshold.
template <typename F>
__device__ void wave_visit(const GraphView& g, int32_t u, uint32_t deg, int32_t c, DecodeSmem<kWave>& dsm, F&& f) {
  if (g.offs && g.intervals) {
    // interval-coded: every lane decodes whole chunks on its own
    const Nbh h = nbh_locate(g, u, deg);
    const uint32_t c0 = c < 0 ? 0u : (uint32_t)c, c1 = c < 0 ? h.nchunks : (uint32_t)c + 1;
    for (uint32_t ch = c0 + (uint32_t)lane_id(); ch < c1; ch += kWave) {
      const uint32_t first = ch * LP_CHUNK_LEN;
      const uint32_t cnt = h.nchunks > 1 ? min((uint32_t)LP_CHUNK_LEN, deg - first) : deg;
      lane_decode_chunk(g, u, nbh_chunk_pos(g, h, ch), cnt, [&](uint32_t, int32_t v, int32_t w) { f(v, w); });
    }
  } else if (g.offs) {
    const Nbh h = nbh_locate(g, u, deg);
    const uint32_t c0 = c < 0 ? 0u : (uint32_t)c, c1 = c < 0 ? h.nchunks : (uint32_t)c + 1;
    for (uint32_t ch = c0; ch < c1; ++ch) {
      uint64_t pos = nbh_chunk_pos(g, h, ch);
      const uint32_t first = ch * LP_CHUNK_LEN;
      const uint32_t cnt = h.nchunks > 1 ? min((uint32_t)LP_CHUNK_LEN, deg - first) : deg;
      int32_t pv = 0, pw = 0;
      (void)group_decode<kWave>(g.bytes, pos, u, cnt, g.weighted, true, pv, pw, dsm,
                                [&](uint32_t, int32_t v, int32_t w) { f(v, w); });
    }
  } else {
    const uint64_t e0 = g.xadj[u];
    uint32_t lo = 0, hi = deg;
    if (c >= 0) {
      lo = (uint32_t)c * LP_CHUNK_LEN;
      hi = min(deg, lo + (uint32_t)LP_CHUNK_LEN);
    }
    for (uint32_t e = lo + (uint32_t)lane_id(); e < hi; e += kWave)
      f(g.adjncy[e0 + e], g.adjwgt ? g.adjwgt[e0 + e] : 1);
  }
}

// Every neighbour of a short neighbourhood, for one lane.
template <typename F>
__device__ __forceinline__ void lane_visit(const GraphView& g, int32_t u, uint32_t deg, F&& f) {
  if (g.offs) {
    lane_decode(g, u, deg, [&](uint32_t, int32_t v, int32_t w) { f(v, w); });
  } else {
    const uint64_t e0 = g.xadj[u];
    for (uint32_t e = 0; e < deg; ++e) f(g.adjncy[e0 + e], g.adjwgt ? g.adjwgt[e0 + e] : 1);
  }
}

// Slice length and kind of every vertex: none for isolated vertices, a dense
// row of k when pow2(2 deg) >= k, else pow2(2 deg) hash slots.
__global__ void k_gt_len(const int32_t* deg, int32_t n, int32_t k, uint64_t* len, uint8_t* dense) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t d = (uint64_t)deg[u];
    uint64_t L = 0;
    uint8_t dn = 0;
    if (d > 0) {
      L = 2;
      while (L < 2 * d) L <<= 1;
      if (L >= (uint64_t)k) {
        L = (uint64_t)k;
        dn = 1;
      }
    }
    len[u] = L;
    dense[u] = dn;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) len[n] = 0;
}

template <typename V>
__global__ void k_gt_clear(int32_t* key, V* val, uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
    key[i] = kGtEmpty;
    val[i] = 0;
  }
}

__global__ void k_gt_zero(uint32_t* a, int64_t m) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

template <typename V>
__global__ __launch_bounds__(256) void k_gt_fill_lane(GraphView g, const int32_t* deg, const int32_t* blocks,
                                                      GtView<V> t) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < t.n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = deg[u];
    if (d == 0 || d > kGtLaneMax) continue;
    lane_visit(g, (int32_t)u, (uint32_t)d, [&](int32_t v, int32_t w) { (void)gt_add(t, (int32_t)u, blocks[v], (V)w); });
  }
}

// Work items of the wavefront fill: one per vertex above kGtLaneMax, one per
// chunk above the chunking threshold. Every thread takes kGtItemRun
// consecutive vertices, so that one counter atomic serves a whole workgroup.
constexpr int kGtItemRun = 16;

__device__ __forceinline__ uint32_t gt_items_of(uint32_t d, uint32_t thr) {
  return d <= (uint32_t)kGtLaneMax ? 0u : d > thr ? (d + LP_CHUNK_LEN - 1) / LP_CHUNK_LEN : 1u;
}

__global__ __launch_bounds__(256) void k_gt_items(const int32_t* deg, int32_t n, uint32_t thr, int2* items,
                                                  uint32_t* nitems) {
  __shared__ int32_t scan[256 / kWave + 1];
  __shared__ uint32_t base_sm;
  constexpr int64_t kSpan = 256 * kGtItemRun;
  for (int64_t b = (int64_t)blockIdx.x * kSpan; b < n; b += (int64_t)gridDim.x * kSpan) {
    const int64_t u0 = b + (int64_t)threadIdx.x * kGtItemRun;
    const int64_t u1 = min((int64_t)n, u0 + kGtItemRun);
    uint32_t cnt = 0;
    for (int64_t u = u0; u < u1; ++u) cnt += gt_items_of((uint32_t)deg[u], thr);
    int32_t tot;
    const uint32_t incl = (uint32_t)block_incl_scan_add<256, int32_t>((int32_t)cnt, scan, &tot);
    if (threadIdx.x == 255) base_sm = tot ? atomicAdd(nitems, (uint32_t)tot) : 0u;
    __syncthreads();
    uint32_t o = base_sm + incl - cnt;
    for (int64_t u = u0; u < u1; ++u) {
      const uint32_t ni = gt_items_of((uint32_t)deg[u], thr);
      for (uint32_t j = 0; j < ni; ++j) items[o++] = make_int2((int)u, ni > 1 ? (int)j : -1);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void lds_add_v(int32_t* p, int32_t w) { atomicAdd(p, w); }
__device__ __forceinline__ void lds_add_v(int64_t* p, int64_t w) {
  atomicAdd((unsigned long long*)p, (unsigned long long)w);
}

// One wavefront per work item. A dense row of at most kGtStage blocks is
// summed in the wavefront's LDS first and flushed with one global atomic per
// nonzero block, so that the edges of a vertex do not all hit the same few
// global addresses.
constexpr int kGtStage = 1024;

template <typename V>
__global__ __launch_bounds__(256) void k_gt_fill_wave(GraphView g, const int32_t* deg, const int32_t* blocks,
                                                      const int2* items, const uint32_t* nitems, GtView<V> t) {
  __shared__ DecodeSmem<kWave> dsm[kGtWaves];
  __shared__ V stage[kGtWaves][kGtStage];
  const int w = threadIdx.x / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const uint32_t m = *nitems;
  const bool staged_k = t.k <= kGtStage;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < m; i += nw) {
    const int2 it = items[i];
    const int32_t u = it.x;
    if (staged_k && t.dense[u]) {
      for (int32_t q = lane_id(); q < t.k; q += kWave) stage[w][q] = 0;
      wave_sync_lds();
      wave_visit(g, u, (uint32_t)deg[u], it.y, dsm[w],
                 [&](int32_t v, int32_t wt) { lds_add_v(&stage[w][blocks[v]], (V)wt); });
      wave_sync_lds();
      const uint64_t base = t.off[u];
      for (int32_t q = lane_id(); q < t.k; q += kWave) {
        const V a = stage[w][q];
        if (a) gt_atomic_add(&t.val[base + q], a);
      }
      wave_sync_lds();
    } else {
      wave_visit(g, u, (uint32_t)deg[u], it.y, dsm[w], [&](int32_t v, int32_t wt) {
        (void)gt_add(t, u, blocks[v], (V)wt);
      });
    }
  }
}

__device__ __forceinline__ void gt_consider(const GtRound& r, int32_t c, int64_t val, int64_t wu, Cand& best) {
  if (val <= 0 || val < best.r) return;
  const Cand cd{val, tiebreak_key(r.seed, r.round, (uint32_t)c), c};
  if (cand_better(cd, best) && r.W[c] + wu <= r.cap) best = cd;
}

__device__ __forceinline__ void gt_emit(const GtRound& r, int32_t u, const Cand& best, int64_t own) {
  if (best.c >= 0 && best.r > own) {
    r.ptgt[u] = best.c;
    r.pgain[u] = best.r - own;
  } else {
    r.ptgt[u] = -1;
  }
}

// One lane per vertex: own affinity and the best feasible other block, by
// (affinity desc, tie-break key asc), as the rating step of the LP rounds.
template <typename V>
__global__ __launch_bounds__(256) void k_gt_select_lane(GtView<V> t, GtRound r, const int32_t* list, int32_t cnt) {
  if (*r.done) return;
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= cnt) return;
  const int32_t u = list[i];
  const int32_t own_c = r.C[u];
  const int64_t wu = r.vwgt ? r.vwgt[u] : 1;
  const uint64_t base = t.off[u];
  const uint32_t L = (uint32_t)(t.off[u + 1] - base);
  const bool dn = t.dense[u];
  int64_t own = 0;
  Cand best = cand_none();
  for (uint32_t q = 0; q < L; ++q) {
    const int32_t c = dn ? (int32_t)q : t.key[base + q];
    if (c == kGtEmpty) continue;
    const int64_t a = (int64_t)t.val[base + q];
    if (c == own_c) own = a;
    else gt_consider(r, c, a, wu, best);
  }
  gt_emit(r, u, best, own);
}

// One wavefront per vertex (lanes stride over the slice).
template <typename V>
__global__ __launch_bounds__(256) void k_gt_select_wave(GtView<V> t, GtRound r, const int32_t* list, int32_t cnt) {
  if (*r.done) return;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < cnt; i += nw) {
    const int32_t u = list[i];
    const int32_t own_c = r.C[u];
    const int64_t wu = r.vwgt ? r.vwgt[u] : 1;
    const uint64_t base = t.off[u];
    const uint32_t L = (uint32_t)(t.off[u + 1] - base);
    const bool dn = t.dense[u];
    int64_t own = 0;
    Cand best = cand_none();
    for (uint32_t q = (uint32_t)lane_id(); q < L; q += kWave) {
      const int32_t c = dn ? (int32_t)q : t.key[base + q];
      if (c == kGtEmpty) continue;
      const int64_t a = (int64_t)t.val[base + q];
      if (c == own_c) own = a;
      else gt_consider(r, c, a, wu, best);
    }
    best = wave_best(best);
    own = wave_reduce_add(own);
    if (lane_id() == 0) gt_emit(r, u, best, own);
  }
}

// The update of one neighbour v of a moved vertex: w(u, v) leaves block
// `from` and joins block `to` in v's slice.
template <typename V>
__device__ __forceinline__ void gt_move_edge(const GtView<V>& t, int32_t v, int32_t from, int32_t to, int32_t wt) {
  const int64_t s = gt_slot(t, v, from, false);
  if (s >= 0) gt_atomic_add(&t.val[s], (V)-wt);
  else atomicAdd(&t.cnt[1], 1u);
  if (!gt_add(t, v, to, (V)wt) && atomicExch(&t.flag[v], 1u) == 0u) t.list[atomicAdd(&t.cnt[0], 1u)] = v;
}

// Work items of an update: one per move of a vertex above kGtLaneMax, one per
// chunk above the chunking threshold ({move index, chunk or -1}).
__global__ __launch_bounds__(256) void k_gt_move_items(const int4* moves, const uint32_t* count, const int32_t* deg,
                                                       uint32_t thr, int2* items, uint32_t* nitems) {
  const int64_t m = *count;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < m; b += stride) {
    const int64_t i = b + threadIdx.x;
    uint32_t ni = 0;
    if (i < m) {
      const int4 mv = moves[i];
      if (mv.x >= 0 && mv.y != mv.z) ni = gt_items_of((uint32_t)deg[mv.x], thr);  // short ones: k_gt_update_lane
    }
    const uint32_t incl = wave_incl_scan_add(ni);
    uint32_t base = 0;
    if (lane_id() == kWave - 1 && incl) base = atomicAdd(nitems, incl);
    base = __shfl(base, kWave - 1, kWave);
    for (uint32_t j = 0; j < ni; ++j) items[base + incl - ni + j] = make_int2((int)i, ni > 1 ? (int)j : -1);
  }
}

// Wavefront per update item of a move {u, from, to}: every neighbour v of u
// (in the item's chunk) moves w(u, v) from block `from` to block `to` in its
// slice. A slice without a free slot for `to` is listed for a rebuild; a
// missing `from` entry is counted (cnt[1]; never expected).
template <typename V>
__global__ __launch_bounds__(256) void k_gt_update(GraphView g, const int32_t* deg, const int4* moves,
                                                   const int2* items, const uint32_t* nitems, GtView<V> t) {
  __shared__ DecodeSmem<kWave> dsm[kGtWaves];
  const int w = threadIdx.x / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const uint32_t m = *nitems;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < m; i += nw) {
    const int2 it = items[i];
    const int4 mv = moves[it.x];
    const int32_t u = mv.x, from = mv.y, to = mv.z;
    wave_visit(g, u, (uint32_t)deg[u], it.y, dsm[w],
               [&](int32_t v, int32_t wt) { gt_move_edge(t, v, from, to, wt); });
  }
}

// One lane per move of a vertex of degree <= kGtLaneMax.
template <typename V>
__global__ __launch_bounds__(256) void k_gt_update_lane(GraphView g, const int32_t* deg, const int4* moves,
                                                        const uint32_t* count, GtView<V> t) {
  const int64_t m = *count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int4 mv = moves[i];
    if (mv.x < 0 || mv.y == mv.z) continue;
    const uint32_t d = (uint32_t)deg[mv.x];
    if (d == 0 || d > (uint32_t)kGtLaneMax) continue;
    lane_visit(g, mv.x, d, [&](int32_t v, int32_t wt) { gt_move_edge(t, v, mv.y, mv.z, wt); });
  }
}

// Rebuilds the listed slices from the current blocks (a slice holds at most
// deg(v) <= L / 2 live blocks, so the rebuild always fits).
template <typename V>
__global__ __launch_bounds__(256) void k_gt_rebuild(GraphView g, const int32_t* deg, const int32_t* blocks,
                                                    GtView<V> t) {
  __shared__ DecodeSmem<kWave> dsm[kGtWaves];
  const int w = threadIdx.x / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const uint32_t m = t.cnt[0];
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < m; i += nw) {
    const int32_t v = t.list[i];
    const uint64_t base = t.off[v];
    const uint32_t L = (uint32_t)(t.off[v + 1] - base);
    for (uint32_t q = (uint32_t)lane_id(); q < L; q += kWave) {
      t.key[base + q] = kGtEmpty;
      t.val[base + q] = 0;
    }
    __threadfence();
    __builtin_amdgcn_wave_barrier();
    wave_visit(g, v, (uint32_t)deg[v], -1, dsm[w],
               [&](int32_t x, int32_t wt) { (void)gt_add(t, v, blocks[x], (V)wt); });
    if (lane_id() == 0) t.flag[v] = 0;
  }
}

// Ends an update: the rebuilt slices are counted (cnt[2]) and the list emptied.
__global__ void k_gt_reset_list(uint32_t* cnt) {
  cnt[2] += cnt[0];
  cnt[0] = 0;
}

template <typename V>
lp_status gt_fill(const GainTable& t, const int32_t* blocks, Scratch& sc) {
  hipStream_t s = sc.stream();
  const lp_graph* g = t.g;
  const GtView<V> v = view_of<V>(t);
  const int32_t n = g->n;
  hipLaunchKernelGGL(k_gt_clear<V>, dim3(grid_for((int64_t)t.entries, 256, 65536)), dim3(256), 0, s, t.key, (V*)t.val,
                     t.entries);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_fill_lane<V>, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, g->view(), t.deg, blocks, v);
  LP_CHECK_LAUNCH();
  uint32_t* nitems = t.cnt + 3;
  hipLaunchKernelGGL(k_gt_zero, dim3(1), dim3(64), 0, s, nitems, (int64_t)1);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_items, dim3(grid_for(n, 256 * kGtItemRun, 65536)), dim3(256), 0, s, t.deg, n,
                     chunk_threshold(g->intervals), t.items, nitems);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_fill_wave<V>, dim3(grid_for(n, 256 / kWave * 8, 16384)), dim3(256), 0, s, g->view(), t.deg,
                     blocks, t.items, nitems, v);
  return last_error();
}

template <typename V>
lp_status gt_select_t(const GainTable& t, const GtRound& r, const int32_t* lane_list, int32_t nlane,
                      const int32_t* wave_list, int32_t nwave, hipStream_t s) {
  const GtView<V> v = view_of<V>(t);
  if (nlane > 0) {
    hipLaunchKernelGGL(k_gt_select_lane<V>, dim3(grid_for(nlane, 256)), dim3(256), 0, s, v, r, lane_list, nlane);
    LP_CHECK_LAUNCH();
  }
  if (nwave > 0) {
    hipLaunchKernelGGL(k_gt_select_wave<V>, dim3(grid_for(nwave, kGtWaves, 1u << 20)), dim3(256), 0, s, v, r,
                       wave_list, nwave);
    LP_CHECK_LAUNCH();
  }
  return LP_OK;
}

template <typename V>
lp_status gt_update_t(const GainTable& t, const int4* moves, const uint32_t* count, int64_t max_moves,
                      const int32_t* blocks, hipStream_t s) {
  const GtView<V> v = view_of<V>(t);
  if (max_moves <= 0) return LP_OK;
  hipLaunchKernelGGL(k_gt_zero, dim3(1), dim3(64), 0, s, t.cnt + 3, (int64_t)1);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_update_lane<V>, dim3(grid_for(max_moves, 256, 16384)), dim3(256), 0, s, t.g->view(), t.deg,
                     moves, count, v);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_move_items, dim3(grid_for(max_moves, 256, 16384)), dim3(256), 0, s, moves, count, t.deg,
                     chunk_threshold(t.g->intervals), t.items, t.cnt + 3);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_update<V>, dim3(grid_for(max_moves, kGtWaves, 8192)), dim3(256), 0, s, t.g->view(), t.deg,
                     moves, t.items, t.cnt + 3, v);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_rebuild<V>, dim3(256), dim3(256), 0, s, t.g->view(), t.deg, blocks, v);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_reset_list, dim3(1), dim3(1), 0, s, t.cnt);
  return last_error();
}

}  // namespace

lp_status gt_create(const lp_graph* g, const int32_t* blocks, int32_t k, hipStream_t s, GainTable* t) {
  *t = GainTable{};
  t->g = g;
  t->k = k;
  t->wide = g->max_wdeg > 0x7FFFFFFFll;
  const int32_t n = g->n;
  LP_CHECK(plan_degrees(g, &t->deg, s));
  auto grab = [&](size_t bytes) {
    void* p = cache_alloc(bytes ? bytes : 1, s);
    t->bytes += bytes;
    return p;
  };
  t->off = (uint64_t*)grab(((size_t)n + 1) * 8);
  t->dense = (uint8_t*)grab((size_t)n);
  t->flag = (uint32_t*)grab((size_t)n * 4);
  t->list = (int32_t*)grab((size_t)n * 4);
  t->cnt = (uint32_t*)grab(4 * 4);
  t->nitems_cap = (uint64_t)n + g->two_m / LP_CHUNK_LEN + 1;
  t->items = (int2*)grab(t->nitems_cap * sizeof(int2));
  if (!t->off || !t->dense || !t->flag || !t->list || !t->cnt || !t->items) {
    gt_release(t, s);
    return LP_ENOMEM;
  }
  Scratch sc(s);
  hipLaunchKernelGGL(k_gt_len, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, t->deg, n, k, t->off, t->dense);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u64(t->off, t->off, (int64_t)n + 1, nullptr, sc));
  uint64_t entries = 0;
  LP_CHECK_HIP(hipMemcpyAsync(&entries, t->off + n, 8, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  t->entries = entries;
  t->key = (int32_t*)grab(entries * 4);
  t->val = grab(entries * (t->wide ? 8 : 4));
  if (!t->key || !t->val) {
    gt_release(t, s);
    return LP_ENOMEM;
  }
  hipLaunchKernelGGL(k_gt_zero, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, t->flag, (int64_t)n);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_zero, dim3(1), dim3(64), 0, s, t->cnt, (int64_t)4);
  LP_CHECK_LAUNCH();
  return t->wide ? gt_fill<int64_t>(*t, blocks, sc) : gt_fill<int32_t>(*t, blocks, sc);
}

void gt_release(GainTable* t, hipStream_t s) {
  for (void* p : {(void*)t->off, (void*)t->dense, (void*)t->flag, (void*)t->list, (void*)t->cnt, (void*)t->key, t->val,
                  (void*)t->items})
    if (p) cache_free(p, s);
  *t = GainTable{};
}

lp_status gt_select(const GainTable& t, const GtRound& r, const int32_t* lane_list, int32_t nlane,
                    const int32_t* wave_list, int32_t nwave, hipStream_t s) {
  return t.wide ? gt_select_t<int64_t>(t, r, lane_list, nlane, wave_list, nwave, s)
                : gt_select_t<int32_t>(t, r, lane_list, nlane, wave_list, nwave, s);
}

lp_status gt_update(const GainTable& t, const int4* moves, const uint32_t* count, int64_t max_moves,
                    const int32_t* blocks, hipStream_t s) {
  return t.wide ? gt_update_t<int64_t>(t, moves, count, max_moves, blocks, s)
                : gt_update_t<int32_t>(t, moves, count, max_moves, blocks, s);
}

}  // namespace lp

// ------------------------------------------------------------ public handle --

using namespace lp;

struct lp_gain_table {
  GainTable t;
  int32_t* blocks = nullptr;  // the table's partition
  int4* moves = nullptr;      // n
  uint32_t* bad = nullptr;    // [0] argument errors of the last call, [1] move count
  hipStream_t stream = nullptr;
  int device = 0;
};

namespace lp {
namespace {

__global__ void k_gt_check_blocks(const int32_t* b, int32_t n, int32_t k, uint32_t* bad) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    if ((uint32_t)b[u] >= (uint32_t)k) *bad = 1u;
}

template <typename V>
__global__ void k_gt_query(GtView<V> t, int64_t m, const int32_t* us, const int32_t* bs, int64_t* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = us[i], b = bs[i];
    out[i] = ((uint32_t)u < (uint32_t)t.n && (uint32_t)b < (uint32_t)t.k) ? (int64_t)gt_get(t, u, b) : -1;
  }
}

// Move batches: vertices in range and distinct (flag exchange), targets in
// range; the flags are cleared again by k_gt_unflag.
__global__ void k_gt_check_moves(const int32_t* us, const int32_t* to, int64_t m, int32_t n, int32_t k, uint32_t* flag,
                                 uint32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = us[i];
    if ((uint32_t)u >= (uint32_t)n || (uint32_t)to[i] >= (uint32_t)k) {
      *bad = 1u;
      continue;
    }
    if (atomicExch(&flag[u], 1u) != 0u) *bad = 1u;
  }
}

__global__ void k_gt_unflag(const int32_t* us, int64_t m, int32_t n, uint32_t* flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    if ((uint32_t)us[i] < (uint32_t)n) flag[us[i]] = 0u;
}

__global__ void k_gt_prep_moves(const int32_t* us, const int32_t* to, int64_t m, int32_t* blocks, int4* moves,
                                uint32_t* count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = us[i];
    moves[i] = make_int4(u, blocks[u], to[i], 0);
    blocks[u] = to[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = (uint32_t)m;
}

lp_status host_flag(const uint32_t* dev, hipStream_t s, uint32_t* out) {
  LP_CHECK_HIP(hipMemcpyAsync(out, dev, 4, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  return LP_OK;
}

}  // namespace
}  // namespace lp

extern "C" lp_status lp_gain_table_create(const lp_graph* g, const int32_t* blocks, int32_t k, void* stream,
                                          lp_gain_table** out) {
  clear_error();
  if (!g || !out || g->nbatch || k < 1 || (g->n > 0 && (k > g->n || !blocks))) return LP_EINVAL;
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  const int32_t n = g->n;
  auto* h = new lp_gain_table();
  h->stream = s;
  LP_CHECK_HIP(hipGetDevice(&h->device));
  h->blocks = (int32_t*)cache_alloc((size_t)std::max(n, 1) * 4, s);
  h->moves = (int4*)cache_alloc((size_t)std::max(n, 1) * 16, s);
  h->bad = (uint32_t*)cache_alloc(16, s);
  lp_status st = (h->blocks && h->moves && h->bad) ? LP_OK : LP_ENOMEM;
  if (!st) {
    hipLaunchKernelGGL(k_gt_zero, dim3(1), dim3(64), 0, s, h->bad, (int64_t)4);
    if (n > 0) {
      hipLaunchKernelGGL(k_gt_check_blocks, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, blocks, n, k, h->bad);
      uint32_t bad = 0;
      st = host_flag(h->bad, s, &bad);
      if (!st && bad) st = LP_EINVAL;
    }
  }
  if (!st && n > 0 && hipMemcpyAsync(h->blocks, blocks, (size_t)n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    st = LP_EDEVICE;
  if (!st && n > 0) st = gt_create(g, h->blocks, k, s, &h->t);
  if (!st && n == 0) {
    h->t.g = g;
    h->t.k = k;
  }
  if (st) {
    lp_gain_table_free(h);
    return st;
  }
  *out = h;
  return LP_OK;
}

extern "C" lp_status lp_gain_table_affinity(const lp_gain_table* h, int64_t count, const int32_t* vertices,
                                            const int32_t* blocks, int64_t* out, void* stream) {
  clear_error();
  if (!h || count < 0 || (count > 0 && (!vertices || !blocks || !out))) return LP_EINVAL;
  if (count == 0) return LP_OK;
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = grid_for(count, 256, 65536);
  if (h->t.g->n == 0) return LP_EINVAL;
  if (h->t.wide)
    hipLaunchKernelGGL(k_gt_query<int64_t>, dim3(grid), dim3(256), 0, s, view_of<int64_t>(h->t), count, vertices,
                       blocks, out);
  else
    hipLaunchKernelGGL(k_gt_query<int32_t>, dim3(grid), dim3(256), 0, s, view_of<int32_t>(h->t), count, vertices,
                       blocks, out);
  return last_error();
}

extern "C" lp_status lp_gain_table_move(lp_gain_table* h, int64_t count, const int32_t* vertices, const int32_t* to,
                                        void* stream) {
  clear_error();
  if (!h || count < 0 || (count > 0 && (!vertices || !to))) return LP_EINVAL;
  const int32_t n = h->t.g->n;
  if (count == 0) return LP_OK;
  if (count > n) return LP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = grid_for(count, 256, 65536);
  hipLaunchKernelGGL(k_gt_zero, dim3(1), dim3(64), 0, s, h->bad, (int64_t)1);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_check_moves, dim3(grid), dim3(256), 0, s, vertices, to, count, n, h->t.k, h->t.flag, h->bad);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gt_unflag, dim3(grid), dim3(256), 0, s, vertices, count, n, h->t.flag);
  LP_CHECK_LAUNCH();
  uint32_t bad = 0;
  LP_CHECK(host_flag(h->bad, s, &bad));
  if (bad) return LP_EINVAL;
  hipLaunchKernelGGL(k_gt_prep_moves, dim3(grid), dim3(256), 0, s, vertices, to, count, h->blocks, h->moves,
                     h->bad + 1);
  LP_CHECK_LAUNCH();
  return gt_update(h->t, h->moves, h->bad + 1, count, h->blocks, s);
}

extern "C" lp_status lp_gain_table_info(const lp_gain_table* h, uint64_t* entries, uint64_t* bytes, int64_t* missing,
                                        int64_t* rebuilds) {
  clear_error();
  if (!h) return LP_EINVAL;
  if (entries) *entries = h->t.entries;
  if (bytes) *bytes = h->t.bytes;
  uint32_t c[4] = {0, 0, 0, 0};
  if ((missing || rebuilds) && h->t.cnt) {
    LP_CHECK_HIP(hipMemcpyAsync(c, h->t.cnt, sizeof(c), hipMemcpyDeviceToHost, h->stream));
    LP_CHECK_HIP(hipStreamSynchronize(h->stream));
  }
  if (missing) *missing = c[1];
  if (rebuilds) *rebuilds = c[2];
  return LP_OK;
}

extern "C" void lp_gain_table_free(lp_gain_table* h) {
  if (!h) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(h->device);
  gt_release(&h->t, h->stream);
  for (void* p : {(void*)h->blocks, (void*)h->moves, (void*)h->bad})
    if (p) cache_free(p, h->stream);
  (void)hipSetDevice(cur);
  delete h;
}
