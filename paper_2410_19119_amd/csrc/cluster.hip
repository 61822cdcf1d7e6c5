// Size-constrained label-propagation clustering (Section IV-A), one
// synchronous round at a time:
//   rating   - every vertex rates the clusters of its neighbours against the
//              round's snapshot (labels C, cluster weights W) and proposes its
//              best feasible move. Degree buckets pick the kernel, following
//              the paper's two-phase split (Section IV-A2): one lane per
//              vertex, one wavefront per vertex, one workgroup per vertex
//              (all with LDS rating tables: phase one), and a chunk-parallel
//              hub path for the highest degrees (phase two);
//   accept   - proposals are gathered in vertex order, radix-sorted by
//              (target, gain descending) and admitted per target while the
//              running weight fits under the cap;
//   apply    - admitted vertices move; W is updated with integer atomics.
#include <string.h>

#include <algorithm>
#include <memory>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "decode.h"
#include "gain.h"
#include "graph.h"
#include "reorder.h"

namespace lp {

namespace {

struct RoundCtx {
  GraphView g;
  const int32_t* C;  // labels of the snapshot
  const int64_t* W;  // cluster weights of the snapshot
  int64_t cap;
  uint64_t seed;
  uint32_t round;
  int32_t* ptgt;     // proposal target per vertex, -1 = none
  int64_t* pgain;    // proposal gain per vertex
  // rating on a degree-ordered copy (reorder.h): original vertex of every
  // vertex of the copy, where its proposal is written (labels hold original
  // cluster IDs); nullptr = not reordered
  const int32_t* pmap;
  const uint32_t* done;
  // batches of graphs (disjoint union): graph of each vertex, first vertex,
  // cap and seed of each graph; gid == nullptr for a single graph
  const int32_t* gid;
  const int32_t* gbase;
  const int64_t* gcap;
  const uint64_t* gseed;
  // edge visits other than rating (C then holds the labels for a cut, the
  // fine -> coarse map for contraction records)
  const uint64_t* rbase;    // records: first record of every coarse vertex
  const uint64_t* voff;     // records: slice of every fine vertex in its coarse vertex's region
  Rec* rec;                 // records: output, {coarse neighbour or -1, weight} per fine edge
  unsigned long long* cut;  // cut: accumulator of the weights of edges between clusters
  // records: each vertex's edges to one coarse neighbour as one record with
  // their summed weight (one of them; the others -1), set where every summed
  // weighted degree fits 32 bits
  int32_t rec_sum;
};

// What an edge visit computes: ratings and proposals, the cut, or the
// contraction records.
constexpr int kModeRate = 0, kModeCut = 1, kModeRec = 2;

// Cap, seed and label offset that apply to vertex u: a graph of a batch keeps
// its own cap and seed, and its tie-break keys use labels local to the graph,
// so every graph gets exactly the labels it would get alone.
struct VParams {
  int64_t cap;
  uint64_t seed;
  int32_t base;
};

__device__ __forceinline__ VParams vparams(const RoundCtx& x, int32_t u) {
  if (!x.gid) return VParams{x.cap, x.seed, 0};
  const int32_t g = x.gid[u];
  return VParams{x.gcap[g], x.gseed[g], x.gbase[g]};
}

__device__ __forceinline__ uint64_t cluster_key(const RoundCtx& x, const VParams& p, int32_t c) {
  return tiebreak_key(p.seed, x.round, (uint32_t)(c - p.base));
}

// Per listed vertex, built once per call: (vertex, degree, byte position of
// its first code [compressed] or first edge [plain]) and the length of the
// code bytes (compressed only).
struct VDesc {
  const int4* d;      // {u, deg, pos_lo, pos_hi}
  const uint32_t* len;
  const uint32_t* num;  // interval-coded graphs: VarInts in the vertex's code bytes
};

__device__ __forceinline__ uint64_t vd_pos(const int4 v) {
  return (uint64_t)(uint32_t)v.z | ((uint64_t)(uint32_t)v.w << 32);
}

// Slot of vertex u's proposal: its original ID when rating a reordered copy.
__device__ __forceinline__ int32_t prop_slot(const RoundCtx& x, int32_t u) { return x.pmap ? x.pmap[u] : u; }

// Writes vertex u's proposal. On a reordered copy the slots were reset to
// "none" before the round and only proposals are written (scattered writes
// to the original vertices cost more than the coalesced ones of the copy).
__device__ __forceinline__ void emit(const RoundCtx& x, int32_t u, const Cand& best, int64_t own) {
  const int32_t pu = prop_slot(x, u);
  if (best.c >= 0 && best.r > own) {
    x.ptgt[pu] = best.c;
    x.pgain[pu] = best.r - own;
  } else if (!x.pmap) {
    x.ptgt[pu] = -1;
  }
}

// Candidate update with lazy feasibility: the cluster weight is only read
// when the candidate would beat the current best.
__device__ __forceinline__ void consider(const RoundCtx& x, const VParams& p, int32_t c, int64_t r, int64_t wu,
                                         Cand& best) {
  if (r < best.r) return;
  Cand cd{r, cluster_key(x, p, c), c};
  if (cand_better(cd, best) && x.W[c] + wu <= p.cap) best = cd;
}

// ------------------------------------------------------- lane per vertex --
template <bool COMP, int MODE = kModeRate, bool ITV = false>
__global__ __launch_bounds__(256) void k_rate_lane(RoundCtx x, VDesc vd, int32_t cnt) {
  if (*x.done) return;
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if constexpr (MODE == kModeCut) {
    __shared__ unsigned long long red[4];
    unsigned long long c = 0;
    if (i < cnt) {
      const int4 v4 = vd.d[i];
      const int32_t u = v4.x, d = v4.y;
      const int32_t own_c = x.C[u];
      uint64_t pos = vd_pos(v4);
      int32_t v = 0, w = 0;
      LaneDec dec;
      if constexpr (ITV) dec.init(x.g, u, pos);
      for (int k = 0; k < d; ++k) {
        if constexpr (ITV) {
          dec.next(v, w);
        } else if constexpr (COMP) {
          const uint64_t code = varint_read(x.g.bytes, pos);
          v = (k == 0) ? u + (int32_t)unzigzag(code) : v + (int32_t)code;
          if (x.g.weighted) w = (k == 0 ? 0 : w) + (int32_t)unzigzag(varint_read(x.g.bytes, pos));
          else w = 1;
        } else {
          v = x.g.adjncy[pos + k];
          w = x.g.adjwgt ? x.g.adjwgt[pos + k] : 1;
        }
        if (x.C[v] != own_c) c += (unsigned long long)w;
      }
    }
    c = block_reduce_add<256, unsigned long long>(c, red);
    if (threadIdx.x == 0 && c) atomicAdd(x.cut, c);
    return;
  }
  if (i >= cnt) return;
  const int4 v4 = vd.d[i];
  const int32_t u = v4.x;
  const int32_t d = v4.y;
  int32_t lab[kMaxLane];
  int32_t wt[kMaxLane];
  if constexpr (ITV) {
    LaneDec dec;
    dec.init(x.g, u, vd_pos(v4));
#pragma unroll
    for (int k = 0; k < kMaxLane; ++k) {
      lab[k] = -1;
      wt[k] = 0;
      if (k < d) {
        int32_t v, w;
        dec.next(v, w);
        lab[k] = x.C[v];
        wt[k] = w;
      }
    }
  } else if constexpr (COMP) {
    uint64_t pos = vd_pos(v4);
    int32_t v = 0, w = 0;
#pragma unroll
    for (int k = 0; k < kMaxLane; ++k) {
      lab[k] = -1;
      wt[k] = 0;
      if (k < d) {
        const uint64_t code = varint_read(x.g.bytes, pos);
        v = (k == 0) ? u + (int32_t)unzigzag(code) : v + (int32_t)code;
        if (x.g.weighted) w = (k == 0 ? 0 : w) + (int32_t)unzigzag(varint_read(x.g.bytes, pos));
        else w = 1;
        lab[k] = x.C[v];
        wt[k] = w;
      }
    }
  } else {
    const uint64_t b = vd_pos(v4);
#pragma unroll
    for (int k = 0; k < kMaxLane; ++k) {
      lab[k] = -1;
      wt[k] = 0;
      if (k < d) {
        lab[k] = x.C[x.g.adjncy[b + k]];
        wt[k] = x.g.adjwgt ? x.g.adjwgt[b + k] : 1;
      }
    }
  }
  const int32_t own_c = x.C[u];
  if constexpr (MODE == kModeRec) {
    Rec* r = x.rec + x.rbase[own_c] + x.voff[prop_slot(x, u)];
    if (x.rec_sum) {
      // the first edge to each coarse neighbour carries the sum of the
      // vertex's edges to it, the others become empty records
#pragma unroll
      for (int k = 0; k < kMaxLane; ++k) {
        if (k >= d) continue;
        const int32_t c = lab[k];
        bool first = c != own_c;
#pragma unroll
        for (int j = 0; j < k; ++j) first &= lab[j] != c;
        int32_t sum = 0;
#pragma unroll
        for (int j = k; j < kMaxLane; ++j) sum += lab[j] == c ? wt[j] : 0;
        r[k] = first ? Rec{c, sum} : Rec{-1, 0};
      }
    } else {
#pragma unroll
      for (int k = 0; k < kMaxLane; ++k)
        if (k < d) r[k] = Rec{lab[k] == own_c ? -1 : lab[k], wt[k]};
    }
    return;
  }
  const int64_t wu = vweight(x.g, u);
  const VParams vp = vparams(x, u);
  int64_t own = 0;
#pragma unroll
  for (int k = 0; k < kMaxLane; ++k) own += (lab[k] == own_c) ? wt[k] : 0;
  Cand best = cand_none();
#pragma unroll
  for (int k = 0; k < kMaxLane; ++k) {
    const int32_t c = lab[k];
    bool first = (c >= 0) && (c != own_c);
#pragma unroll
    for (int j = 0; j < k; ++j) first &= (lab[j] != c);
    if (first) {
      int64_t r = 0;
#pragma unroll
      for (int j = k; j < kMaxLane; ++j) r += (lab[j] == c) ? wt[j] : 0;
      consider(x, vp, c, r, wu, best);
    }
  }
  emit(x, u, best, own);
}

// ------------------------------------------- LDS rating table (phase one) --
template <typename V>
__device__ __forceinline__ void lds_add(V* p, V w) {
  if constexpr (sizeof(V) == 8) atomicAdd((unsigned long long*)p, (unsigned long long)w);
  else atomicAdd((int*)p, (int)w);
}

__host__ __device__ __forceinline__ uint32_t ceil_log2(uint32_t x) {
  uint32_t k = 0;
  while ((1u << k) < x) ++k;
  return k;
}

// ------------------------------------ edge-balanced tiles (phase one) -----
// Vertices of a tile bucket are cut, in bucket order, into tiles of at most
// E neighbours and VT vertices. One workgroup rates a whole tile, so that
// the loads of each step are independent of one another:
//   1. the tile's code bytes are copied to LDS as aligned dwords; bytes of a
//      dword outside a vertex's codes are set to 0, so each of them decodes
//      as one extra (ignored) number;
//   2. every thread takes a contiguous run of dwords and extracts the numbers
//      that end in it from an 8-byte register window (a VarInt has at most
//      five bytes), placing them by a prefix count of terminators;
//   3. every thread takes a contiguous slice of the tile's neighbours; a
//      segmented prefix sum (segments = vertices) turns gaps and weight
//      differences into IDs and weights, and all neighbour labels are
//      fetched at once;
//   4. each vertex owns a region of 1.5 * deg + 1 slots of an LDS hash table
//      (aliasing the bytes and numbers of steps 1-2) in which its ratings
//      are summed;
//   5. a selection group (a wavefront, or the whole workgroup for tiles of
//      very few vertices) walks a vertex's slots once: own rating and best
//      other cluster by (rating desc, tie-break key asc), reduced across the
//      group; the winner is checked against the cap, and only vertices whose
//      winner is full repeat the walk with the cap applied to every
//      candidate that beats the own rating.
template <int NT, int E, int VT>
struct TileCfg {
  static constexpr int kThreads = NT;
  static constexpr int kEdges = E;
  static constexpr int kVerts = VT;
  static constexpr int kItems = E / NT;
  static constexpr int kSlots = E + E / 2 + VT;
  static constexpr int kSelGroup = VT > 8 ? kWave : NT;  // threads per selected vertex
};

// Waves per SIMD a tile kernel is compiled for: the small tiles' rating of a
// compressed graph is capped at 80 registers, so six workgroups share a CU
// (as many as their LDS allows) to hide the latency of their gathers and
// barriers; other instances keep the compiler's choice.
template <class T, int MODE, bool COMP>
constexpr int tile_waves_per_eu() {
  return T::kThreads == 256 && MODE == kModeRate && COMP ? 6 : 1;
}
using TileSmall = TileCfg<256, 2048, 80>;
using TileLarge = TileCfg<512, 4096, 4>;
constexpr int kTileSeg = 128;  // vertices walked by one thread of the tiling pass
constexpr int kTileGrab = 8;   // tiles taken per atomic of a hand-out counter
constexpr int kTileMaxDeg = 2048;  // largest degree of the small-tile bucket (default and bound of t_tile)

template <int NT, int VT>
struct TileShared {
  int32_t u[VT];
  int32_t own_c[VT];
  int32_t wu[VT];
  int32_t best_c[VT];
  uint64_t pos[VT];  // compressed: byte of the first code; plain: first edge
  uint32_t len[VT];  // compressed: code bytes
  uint32_t ebase[VT + 1];
  uint32_t dwbase[VT + 1];
  uint32_t rstart[VT + 1];  // index of the vertex's first real number
  uint32_t tbase[VT + 1];
  int64_t own_r[VT];
  int64_t gain[VT];
  VParams vp;  // the tile's graph (tiles never span two graphs of a batch)
  uint32_t max_nsl;  // most table slots of one vertex of the tile
  uint64_t rb[VT];  // records: first record of every vertex
  unsigned long long red_u[NT / kWave];
  int32_t scan[NT / kWave];
  int32_t scan2[NT / kWave];
  Cand cb[NT / kWave];
  int64_t red[NT / kWave];
  uint32_t seg_flags;
  uint32_t any_redo;
  uint32_t next;  // tile handed to the workgroup
};

// LDS layout of a tile workgroup: region A holds the staged bytes followed by
// the decoded numbers, and later the rating table (keys, then values).
struct TileLayout {
  uint32_t table_bytes;  // kSlots * (4 + sizeof(V))
  uint32_t nums_off;     // byte offset of the numbers in region A
  uint32_t stage_bytes;  // staged-byte budget of a tile
  uint32_t abytes;       // size of region A
};

template <class T, typename V>
__host__ __device__ inline TileLayout tile_layout(bool comp, bool weighted) {
  TileLayout L;
  const uint32_t per = weighted ? 2u : 1u;
  L.table_bytes = (uint32_t)T::kSlots * (4u + (uint32_t)sizeof(V));
  // numbers: at most per * E VarInts of the neighbours, one interval count per
  // vertex of an interval-coded graph, and up to six zero bytes around each
  // vertex's codes
  const uint32_t nums = comp ? (per * T::kEdges + 7u * T::kVerts) * 4u : 0u;
  // any single vertex of the bucket must fit: <= 5 bytes per number; the
  // staging area later holds the interval table of an interval-coded tile
  const uint32_t worst = comp ? 5u * per * T::kEdges + 16u : 0u;
  const uint32_t itv = comp ? (2u * T::kVerts + 2u + 2u * ((uint32_t)T::kEdges / 3u + 1u)) * 4u : 0u;
  uint32_t sb = L.table_bytes > nums ? L.table_bytes - nums : 0u;
  if (sb < worst) sb = worst;
  if (sb < itv) sb = itv;
  sb = (sb + 15u) & ~15u;
  L.stage_bytes = comp ? sb : 0u;
  L.nums_off = L.stage_bytes;
  L.abytes = L.stage_bytes + nums;
  if (L.abytes < L.table_bytes) L.abytes = L.table_bytes;
  L.abytes = (L.abytes + 15u) & ~15u;
  return L;
}

// Index i in [0, cnt) with base[i] <= x < base[i + 1].
__device__ __forceinline__ int32_t tile_find(const uint32_t* base, int32_t cnt, uint32_t x) {
  int32_t lo = 0, hi = cnt;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (base[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t tile_slots(uint32_t d) { return d + (d >> 1) + 1; }

// Adds w to slot q of the rating table.
template <typename V>
__device__ __forceinline__ void tile_add(V* vals, uint32_t q, V w) {
  if constexpr (sizeof(V) == 2) {
    atomicAdd(reinterpret_cast<unsigned*>(vals) + (q >> 1), (unsigned)(uint16_t)w << ((q & 1u) * 16u));
  } else {
    lds_add(&vals[q], w);
  }
}

// A thread's ITEMS records (cluster nb[k], weight wt[k] of vertex vi[k]; vi[k]
// < 0 skips) into the LDS table, the vertex's slots [base, base + size) given
// by span(vi): every record's first slot is computed, then the first probes
// of all records are issued together (independent LDS atomics), then the few
// that collided walk on. With CLAIM, qo[k] receives record k's slot and bit k
// of *claim is set if record k put its cluster into the table (exactly one
// record per distinct cluster of a vertex does).
template <int ITEMS, typename V, class Span, bool CLAIM = false>
__device__ __forceinline__ void tile_insert_all(int32_t* keys, V* vals, const int32_t* vi, const int32_t* nb,
                                                const int32_t* wt, Span span, uint32_t* qo = nullptr,
                                                uint32_t* claim = nullptr) {
  uint32_t q[ITEMS], b[ITEMS], sz[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    span(vi[k] < 0 ? 0 : vi[k], b[k], sz[k]);
    q[k] = b[k] + __umulhi(slot_hash((uint32_t)nb[k]), sz[k]);
  }
  int32_t old[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    old[k] = kEmpty;
    if (vi[k] >= 0) old[k] = atomicCAS(&keys[q[k]], kEmpty, nb[k]);
  }
  uint32_t cl = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    if (vi[k] < 0) continue;
    bool mine = old[k] == kEmpty;
    if (old[k] != kEmpty && old[k] != nb[k]) {
      uint32_t h = q[k] - b[k];
      while (true) {
        if (++h == sz[k]) h = 0;
        const int32_t o = atomicCAS(&keys[b[k] + h], kEmpty, nb[k]);
        if (o == kEmpty || o == nb[k]) {
          mine = o == kEmpty;
          break;
        }
      }
      q[k] = b[k] + h;
    }
    tile_add<V>(vals, q[k], (V)wt[k]);
    if constexpr (CLAIM) {
      qo[k] = q[k];
      cl |= (mine ? 1u : 0u) << k;
    }
  }
  if constexpr (CLAIM) *claim = cl;
}

// Segmented scan over the workgroup of (head, s, s2): a head restarts the
// sums. Gives the exclusive prefix of this thread.
template <int NT>
__device__ __forceinline__ void tile_seg_scan(bool head, int32_t s, int32_t s2, int32_t* sm, int32_t* sm2,
                                             uint32_t* smf, int32_t& ex, int32_t& ex2) {
  const int lane = lane_id();
  int32_t f = head ? 1 : 0;
  // inclusive segmented scan of the wave with DPP moves (as in
  // wave_incl_scan_add_i32): a lane adds what reaches it only while it has
  // not seen a head, and takes over the head flag
  auto step = [&](int32_t fu, int32_t su, int32_t su2) {
    if (!f) {
      s += su;
      s2 += su2;
    }
    f |= fu;
  };
  step(dpp_i32<0x111>(f), dpp_i32<0x111>(s), dpp_i32<0x111>(s2));
  step(dpp_i32<0x112>(f), dpp_i32<0x112>(s), dpp_i32<0x112>(s2));
  step(dpp_i32<0x114>(f), dpp_i32<0x114>(s), dpp_i32<0x114>(s2));
  step(dpp_i32<0x118>(f), dpp_i32<0x118>(s), dpp_i32<0x118>(s2));
  step(dpp_i32<0x142, 0xa>(f), dpp_i32<0x142, 0xa>(s), dpp_i32<0x142, 0xa>(s2));
  step(dpp_i32<0x143, 0xc>(f), dpp_i32<0x143, 0xc>(s), dpp_i32<0x143, 0xc>(s2));
  // exclusive values: one lane up (lane 0 gets zeros)
  const int32_t ef = dpp_i32<0x138>(f), es = dpp_i32<0x138>(s), es2 = dpp_i32<0x138>(s2);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane == kWave - 1) {
    sm[w] = s;
    sm2[w] = s2;
    atomicOr(smf, (uint32_t)f << w);
  }
  __syncthreads();
  int32_t cs = 0, cs2 = 0;
  const uint32_t flags = *smf;
  for (int k = 0; k < w; ++k) {
    if ((flags >> k) & 1u) {
      cs = sm[k];
      cs2 = sm2[k];
    } else {
      cs += sm[k];
      cs2 += sm2[k];
    }
  }
  ex = ef ? es : cs + es;
  ex2 = ef ? es2 : cs2 + es2;
}

// Interval-coded segments (vertices of a tile, code streams of a hub piece):
// the per-workgroup table of intervals, built from the numbers of step 2 in
// the staging area that step 2 has finished with. Segment i's numbers start
// at rstart[i] with its interval count k_i, then its (zigzag(x - u), l - 3)
// pairs. The table gives every interval its start ID and the number of the
// segment's neighbours in its earlier intervals; L[i] = all of segment i's
// interval neighbours, which come first in its decoding order.
struct ItvTable {
  uint32_t* base;   // nseg + 1: first interval of each segment
  uint32_t* L;      // nseg: interval neighbours of each segment
  int32_t* start;   // per interval: first neighbour ID
  uint32_t* cum;    // per interval: neighbours of the segment's earlier intervals
};

template <int NT, int MAXSEG, int MAXITV>
__device__ __forceinline__ ItvTable itv_table(uint32_t* area, const uint32_t* nums, const uint32_t* rstart,
                                              const uint32_t* ebase, const int32_t* seg_u, int32_t nseg,
                                              int32_t* scan_sm, int32_t* scan_sm2, uint32_t* seg_flags) {
  ItvTable t;
  t.base = area;
  t.L = area + (MAXSEG + 1);
  t.start = (int32_t*)(area + 2 * MAXSEG + 2);
  t.cum = area + 2 * MAXSEG + 2 + MAXITV;
  const int tid = threadIdx.x;
  uint32_t kk = 0;
  if (tid < nseg && ebase[tid + 1] > ebase[tid]) kk = nums[rstart[tid]];  // empty segments have no count
  int32_t tot;
  const int32_t inc = block_incl_scan_add<NT, int32_t>((int32_t)kk, scan_sm, &tot);
  if (tid < nseg) t.base[tid] = (uint32_t)(inc - (int32_t)kk);
  if (tid == 0) {
    t.base[nseg] = (uint32_t)tot;
    *seg_flags = 0;
  }
  __syncthreads();
  const uint32_t K = (uint32_t)tot;
  const uint32_t Q = (K + NT - 1) / NT;
  const uint32_t q0 = min(K, (uint32_t)tid * Q), q1 = min(K, q0 + Q);
  int32_t run = 0;
  bool anyh = false;
  uint32_t first_head = q1;
  int32_t i = q0 < K ? tile_find(t.base, nseg, q0) : 0;
  for (uint32_t q = q0; q < q1; ++q) {
    while (q >= t.base[i + 1]) ++i;
    const uint32_t j = q - t.base[i];
    const uint32_t b = rstart[i] + 1u + 2u * j;
    t.start[q] = seg_u[i] + unzigzag32(nums[b]);
    if (j == 0) {
      if (!anyh) first_head = q;
      anyh = true;
      run = 0;
    }
    t.cum[q] = (uint32_t)run;
    run += (int32_t)nums[b + 1] + 3;
  }
  int32_t ex, ex2;
  tile_seg_scan<NT>(anyh, run, 0, scan_sm, scan_sm2, seg_flags, ex, ex2);
  for (uint32_t q = q0; q < first_head; ++q) t.cum[q] += (uint32_t)ex;
  __syncthreads();
  if (tid < nseg) {
    const uint32_t b0 = t.base[tid], b1 = t.base[tid + 1];
    uint32_t L = 0;
    if (b1 > b0) L = t.cum[b1 - 1] + nums[rstart[tid] + 2u * (b1 - b0)] + 3u;
    t.L[tid] = L;
  }
  if (tid == 0) *seg_flags = 0;
  __syncthreads();
  return t;
}

// Neighbour `loc` of segment i of an interval-coded tile or piece, as one
// item of the segmented prefix sums: the ID (absolute inside intervals, a
// head; else the first residual restarts from base_v, later ones are gaps)
// and the weight difference (the chain restarts at the segment's first
// neighbour).
__device__ __forceinline__ void itv_item(const ItvTable& t, const uint32_t* nums, uint32_t rs, int32_t i, uint32_t loc,
                                         int32_t base_v, bool weighted, int32_t& dv, int32_t& dw, bool& hid) {
  const uint32_t b0 = t.base[i], b1 = t.base[i + 1];
  const uint32_t L = t.L[i];
  const uint32_t wb = rs + 1u + 2u * (b1 - b0);  // first interval weight (or residual code)
  if (loc < L) {
    uint32_t lo = b0, hi = b1;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (t.cum[mid] <= loc) lo = mid;
      else hi = mid;
    }
    dv = t.start[lo] + (int32_t)(loc - t.cum[lo]);
    hid = true;
    dw = weighted ? unzigzag32(nums[wb + loc]) : 0;
  } else {
    const uint32_t r = loc - L;
    const uint32_t ci = wb + (weighted ? L + 2u * r : r);
    const uint32_t code = nums[ci];
    hid = r == 0;
    dv = hid ? base_v + unzigzag32(code) : (int32_t)code;
    dw = weighted ? unzigzag32(nums[ci + 1]) : 0;
  }
}

// Value of the VarInt whose last byte is byte b (4..7) of the 8-byte window
// w (bytes 0..3 = previous dword, 4..7 = current); term = terminator bits
// (bit 7 of every byte with its top bit clear) of the window.
__device__ __forceinline__ uint32_t window_value(uint64_t w, uint64_t term, uint32_t b) {
  const uint64_t below = term & ((1ull << (8 * b)) - 1ull);
  const uint32_t s = below ? (uint32_t)((63 - __clzll(below)) >> 3) + 1u : (b >= 4 ? b - 4 : 0u);
  const uint32_t len = min(b - s + 1u, 5u);  // a longer run (a malformed stream) reads five bytes
  uint32_t y = (uint32_t)(w >> (8 * s));
  if (len < 4) y &= (1u << (8 * len)) - 1u;
  // the 7-bit groups of the first four bytes, then the fifth's low bits
  uint32_t v = (y & 0x7Fu) | ((y >> 1) & 0x3F80u) | ((y >> 2) & 0x1FC000u) | ((y >> 3) & 0xFE00000u);
  if (len == 5) v |= (uint32_t)((w >> (8 * (s + 4))) & 0x7Full) << 28;
  return v;
}

// Step 2 of a staged code stream (Dt dwords in A32): the numbers in stream
// order, one thread per run of consecutive dwords. With POS (gap-only
// format) only the byte at which every number ends is stored, and
// number_at reads a number's value when it is needed; otherwise the values
// themselves (interval-coded streams, whose pairs the interval table reads).
template <int NT, bool POS>
__device__ __forceinline__ void stage_numbers(const uint32_t* A32, uint32_t Dt, uint32_t* nums, int32_t* scan_sm) {
  const uint32_t Q = (Dt + NT - 1) / NT;
  const uint32_t j0 = min(Dt, threadIdx.x * Q), j1 = min(Dt, j0 + Q);
  int32_t cnt = 0;
  for (uint32_t j = j0; j < j1; ++j) cnt += __popc(~A32[j] & 0x80808080u);
  int32_t tot;
  uint32_t idx = (uint32_t)(block_incl_scan_add<NT, int32_t>(cnt, scan_sm, &tot) - cnt);
  uint32_t prev = j0 > 0 ? A32[j0 - 1] : 0u;
  for (uint32_t j = j0; j < j1; ++j) {
    const uint32_t cur = A32[j];
    if constexpr (POS) {
      const uint32_t t = ~cur & 0x80808080u;
#pragma unroll
      for (uint32_t b = 0; b < 4; ++b)
        if ((t >> (8 * b + 7)) & 1u) nums[idx++] = 4u * j + b;
    } else {
      const uint64_t w = ((uint64_t)cur << 32) | prev;
      const uint64_t term = ~w & 0x8080808080808080ull;
      uint32_t tc = (uint32_t)(term >> 32);
      while (tc) {
        const uint32_t b = 4u + (((uint32_t)__ffs(tc) - 1u) >> 3);
        tc &= tc - 1u;
        nums[idx++] = window_value(w, term, b);
      }
    }
    prev = cur;
  }
  __syncthreads();
}

// Value of number k of a staged stream whose end bytes stage_numbers<POS>
// stored in ends[]: it starts after number k - 1 ends and runs to the first
// byte with the top bit clear (at most five bytes: if none of the first four
// ends it, the fifth does).
__device__ __forceinline__ uint32_t number_at(const uint32_t* A32, const uint32_t* ends, uint32_t k) {
  const uint32_t s = k ? ends[k - 1] + 1u : 0u;
  const uint32_t lo = A32[s >> 2], hi = A32[(s >> 2) + 1];
  uint32_t y = __builtin_amdgcn_alignbyte(hi, lo, s & 3u);  // bytes s .. s + 3
  const uint32_t t = ~y & 0x80808080u;
  y &= t ^ (t - 1u);  // up to the first byte that ends the number
  uint32_t v = (y & 0x7Fu) | (__builtin_amdgcn_ubfe(y, 8, 7) << 7) | (__builtin_amdgcn_ubfe(y, 16, 7) << 14) |
               (__builtin_amdgcn_ubfe(y, 24, 7) << 21);
  if (t == 0u) v |= ((hi >> (8u * (s & 3u))) & 0x7Fu) << 28;
  return v;
}

// DPP move of a 64-bit value (row_shl:n = 0x100 + n: lane i of a row of 16
// gets lane i + n); lanes that receive nothing keep `fill`.
template <int CTRL>
__device__ __forceinline__ int64_t dpp_i64(int64_t v, int64_t fill) {
  const int32_t lo = __builtin_amdgcn_update_dpp((int32_t)fill, (int32_t)v, CTRL, 0xf, 0xf, false);
  const int32_t hi = __builtin_amdgcn_update_dpp((int32_t)(fill >> 32), (int32_t)(v >> 32), CTRL, 0xf, 0xf, false);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int CTRL>
__device__ __forceinline__ Cand dpp_cand(const Cand& x) {
  return Cand{dpp_i64<CTRL>(x.r, -1), (uint64_t)dpp_i64<CTRL>((int64_t)x.key, -1),
              __builtin_amdgcn_update_dpp(-1, x.c, CTRL, 0xf, 0xf, false)};
}

__device__ __forceinline__ Cand readlane_cand(const Cand& x, int l) {
  const int32_t rl = __builtin_amdgcn_readlane((int32_t)x.r, l), rh = __builtin_amdgcn_readlane((int32_t)(x.r >> 32), l);
  const int32_t kl = __builtin_amdgcn_readlane((int32_t)x.key, l);
  const int32_t kh = __builtin_amdgcn_readlane((int32_t)(x.key >> 32), l);
  return Cand{(int64_t)(((uint64_t)(uint32_t)rh << 32) | (uint32_t)rl), ((uint64_t)(uint32_t)kh << 32) | (uint32_t)kl,
              __builtin_amdgcn_readlane(x.c, l)};
}

// Best candidate and sum over groups of G lanes of a wavefront (G = 16 or
// 64), delivered to the group's first lane (the others hold partial
// results): DPP shifts inside rows of 16 lanes (lanes that receive nothing
// see "no candidate" / 0), then for G = 64 the rows' first lanes read out.
template <int G>
__device__ __forceinline__ Cand group_best_lanes(Cand x) {
  static_assert(G == 16 || G == kWave, "groups of 16 lanes or the wavefront");
  auto take = [&](const Cand& y) {
    if (cand_better(y, x)) x = y;
  };
  take(dpp_cand<0x101>(x));
  take(dpp_cand<0x102>(x));
  take(dpp_cand<0x104>(x));
  take(dpp_cand<0x108>(x));
  if constexpr (G == kWave) {
    take(readlane_cand(x, 16));
    take(readlane_cand(x, 32));
    take(readlane_cand(x, 48));
  }
  return x;
}

template <int G>
__device__ __forceinline__ int64_t group_sum_lanes(int64_t v) {
  static_assert(G == 16 || G == kWave, "groups of 16 lanes or the wavefront");
  v += dpp_i64<0x101>(v, 0);
  v += dpp_i64<0x102>(v, 0);
  v += dpp_i64<0x104>(v, 0);
  v += dpp_i64<0x108>(v, 0);
  if constexpr (G == kWave) {
    int64_t t = 0;
#pragma unroll
    for (int l = 16; l < kWave; l += 16)
      t += (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(v >> 32), l) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane((int32_t)v, l));
    v += t;
  }
  return v;
}

// Selection over the tile's vertices by groups of G threads (G lanes of a
// wavefront, or the whole workgroup when G == NT): a group walks one
// vertex's slots. First walk (redo == false): own rating and best other
// cluster by (rating desc, key asc). Capped walk (redo == true), only for the
// vertices marked -2: the best cluster beating the own rating whose weight
// leaves room for the vertex.
template <int G, int NT, typename V, class SH>
__device__ __forceinline__ void tile_select(const RoundCtx& x, const int32_t* keys, const V* vals, SH& sh,
                                            int32_t nv, int tid, bool redo) {
  constexpr int NG = NT / G;
  const int gi = tid / G, gl = tid % G;
  for (int32_t i = gi; i < nv; i += NG) {
    if (redo && sh.best_c[i] != -2) continue;  // uniform across the group
    const uint32_t b0 = sh.tbase[i], b1 = sh.tbase[i + 1];
    const int32_t oc = sh.own_c[i];
    const int64_t own0 = redo ? sh.own_r[i] : 0;
    const int64_t wu = sh.wu[i];
    int64_t own = 0;
    Cand best = cand_none();
    for (uint32_t q = b0 + gl; q < b1; q += G) {
      const int32_t c = keys[q];
      if (c == kEmpty) continue;
      const int64_t r = (int64_t)vals[q];
      if (c == oc) {
        own = r;
        continue;
      }
      if (r < best.r || (redo && r <= own0)) continue;
      const Cand cd{r, cluster_key(x, sh.vp, c), c};
      if (cand_better(cd, best) && (!redo || x.W[c] + wu <= sh.vp.cap)) best = cd;
    }
    if constexpr (G == NT && NT > kWave) {
      best = block_best<NT>(best, sh.cb);
      own = block_reduce_add<NT, int64_t>(own, sh.red);
    } else {
      best = group_best_lanes<G>(best);
      own = group_sum_lanes<G>(own);
    }
    if (gl == 0) {
      if (!redo) {
        sh.own_r[i] = own;
        sh.best_c[i] = best.r > own ? best.c : -1;
        sh.gain[i] = best.r - own;
      } else {
        const int32_t pu = prop_slot(x, sh.u[i]);
        if (best.c >= 0) {
          x.ptgt[pu] = best.c;
          x.pgain[pu] = best.r - own0;
        } else if (!x.pmap) {
          x.ptgt[pu] = -1;
        }
      }
    }
  }
}

template <class T, typename V, bool COMP, int MODE = kModeRate, bool ITV = false>
__global__ __launch_bounds__(T::kThreads) __attribute__((amdgpu_waves_per_eu(tile_waves_per_eu<T, MODE, COMP>())))
void k_rate_tile(RoundCtx x, VDesc vd, const int32_t* tiles,
                                                           const uint32_t* ntiles_p, uint32_t* ctr, TileLayout L) {
  constexpr int NT = T::kThreads, VT = T::kVerts, ITEMS = T::kItems, SG = T::kSelGroup;
  constexpr int NSG = NT / SG;  // selection groups per workgroup
  extern __shared__ __align__(16) uint8_t smem_raw[];
  if (*x.done) return;
  const int tid = threadIdx.x;
  const bool weighted = x.g.weighted;
  const uint32_t per = weighted ? 2u : 1u;
  uint8_t* A = smem_raw;
  uint32_t* A32 = (uint32_t*)A;
  int32_t* keys = (int32_t*)A;
  V* vals = (V*)(A + (size_t)T::kSlots * 4);
  uint32_t* nums = (uint32_t*)(A + L.nums_off);
  TileShared<NT, VT>& sh = *(TileShared<NT, VT>*)(A + L.abytes);
  const int sgi = tid / SG;           // selection group of this thread
  const int sl = tid % SG;            // lane within the selection group

  // Tiles are handed out at run time, kTileGrab at a time (a device-wide
  // atomic costs about as much as the setup of a tile, and all workgroups
  // contend for few counters): the workgroups of one XCD first take tiles of
  // their own eighth of the list (one counter per eighth), then help with the
  // other eighths, so that workgroups that become resident late (the kernel
  // may share the device with the other rating paths) take fewer tiles.
  const uint32_t T_ = *ntiles_p;
  const uint32_t xcd = blockIdx.x & 7u;
  for (uint32_t k8 = 0; k8 < 8; ++k8) {
    const uint32_t xr = (xcd + k8) & 7u;
    const uint32_t lo = (uint32_t)(((uint64_t)T_ * xr) >> 3), hi = (uint32_t)(((uint64_t)T_ * (xr + 1)) >> 3);
    uint32_t t = hi, tend = hi;
    while (true) {
      if (t >= tend) {
        if (tid == 0) sh.next = lo + atomicAdd(&ctr[xr], (uint32_t)kTileGrab);
        __syncthreads();
        t = sh.next;
        __syncthreads();
        if (t >= hi) break;
        tend = min(hi, t + (uint32_t)kTileGrab);
      }
      const uint32_t tcur = t++;
      const int32_t t0 = tiles[tcur];
      const int32_t nv = tiles[tcur + 1] - t0;
      // 0. vertex descriptors and bases
      uint32_t d = 0, ndw = 0, nnum = 0, nsl = 0;
      if (tid < nv) {
        const int4 v4 = vd.d[t0 + tid];
        const int32_t u = v4.x;
        d = (uint32_t)v4.y;
        const uint64_t pos = vd_pos(v4);
        sh.u[tid] = u;
        sh.own_c[tid] = x.C[u];
        sh.wu[tid] = x.g.vwgt ? x.g.vwgt[u] : 1;
        sh.pos[tid] = pos;
        if constexpr (MODE == kModeRec) sh.rb[tid] = x.rbase[sh.own_c[tid]] + x.voff[prop_slot(x, u)];
        if constexpr (COMP) {
          const uint32_t len = vd.len[t0 + tid];
          const uint32_t pre = (uint32_t)(pos & 3u);
          ndw = (pre + len + 3u) >> 2;
          // numbers from the vertex's dwords: its VarInts plus one per zero byte
          nnum = (ITV ? vd.num[t0 + tid] : per * d) + 4u * ndw - len;
          sh.len[tid] = len;
        }
        nsl = tile_slots(d);
      }
      {
        int32_t tot1, tot2;
        const int32_t p1 = (int32_t)(d | (ndw << 16));
        const int32_t p2 = (int32_t)(nnum | (nsl << 16));
        const int32_t i1 = block_incl_scan_add<NT, int32_t>(p1, sh.scan, &tot1);
        const int32_t i2 = block_incl_scan_add<NT, int32_t>(p2, sh.scan2, &tot2);
        const uint32_t e1 = (uint32_t)(i1 - p1), e2 = (uint32_t)(i2 - p2);
        if (tid < nv) {
          sh.ebase[tid] = e1 & 0xFFFFu;
          sh.dwbase[tid] = e1 >> 16;
          sh.rstart[tid] = (e2 & 0xFFFFu) + (COMP ? (uint32_t)(sh.pos[tid] & 3u) : 0u);
          sh.tbase[tid] = e2 >> 16;
        }
        if (tid == 0) {
          sh.ebase[nv] = (uint32_t)tot1 & 0xFFFFu;
          sh.dwbase[nv] = (uint32_t)tot1 >> 16;
          sh.rstart[nv] = (uint32_t)tot2 & 0xFFFFu;
          sh.tbase[nv] = (uint32_t)tot2 >> 16;
          sh.any_redo = 0;
          sh.seg_flags = 0;
          sh.max_nsl = 0;
          sh.vp = vparams(x, sh.u[0]);
        }
      }
      __syncthreads();
      const uint32_t Et = sh.ebase[nv];
      const uint32_t St = sh.tbase[nv];
      auto tspan = [&](int32_t i, uint32_t& b, uint32_t& sz) {
        b = sh.tbase[i];
        sz = sh.tbase[i + 1] - b;
      };
      if constexpr (COMP) {
        // 1. stage the code bytes: four consecutive dwords per thread (one
        // search for their vertex, four independent loads in flight)
        const uint32_t Dt = sh.dwbase[nv];
        for (uint32_t jb = 4 * tid; jb < Dt; jb += 4 * NT) {
          uint32_t w[4], off[4];
          int32_t vi4[4];
          int32_t i = tile_find(sh.dwbase, nv, jb);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t j = jb + (uint32_t)k;
            vi4[k] = -1;
            w[k] = 0;
            off[k] = 0;
            if (j < Dt) {
              while (j >= sh.dwbase[i + 1]) ++i;
              vi4[k] = i;
              off[k] = 4u * (j - sh.dwbase[i]);
              w[k] = *(const uint32_t*)(x.g.bytes + (sh.pos[i] & ~3ull) + off[k]);
            }
          }
          uint4 o;
          uint32_t* ov = (uint32_t*)&o;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            ov[k] = 0;
            if (vi4[k] < 0) continue;
            const int32_t i2 = vi4[k];
            // bytes [b0, b1) of the vertex's dwords are its codes
            const int32_t b0 = (int32_t)(sh.pos[i2] & 3u), b1 = b0 + (int32_t)sh.len[i2];
            const int32_t lo = min(max(b0 - (int32_t)off[k], 0), 4), hi = min(max(b1 - (int32_t)off[k], 0), 4);
            ov[k] = w[k] & (uint32_t)(((1ull << (8 * hi)) - 1ull) ^ ((1ull << (8 * lo)) - 1ull));
          }
          if (jb + 4 <= Dt) {
            *(uint4*)&A32[jb] = o;
          } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (jb + k < Dt) A32[jb + k] = ov[k];
          }
        }
        __syncthreads();
        // 2. numbers in stream order (gap-only: where each one ends)
        stage_numbers<NT, !ITV>(A32, Dt, nums, sh.scan);
        __syncthreads();
      }
      // 3. neighbour IDs, weights and labels of this thread's slice
      const uint32_t Dd = (Et + NT - 1) / NT;
      const uint32_t e0 = tid * Dd;
      int32_t vi[ITEMS], nb[ITEMS], wt[ITEMS];
      if constexpr (COMP && ITV) {
        // interval-coded: the interval table (in the staging area), then every
        // item's ID and weight difference; IDs restart at every interval
        // neighbour and at the first residual, weights at the vertex's start
        const ItvTable itv = itv_table<NT, VT, T::kEdges / 3 + 1>(A32, nums, sh.rstart, sh.ebase, sh.u, nv, sh.scan,
                                                                    sh.scan2, &sh.seg_flags);
        int32_t i = e0 < Et ? tile_find(sh.ebase, nv, e0) : 0;
        uint32_t hidm = 0, hwm = 0;
        int32_t a = 0, a2 = 0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          const uint32_t e = e0 + k;
          vi[k] = -1;
          nb[k] = 0;
          wt[k] = 1;
          if ((uint32_t)k < Dd && e < Et) {
            while (e >= sh.ebase[i + 1]) ++i;
            vi[k] = i;
            const uint32_t loc = e - sh.ebase[i];
            int32_t dv, dw;
            bool hid;
            itv_item(itv, nums, sh.rstart[i], i, loc, sh.u[i], weighted, dv, dw, hid);
            const bool hw = loc == 0;
            a = hid ? dv : a + dv;
            a2 = hw ? dw : a2 + dw;
            hidm |= (uint32_t)hid << k;
            hwm |= (uint32_t)hw << k;
            nb[k] = a;
            wt[k] = a2;
          }
        }
        int32_t ex, ex2, unused;
        tile_seg_scan<NT>(hidm != 0, a, 0, sh.scan, sh.scan2, &sh.seg_flags, ex, unused);
        __syncthreads();
        if (tid == 0) sh.seg_flags = 0;
        __syncthreads();
        if (weighted) {
          tile_seg_scan<NT>(hwm != 0, a2, 0, sh.scan, sh.scan2, &sh.seg_flags, ex2, unused);
          __syncthreads();
          if (tid == 0) sh.seg_flags = 0;
        }
        const uint32_t fid = hidm ? (uint32_t)__ffs(hidm) - 1u : 32u;
        const uint32_t fw = hwm ? (uint32_t)__ffs(hwm) - 1u : 32u;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          if (vi[k] < 0) continue;
          if ((uint32_t)k < fid) nb[k] += ex;
          if (weighted) {
            if ((uint32_t)k < fw) wt[k] += ex2;
          } else {
            wt[k] = 1;
          }
        }
      } else {
        int32_t i = e0 < Et ? tile_find(sh.ebase, nv, e0) : 0;
        bool any_head = false;
        int32_t s = 0, s2 = 0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          const uint32_t e = e0 + k;
          vi[k] = -1;
          nb[k] = 0;
          wt[k] = 1;
          if ((uint32_t)k < Dd && e < Et) {
            while (e >= sh.ebase[i + 1]) ++i;
            vi[k] = i;
            const uint32_t loc = e - sh.ebase[i];
            if constexpr (COMP) {
              const uint32_t ci = sh.rstart[i] + per * loc;
              const uint32_t code = number_at(A32, nums, ci);
              const bool head = loc == 0;
              const int32_t dv = head ? sh.u[i] + unzigzag32(code) : (int32_t)code;
              const int32_t dw = weighted ? unzigzag32(number_at(A32, nums, ci + 1)) : 0;
              if (head) {
                any_head = true;
                s = dv;
                s2 = dw;
              } else {
                s += dv;
                s2 += dw;
              }
              nb[k] = s;
              wt[k] = s2;
            } else {
              const uint64_t ge = sh.pos[i] + loc;
              nb[k] = x.g.adjncy[ge];
              if (weighted) wt[k] = x.g.adjwgt[ge];
            }
          }
        }
        if constexpr (COMP) {
          int32_t ex, ex2;
          tile_seg_scan<NT>(any_head, s, s2, sh.scan, sh.scan2, &sh.seg_flags, ex, ex2);
          bool before = true;
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) {
            if (vi[k] < 0) continue;
            if (e0 + k == sh.ebase[vi[k]]) before = false;
            if (before) {
              nb[k] += ex;
              wt[k] += ex2;
            }
            if (!weighted) wt[k] = 1;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (vi[k] < 0) continue;
        if ((uint32_t)nb[k] < (uint32_t)x.g.n) nb[k] = x.C[nb[k]];
        else vi[k] = -1;  // unreachable for a valid handle; keeps the gather in bounds
      }
      if constexpr (MODE == kModeCut) {
        unsigned long long c = 0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
          if (vi[k] >= 0 && nb[k] != sh.own_c[vi[k]]) c += (unsigned long long)wt[k];
        c = block_reduce_add<NT, unsigned long long>(c, sh.red_u);
        if (tid == 0 && c) atomicAdd(x.cut, c);
        __syncthreads();
        continue;
      }
      if constexpr (MODE == kModeRec) {
        if (x.rec_sum) {
          // each vertex's edges summed per coarse neighbour in the vertex's
          // table: the edge that put a neighbour into the table carries the
          // sum, the vertex's other edges to it (and to its own coarse
          // vertex) become empty records
          __syncthreads();  // numbers consumed: region A becomes the table
          for (uint32_t q = tid; q < St; q += NT) keys[q] = kEmpty;
          for (uint32_t q = tid; q < St; q += NT) vals[q] = 0;
          __syncthreads();
          int32_t vj[ITEMS];
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) vj[k] = vi[k] >= 0 && nb[k] != sh.own_c[vi[k]] ? vi[k] : -1;
          uint32_t qs[ITEMS], claim = 0;
          tile_insert_all<ITEMS, V, decltype(tspan), true>(keys, vals, vj, nb, wt, tspan, qs, &claim);
          __syncthreads();
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) {
            if (vi[k] < 0) continue;
            const int32_t i = vi[k];
            const uint32_t loc = e0 + k - sh.ebase[i];
            const bool lead = vj[k] >= 0 && ((claim >> k) & 1u);
            x.rec[sh.rb[i] + loc] = lead ? Rec{nb[k], (int32_t)vals[qs[k]]} : Rec{-1, 0};
          }
        } else {
#pragma unroll
          for (int k = 0; k < ITEMS; ++k) {
            if (vi[k] < 0) continue;
            const int32_t i = vi[k];
            const uint32_t loc = e0 + k - sh.ebase[i];
            x.rec[sh.rb[i] + loc] = Rec{nb[k] == sh.own_c[i] ? -1 : nb[k], wt[k]};
          }
        }
        __syncthreads();
        continue;
      }
      __syncthreads();  // numbers consumed: region A becomes the table
      if (tid < nv) atomicMax(&sh.max_nsl, sh.tbase[tid + 1] - sh.tbase[tid]);
      for (uint32_t q = tid; q < St; q += NT) keys[q] = kEmpty;
      for (uint32_t q = tid; q < St; q += NT) vals[q] = 0;
      __syncthreads();
      // 4. ratings
      tile_insert_all<ITEMS, V>(keys, vals, vi, nb, wt, tspan);
      __syncthreads();
      // 5. selection: one walk over the slots of each vertex; tiles of small
      // vertices use 16-lane groups (four vertices per wavefront at a time)
      const bool small_v = SG == kWave && sh.max_nsl <= 256;
      if (small_v) tile_select<16, NT, V>(x, keys, vals, sh, nv, tid, false);
      else tile_select<SG, NT, V>(x, keys, vals, sh, nv, tid, false);
      __syncthreads();
      if (tid < nv) {
        const int32_t u = prop_slot(x, sh.u[tid]);
        const int32_t c = sh.best_c[tid];
        if (c < 0) {
          if (!x.pmap) x.ptgt[u] = -1;
        } else if (x.W[c] + sh.wu[tid] <= sh.vp.cap) {
          x.ptgt[u] = c;
          x.pgain[u] = sh.gain[tid];
        } else {
          sh.best_c[tid] = -2;  // walk again with the cap
          atomicOr(&sh.any_redo, 1u);
        }
      }
      __syncthreads();
      if (sh.any_redo) {
        if (small_v) tile_select<16, NT, V>(x, keys, vals, sh, nv, tid, true);
        else tile_select<SG, NT, V>(x, keys, vals, sh, nv, tid, true);
      }
      __syncthreads();
    }
  }
}

// Greedy tiling of a tile bucket: each thread walks kTileSeg consecutive
// vertices and starts a new tile whenever the next vertex would exceed the
// tile's edge, vertex or staged-byte budget. COUNT: tiles per segment;
// otherwise the first vertex of every tile (and the end sentinel).
template <bool COUNT>
__global__ void k_tile_plan(VDesc vd, int32_t cnt, uint32_t emax, uint32_t vmax, uint32_t bmax, bool comp,
                            const int32_t* gid, uint32_t* counts, const uint32_t* offs, int32_t* tiles) {
  const int64_t sgi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t a = sgi * kTileSeg;
  if (a >= cnt) return;
  const int64_t b = a + kTileSeg < (int64_t)cnt ? a + kTileSeg : (int64_t)cnt;
  uint32_t e = 0, nvv = 0, by = 0, nt = 0;
  int32_t g0 = -1;
  const uint32_t o = COUNT ? 0u : offs[sgi];
  for (int64_t i = a; i < b; ++i) {
    const int4 v4 = vd.d[i];
    const uint32_t d = (uint32_t)v4.y;
    const uint32_t sb = comp ? 4u * ((((uint32_t)v4.z & 3u) + vd.len[i] + 3u) / 4u) : 0u;
    const int32_t gv = gid ? gid[v4.x] : 0;
    if (nvv == 0 || e + d > emax || nvv == vmax || by + sb > bmax || gv != g0) {
      g0 = gv;
      if (!COUNT) tiles[o + nt] = (int32_t)i;
      ++nt;
      e = 0;
      nvv = 0;
      by = 0;
    }
    e += d;
    ++nvv;
    by += sb;
  }
  if (COUNT) counts[sgi] = nt;
  else if (b == cnt) tiles[o + nt] = (int32_t)cnt;
}

// --------------------------------------------------- hub path (phase two) --
// A hub's neighbours are cut into pieces of kHubPiece (four of the format's
// chunks, or, for an unchunked record, runs whose decoder state at the cut
// is recorded once per call). Step H1 rates every piece like a tile: staged
// bytes, register-window VarInt extraction, segmented decode, all label
// gathers at once, summing in an LDS table; the piece then writes its
// distinct (cluster, partial rating) pairs grouped by a hash partition of
// the cluster ID. Step H2 sums each (hub, partition) over the hub's pieces in
// an LDS table and reports the partition's best feasible cluster and the
// hub's own rating if its cluster hashes there. Step H3 combines the
// partitions of a hub.
constexpr int kHubPiece = 4 * LP_CHUNK_LEN;
constexpr int kHubStreams = 4;  // code streams per piece

// Workgroup shape of a piece: threads, neighbours, code streams. Whole hubs
// (kWhole) are rated by one workgroup alone, their table in LDS, without
// partial records: up to sixteen of the format's chunks with 16-bit ratings,
// twelve with 32-bit ones.
template <int NT_, int E_, int NS_, bool WHOLE_>
struct PieceCfg {
  static constexpr int kThreads = NT_;
  static constexpr int kEdges = E_;
  static constexpr int kStreams = NS_;
  static constexpr bool kWhole = WHOLE_;
  static constexpr int kItems = (E_ + NT_ - 1) / NT_;
  static constexpr int kSlots = E_ + E_ / 2 + 16;
};
using PieceHub = PieceCfg<512, kHubPiece, kHubStreams, false>;
using PieceWhole16 = PieceCfg<1024, 16 * LP_CHUNK_LEN, 16, true>;
using PieceWhole32 = PieceCfg<1024, 12 * LP_CHUNK_LEN, 12, true>;
static_assert(PieceHub::kEdges == PieceHub::kStreams * LP_CHUNK_LEN && PieceWhole16::kEdges == PieceWhole16::kStreams * LP_CHUNK_LEN &&
                  PieceWhole32::kEdges == PieceWhole32::kStreams * LP_CHUNK_LEN,
              "a piece holds whole chunks, one stream each");
constexpr int kMaxParts = 1024;
constexpr int kPieceGrab = 4;  // pieces taken per atomic of the hand-out counter
constexpr int kDefaultHubPart = 2048;
constexpr int kMaxSubrounds = 64;  // target partial records per (hub, partition) task
constexpr uint32_t kStreamZig = 0x80000000u;  // first code is zigzag(v - base_v)

// One code stream of a piece: a chunk of a split record, or a run of an
// unsplit one starting at a recorded decoder state.
struct HubStream {
  uint64_t pos;    // compressed: byte of the first code; plain: first edge
  uint32_t len;    // compressed: code bytes
  uint32_t cnt;    // neighbours | kStreamZig
  int32_t base_v;  // the first neighbour is base_v + (zigzag or gap) code
  int32_t base_w;  // the first weight is base_w + unzigzag(code)
  uint32_t nnum;   // interval-coded: VarInts in the stream's bytes
  uint32_t pad;
};

// VarInts (bytes with the continuation bit clear) in bytes [p0, p1).
__device__ __forceinline__ uint32_t count_varints(const uint8_t* b, uint64_t p0, uint64_t p1) {
  uint32_t c = 0;
  for (uint64_t p = p0; p < p1; ++p) c += (b[p] & 0x80u) ? 0u : 1u;
  return c;
}

// A (hub, partition) reduction task, everything H2 needs in one load.
struct HubTask {
  int32_t u;        // hub vertex
  int32_t nparts;   // P_h
  int32_t nseg;     // pieces of the hub
  int32_t part;     // the partition
  uint64_t rec0;    // first record of the hub (piece j at + j * kHubPiece)
  uint64_t poff0;   // piece j's P_h + 1 partition offsets at + j * (P_h + 1)
};
static_assert(sizeof(HubTask) == 32, "HubTask is eight words");

struct HubMeta {
  const int32_t* u;          // hub vertex
  const int32_t* deg;
  const int32_t* nparts;     // P_h
  const int32_t* npieces;    // pieces of the hub
  const int32_t* piece_base; // first piece of the hub (global index)
  const uint64_t* rec_base;  // first record of the hub (piece j at + j * kHubPiece)
  const uint64_t* poff_base; // piece j's P_h + 1 partition offsets at + j * (P_h + 1)
  const int32_t* task_base;  // first (hub, partition) task
  const int2* pieces;        // (hub, piece within the hub)
  const HubTask* tdesc;      // (hub, partition) tasks
  HubStream* streams;        // kHubStreams per piece
  int32_t* rec_c;            // records: cluster (packed: cluster << rbits | partial rating)
  void* rec_r;               // records: partial rating (int32 or int64); unused when packed
  // unit edge weights: one 32-bit word per record, the cluster in the high
  // 32 - rbits bits and a partial rating of at most 2^rbits - 1 in the low
  // ones (a larger rating takes several records, so a piece still needs at
  // most one record per neighbour)
  int32_t packed;
  uint32_t rbits;
  uint32_t tmax;  // LDS table entries of a reduction task (power of two)
  uint32_t* poff;
  int64_t* res_r;            // per task
  uint64_t* res_key;
  int32_t* res_c;
  int64_t* res_own;
};

// Stream descriptors of every hub piece, once per call: one wavefront per
// hub. Split records take their chunk table; unsplit records are decoded
// once to record the decoder state at every piece boundary.
template <class Cfg>
__global__ __launch_bounds__(256) void k_hub_streams(GraphView g, HubMeta hm, int32_t nhubs) {
  constexpr uint32_t NS = (uint32_t)Cfg::kStreams, PIECE = (uint32_t)Cfg::kEdges;
  __shared__ DecodeSmem<kWave> dsm[4];
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t h = wid; h < nhubs; h += nw) {
    const int32_t u = hm.u[h];
    const uint32_t d = (uint32_t)hm.deg[h];
    const uint32_t npc = (uint32_t)hm.npieces[h];
    HubStream* st = hm.streams + (uint64_t)hm.piece_base[h] * NS;
    const HubStream none{0, 0, 0, 0, 0, 0, 0};
    if (g.offs) {
      const Nbh hb = nbh_locate(g, u, d);
      if (hb.nchunks > 1) {
        // chunk k is stream k % NS of piece k / NS; unused slots of the last piece are empty
        for (uint32_t k = lane; k < npc * NS; k += kWave) {
          if (k < hb.nchunks) {
            const uint64_t p0 = nbh_chunk_pos(g, hb, k);
            const uint64_t p1 = k + 1 < hb.nchunks ? nbh_chunk_pos(g, hb, k + 1) : g.offs[u + 1];
            const uint32_t cnt = min((uint32_t)LP_CHUNK_LEN, d - k * LP_CHUNK_LEN);
            const uint32_t nn = g.intervals ? count_varints(g.bytes, p0, p1) : 0u;
            st[k] = HubStream{p0, (uint32_t)(p1 - p0), cnt | kStreamZig, u, 0, nn, 0};
          } else {
            st[k] = none;
          }
        }
      } else if (g.intervals) {
        // an unsplit interval-coded record has at most PIECE neighbours:
        // one piece, one stream over the whole record
        const uint64_t p0 = hb.codes, p1 = g.offs[u + 1];
        const uint32_t nn = count_varints(g.bytes, p0, p1);  // every lane counts; lane 0 writes
        for (uint32_t k = lane; k < npc * NS; k += kWave)
          st[k] = k == 0 ? HubStream{p0, (uint32_t)(p1 - p0), d | kStreamZig, u, 0, nn, 0} : none;
      } else {
        uint64_t pos = hb.codes;
        int32_t pv = 0, pw = 0;
        for (uint32_t j = 0; j < npc; ++j) {
          const uint32_t cnt = min(PIECE, d - j * PIECE);
          const uint64_t p0 = pos;
          const int32_t bv = j == 0 ? u : pv, bw = j == 0 ? 0 : pw;
          (void)group_decode<kWave>(g.bytes, pos, u, cnt, g.weighted, j == 0, pv, pw, dsm[w],
                                    [](uint32_t, int32_t, int32_t) {});
          if (lane < NS)
            st[(uint64_t)j * NS + lane] =
                lane == 0 ? HubStream{p0, (uint32_t)(pos - p0), cnt | (j == 0 ? kStreamZig : 0u), bv, bw, 0, 0}
                          : none;
        }
      }
    } else {
      const uint64_t e0 = g.xadj[u];
      for (uint32_t k = lane; k < npc * NS; k += kWave) {
        const uint32_t j = k / NS;
        const uint32_t cnt = min(PIECE, d - j * PIECE);
        st[k] = (k % NS == 0) ? HubStream{e0 + (uint64_t)j * PIECE, 0, cnt, 0, 0, 0, 0} : none;
      }
    }
  }
}

template <class Cfg>
struct PieceShared {
  static constexpr int NS = Cfg::kStreams, NW = Cfg::kThreads / kWave;
  uint64_t pos[NS];
  uint32_t len[NS];
  int32_t base_v[NS];
  int32_t base_w[NS];
  uint32_t zig[NS];
  uint32_t ebase[NS + 1];
  uint32_t dwbase[NS + 1];
  uint32_t rstart[NS + 1];
  uint32_t hist[Cfg::kWhole ? 1 : kMaxParts];
  unsigned long long red_u[NW];
  int32_t scan[NW];
  int32_t scan2[NW];
  Cand best[NW];
  int64_t red[NW];
  uint32_t seg_flags;
  uint32_t next;  // piece handed to the workgroup
};

// H1: one workgroup per hub piece (of a whole hub: H1 to H3 at once).
template <class Cfg, typename V, bool COMP, int MODE = kModeRate, bool ITV = false>
__global__ __launch_bounds__(Cfg::kThreads) void k_hub_piece(RoundCtx x, HubMeta hm, int32_t npieces,
                                                            uint32_t* ctr, TileLayout L) {
  constexpr int NT = Cfg::kThreads, ITEMS = Cfg::kItems, NS = Cfg::kStreams;
  constexpr bool WHOLE = Cfg::kWhole;
  extern __shared__ __align__(16) uint8_t smem_raw[];
  if (*x.done) return;
  const int tid = threadIdx.x;
  const bool weighted = x.g.weighted;
  const uint32_t per = weighted ? 2u : 1u;
  uint8_t* A = smem_raw;
  uint32_t* A32 = (uint32_t*)A;
  int32_t* keys = (int32_t*)A;
  V* vals = (V*)(A + (size_t)Cfg::kSlots * 4);
  uint32_t* nums = (uint32_t*)(A + L.nums_off);
  PieceShared<Cfg>& sh = *(PieceShared<Cfg>*)(A + L.abytes);
  V* rec_r = (V*)hm.rec_r;
  // pieces are handed out at run time, kPieceGrab at a time (one counter)
  uint32_t pnext = 0, pend = 0;
  while (true) {
    if (pnext >= pend) {
      if (tid == 0) sh.next = atomicAdd(ctr, (uint32_t)kPieceGrab);
      __syncthreads();
      pnext = sh.next;
      __syncthreads();
      if (pnext >= (uint32_t)npieces) break;
      pend = min((uint32_t)npieces, pnext + (uint32_t)kPieceGrab);
    }
    const int64_t pc = pnext++;
    const int2 pj = hm.pieces[pc];
    const int h = pj.x;
    const uint32_t P = WHOLE ? 1u : (uint32_t)hm.nparts[h];
    const uint64_t rbase = WHOLE ? 0ull : hm.rec_base[h] + (uint64_t)pj.y * kHubPiece;
    uint32_t* po = WHOLE ? nullptr : hm.poff + hm.poff_base[h] + (uint64_t)pj.y * (P + 1);
    // 0. streams
    if (tid == 0) {
      uint32_t e = 0, dw = 0, nn = 0;
      for (int s = 0; s < NS; ++s) {
        const HubStream hs = hm.streams[pc * NS + s];
        const uint32_t cnt = hs.cnt & ~kStreamZig;
        sh.pos[s] = hs.pos;
        sh.len[s] = hs.len;
        sh.base_v[s] = hs.base_v;
        sh.base_w[s] = hs.base_w;
        sh.zig[s] = (hs.cnt & kStreamZig) ? 1u : 0u;
        sh.ebase[s] = e;
        sh.dwbase[s] = dw;
        const uint32_t pre = COMP ? (uint32_t)(hs.pos & 3u) : 0u;
        sh.rstart[s] = nn + pre;
        e += cnt;
        if (COMP && cnt > 0) {
          const uint32_t ndw = (pre + hs.len + 3u) >> 2;
          dw += ndw;
          nn += (ITV ? hs.nnum : per * cnt) + 4u * ndw - hs.len;
        }
      }
      sh.ebase[NS] = e;
      sh.dwbase[NS] = dw;
      sh.rstart[NS] = nn;
      sh.seg_flags = 0;
    }
    if constexpr (!WHOLE)
      for (uint32_t p = tid; p < P; p += NT) sh.hist[p] = 0;
    __syncthreads();
    const uint32_t Et = sh.ebase[NS];
    if constexpr (COMP) {
      const uint32_t Dt = sh.dwbase[NS];
      // four consecutive dwords per thread, four independent loads in flight
      for (uint32_t jb = 4 * tid; jb < Dt; jb += 4 * NT) {
        uint32_t w[4], off[4];
        int32_t si[4];
        int32_t s = 0;
        while (jb >= sh.dwbase[s + 1]) ++s;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t j = jb + (uint32_t)k;
          si[k] = -1;
          w[k] = 0;
          off[k] = 0;
          if (j < Dt) {
            while (j >= sh.dwbase[s + 1]) ++s;
            si[k] = s;
            off[k] = 4u * (j - sh.dwbase[s]);
            w[k] = *(const uint32_t*)(x.g.bytes + (sh.pos[s] & ~3ull) + off[k]);
          }
        }
        uint4 o;
        uint32_t* ov = (uint32_t*)&o;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          ov[k] = 0;
          if (si[k] < 0) continue;
          const int32_t s2 = si[k];
          // bytes [b0, b1) of the stream's dwords are its codes
          const int32_t b0 = (int32_t)(sh.pos[s2] & 3u), b1 = b0 + (int32_t)sh.len[s2];
          const int32_t lo = min(max(b0 - (int32_t)off[k], 0), 4), hi = min(max(b1 - (int32_t)off[k], 0), 4);
          ov[k] = w[k] & (uint32_t)(((1ull << (8 * hi)) - 1ull) ^ ((1ull << (8 * lo)) - 1ull));
        }
        if (jb + 4 <= Dt) {
          *(uint4*)&A32[jb] = o;
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (jb + k < Dt) A32[jb + k] = ov[k];
        }
      }
      __syncthreads();
      stage_numbers<NT, !ITV>(A32, Dt, nums, sh.scan);
      __syncthreads();
    }
    // neighbour IDs, weights and labels of this thread's slice
    const uint32_t Dd = (Et + NT - 1) / NT;
    const uint32_t e0 = tid * Dd;
    int32_t vi[ITEMS], nb[ITEMS], wt[ITEMS];
    if constexpr (COMP && ITV) {
      // interval-coded: every stream is a chunk start (see k_hub_streams)
      const ItvTable itv = itv_table<NT, NS, Cfg::kEdges / 3 + 1>(A32, nums, sh.rstart, sh.ebase, sh.base_v, NS,
                                                                 sh.scan, sh.scan2, &sh.seg_flags);
      int32_t s = 0;
      if (e0 < Et)
        while (e0 >= sh.ebase[s + 1]) ++s;
      uint32_t hidm = 0, hwm = 0;
      int32_t a = 0, a2 = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t e = e0 + k;
        vi[k] = -1;
        nb[k] = 0;
        wt[k] = 1;
        if ((uint32_t)k < Dd && e < Et) {
          while (e >= sh.ebase[s + 1]) ++s;
          vi[k] = s;
          const uint32_t loc = e - sh.ebase[s];
          int32_t dv, dw;
          bool hid;
          itv_item(itv, nums, sh.rstart[s], s, loc, sh.base_v[s], weighted, dv, dw, hid);
          const bool hw = loc == 0;
          a = hid ? dv : a + dv;
          a2 = hw ? dw : a2 + dw;
          hidm |= (uint32_t)hid << k;
          hwm |= (uint32_t)hw << k;
          nb[k] = a;
          wt[k] = a2;
        }
      }
      int32_t ex, ex2, unused;
      tile_seg_scan<NT>(hidm != 0, a, 0, sh.scan, sh.scan2, &sh.seg_flags, ex, unused);
      __syncthreads();
      if (tid == 0) sh.seg_flags = 0;
      __syncthreads();
      if (weighted) {
        tile_seg_scan<NT>(hwm != 0, a2, 0, sh.scan, sh.scan2, &sh.seg_flags, ex2, unused);
        __syncthreads();
        if (tid == 0) sh.seg_flags = 0;
      }
      const uint32_t fid = hidm ? (uint32_t)__ffs(hidm) - 1u : 32u;
      const uint32_t fw = hwm ? (uint32_t)__ffs(hwm) - 1u : 32u;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (vi[k] < 0) continue;
        if ((uint32_t)k < fid) nb[k] += ex;
        if (weighted) {
          if ((uint32_t)k < fw) wt[k] += ex2;
        } else {
          wt[k] = 1;
        }
      }
    } else {
      int32_t s = 0;
      if (e0 < Et)
        while (e0 >= sh.ebase[s + 1]) ++s;
      bool any_head = false;
      int32_t a = 0, a2 = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t e = e0 + k;
        vi[k] = -1;
        nb[k] = 0;
        wt[k] = 1;
        if ((uint32_t)k < Dd && e < Et) {
          while (e >= sh.ebase[s + 1]) ++s;
          vi[k] = s;
          const uint32_t loc = e - sh.ebase[s];
          if constexpr (COMP) {
            const uint32_t ci = sh.rstart[s] + per * loc;
            const uint32_t code = number_at(A32, nums, ci);
            const bool head = loc == 0;
            const int32_t dv =
                head ? sh.base_v[s] + (sh.zig[s] ? unzigzag32(code) : (int32_t)code) : (int32_t)code;
            const int32_t dw = weighted ? (head ? sh.base_w[s] : 0) + unzigzag32(number_at(A32, nums, ci + 1)) : 0;
            if (head) {
              any_head = true;
              a = dv;
              a2 = dw;
            } else {
              a += dv;
              a2 += dw;
            }
            nb[k] = a;
            wt[k] = a2;
          } else {
            const uint64_t ge = sh.pos[s] + loc;
            nb[k] = x.g.adjncy[ge];
            if (weighted) wt[k] = x.g.adjwgt[ge];
          }
        }
      }
      if constexpr (COMP) {
        int32_t ex, ex2;
        tile_seg_scan<NT>(any_head, a, a2, sh.scan, sh.scan2, &sh.seg_flags, ex, ex2);
        bool before = true;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          if (vi[k] < 0) continue;
          if (e0 + k == sh.ebase[vi[k]]) before = false;
          if (before) {
            nb[k] += ex;
            wt[k] += ex2;
          }
          if (!weighted) wt[k] = 1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      if (vi[k] < 0) continue;
      if ((uint32_t)nb[k] < (uint32_t)x.g.n) nb[k] = x.C[nb[k]];
      else vi[k] = -1;  // unreachable for a valid handle; keeps the gather in bounds
    }
    if constexpr (MODE != kModeRate) {
      const int32_t u = hm.u[h];
      const int32_t own = x.C[u];
      if constexpr (MODE == kModeCut) {
        unsigned long long c = 0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
          if (vi[k] >= 0 && nb[k] != own) c += (unsigned long long)wt[k];
        c = block_reduce_add<NT, unsigned long long>(c, sh.red_u);
        if (tid == 0 && c) atomicAdd(x.cut, c);
      } else if (x.rec_sum) {
        // the piece's edges summed per coarse neighbour in the table (as in
        // the tiles): the edge that put a neighbour into the table carries
        // the sum, the others become empty records
        __syncthreads();  // numbers consumed: region A becomes the table
        const uint32_t S = tile_slots(Et);
        for (uint32_t q = tid; q < S; q += NT) keys[q] = kEmpty;
        for (uint32_t q = tid; q < S; q += NT) vals[q] = 0;
        __syncthreads();
        int32_t vj[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) vj[k] = vi[k] >= 0 && nb[k] != own ? vi[k] : -1;
        uint32_t qs[ITEMS], claim = 0;
        auto pspan = [&](int32_t, uint32_t& b, uint32_t& sz) {
          b = 0;
          sz = S;
        };
        tile_insert_all<ITEMS, V, decltype(pspan), true>(keys, vals, vj, nb, wt, pspan, qs, &claim);
        __syncthreads();
        Rec* r = x.rec + x.rbase[own] + x.voff[prop_slot(x, u)] + (uint64_t)pj.y * Cfg::kEdges;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
          if (vi[k] < 0) continue;
          const bool lead = vj[k] >= 0 && ((claim >> k) & 1u);
          r[e0 + k] = lead ? Rec{nb[k], (int32_t)vals[qs[k]]} : Rec{-1, 0};
        }
      } else {
        Rec* r = x.rec + x.rbase[own] + x.voff[prop_slot(x, u)] + (uint64_t)pj.y * Cfg::kEdges;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
          if (vi[k] >= 0) r[e0 + k] = Rec{nb[k] == own ? -1 : nb[k], wt[k]};
      }
      __syncthreads();
      continue;
    }
    __syncthreads();  // numbers consumed: region A becomes the table
    const uint32_t S = tile_slots(Et);
    for (uint32_t q = tid; q < S; q += NT) keys[q] = kEmpty;
    for (uint32_t q = tid; q < S; q += NT) vals[q] = 0;
    __syncthreads();
    tile_insert_all<ITEMS, V>(keys, vals, vi, nb, wt, [&](int32_t, uint32_t& b, uint32_t& sz) {
      b = 0;
      sz = S;
    });
    __syncthreads();
    if constexpr (WHOLE) {
      // the hub's own rating and best cluster by (rating, smallest key),
      // keys computed only for slots that reach the thread's best rating;
      // if that cluster is full, the best one with room
      const int32_t u = hm.u[h];
      const int32_t own_c = x.C[u];
      const int64_t wu = vweight(x.g, u);
      const VParams vp = vparams(x, u);
      Cand lb = cand_none();
      int64_t own = 0;
      for (uint32_t q = tid; q < S; q += NT) {
        const int32_t c = keys[q];
        if (c == kEmpty) continue;
        const int64_t r = (int64_t)vals[q];
        if (c == own_c) {
          own = r;
          continue;
        }
        if (r < lb.r) continue;
        const Cand cd{r, cluster_key(x, vp, c), c};
        if (cand_better(cd, lb)) lb = cd;
      }
      lb = block_best<NT>(lb, sh.best);
      own = block_reduce_add<NT, int64_t>(own, sh.red);
      Cand best = cand_none();
      if (lb.c >= 0 && lb.r > own) {
        if (x.W[lb.c] + wu <= vp.cap) {
          best = lb;
        } else {
          Cand fb = cand_none();
          for (uint32_t q = tid; q < S; q += NT) {
            const int32_t c = keys[q];
            if (c == kEmpty || c == own_c) continue;
            const int64_t r = (int64_t)vals[q];
            if (r <= own || r < fb.r) continue;
            const Cand cd{r, cluster_key(x, vp, c), c};
            if (cand_better(cd, fb) && x.W[c] + wu <= vp.cap) fb = cd;
          }
          best = block_best<NT>(fb, sh.best);
        }
      }
      if (tid == 0) emit(x, u, best, own);
      __syncthreads();
      continue;
    }
    // distinct clusters grouped by partition
    const uint32_t rmax = hm.packed ? (1u << hm.rbits) - 1u : 0u;
    for (uint32_t q = tid; q < S; q += NT) {
      const int32_t c = keys[q];
      if (c == kEmpty) continue;
      const uint32_t nr = hm.packed ? ((uint32_t)vals[q] + rmax - 1u) / rmax : 1u;
      atomicAdd(&sh.hist[part_hash((uint32_t)c) % P], nr);
    }
    __syncthreads();
    {
      uint32_t carry = 0;
      for (uint32_t b0 = 0; b0 < P; b0 += NT) {
        const uint32_t p = b0 + tid;
        const int32_t v = p < P ? (int32_t)sh.hist[p] : 0;
        int32_t tot;
        const int32_t inc = block_incl_scan_add<NT, int32_t>(v, sh.scan, &tot);
        if (p < P) {
          sh.hist[p] = carry + (uint32_t)(inc - v);
          po[p] = carry + (uint32_t)(inc - v);
        }
        carry += (uint32_t)tot;
      }
      if (tid == 0) po[P] = carry;
    }
    __syncthreads();
    for (uint32_t q = tid; q < S; q += NT) {
      const int32_t c = keys[q];
      if (c == kEmpty) continue;
      if (hm.packed) {
        uint32_t r = (uint32_t)vals[q];
        const uint32_t nr = (r + rmax - 1u) / rmax;
        uint32_t slot = atomicAdd(&sh.hist[part_hash((uint32_t)c) % P], nr);
        for (; r > 0; ++slot) {
          const uint32_t part = r < rmax ? r : rmax;
          hm.rec_c[rbase + slot] = (int32_t)(((uint32_t)c << hm.rbits) | part);
          r -= part;
        }
      } else {
        const uint32_t slot = atomicAdd(&sh.hist[part_hash((uint32_t)c) % P], 1u);
        hm.rec_c[rbase + slot] = c;
        rec_r[rbase + slot] = vals[q];
      }
    }
    __syncthreads();
  }
}

constexpr uint32_t kHubTableMin = 1024, kHubTableMax = 16384;

// LDS entries of a (hub, partition) task's table: a power of two that holds
// hub_part records at a load of at most 5/8 (a partition with more records
// is summed in label-range sub-passes).
inline uint32_t hub_table(int32_t hub_part, bool wide) {
  const uint32_t cap = wide ? kHubTableMax / 2 : kHubTableMax;  // 64-bit ratings: 12 bytes per entry
  uint32_t t = kHubTableMin;
  while ((uint64_t)t * 5u < (uint64_t)hub_part * 8u && t < cap) t <<= 1;
  return t;
}
constexpr int kRedItems = 8;                          // records per thread and window
constexpr int kRedWindow = kHubThreads * kRedItems;  // records placed by one owner map

struct HubReduceSmem {
  Cand best[kHubThreads / kWave];
  int64_t red[kHubThreads / kWave];
  int32_t scan[kHubThreads / kWave];
  uint32_t distinct;
  uint32_t overflow;
  alignas(16) uint64_t base[kHubThreads];  // per piece of a batch: its first record's address minus its first position
  alignas(16) uint16_t own[kRedWindow];    // owner map of a window: 1 + the batch's piece that holds each position
};

// Block-wide inclusive max-scan of one non-negative int per thread, seeded
// with `carry`; *total = the maximum over the block and the carry.
template <int NT>
__device__ __forceinline__ int32_t block_incl_scan_max(int32_t x, int32_t carry, int32_t* sm, int32_t* total) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t y = __shfl_up(x, d, kWave);
    if (lane_id() >= d) x = y > x ? y : x;
  }
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == kWave - 1) sm[w] = x;
  __syncthreads();
  int32_t off = carry, tot = carry;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) {
    const int32_t v = sm[i];
    if (i < w) off = v > off ? v : off;
    tot = v > tot ? v : tot;
  }
  *total = tot;
  return x > off ? x : off;
}

// H2: (hub, partition) tasks, a fixed stride of them per workgroup; the
// next task's descriptor is loaded while the current one runs. The table
// holds the partition's record count at a load of at most 5/8 (at most
// hm.tmax entries; more records are summed in label-range sub-passes,
// doubled again if a sub-pass still sees too many distinct clusters). The
// partition's records lie in one run per piece; a batch of kHubThreads
// pieces is walked as one flat range, window by window, each record finding
// its piece through an owner map (piece starts scattered into LDS, then a
// block-wide max-scan).
template <typename V>
__global__ __launch_bounds__(kHubThreads) void k_hub_reduce(RoundCtx x, HubMeta hm, int32_t ntasks) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  constexpr int NT = kHubThreads;
  int32_t* keys = (int32_t*)smem_raw;
  const uint32_t tmax = hm.tmax;
  V* vals = (V*)(smem_raw + (size_t)tmax * 4);
  HubReduceSmem& sm = *(HubReduceSmem*)(smem_raw + (size_t)tmax * (4 + sizeof(V)));
  const V* rec_r = (const V*)hm.rec_r;
  if (*x.done) return;
  const int tid = threadIdx.x, lane = lane_id();
  constexpr int kDescWords = (int)(sizeof(HubTask) / 4);
  // lanes 0..7 of every wave hold the current task's descriptor words
  const int64_t t0 = blockIdx.x;
  uint32_t dw = (t0 < ntasks && lane < kDescWords) ? ((const uint32_t*)(hm.tdesc + t0))[lane] : 0u;
  for (int64_t t = t0; t < ntasks; t += gridDim.x) {
    const int32_t u = __builtin_amdgcn_readlane((int)dw, 0);
    const uint32_t P = (uint32_t)__builtin_amdgcn_readlane((int)dw, 1);
    const uint32_t nseg = (uint32_t)__builtin_amdgcn_readlane((int)dw, 2);
    const uint32_t p = (uint32_t)__builtin_amdgcn_readlane((int)dw, 3);
    const uint64_t rb0 = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)dw, 4) |
                         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)dw, 5) << 32);
    const uint64_t pb0 = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)dw, 6) |
                         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)dw, 7) << 32);
    const int64_t tn = t + gridDim.x;
    dw = (tn < ntasks && lane < kDescWords) ? ((const uint32_t*)(hm.tdesc + tn))[lane] : 0u;
    const uint32_t* po = hm.poff + pb0;
    const int32_t own_c = x.C[u];
    const int64_t wu = vweight(x.g, u);
    const VParams vp = vparams(x, u);
    // records of this partition; the first batch's runs stay in registers
    uint32_t ra0 = 0, c0 = 0;
    int64_t cnt = 0;
    for (uint32_t k = tid; k < nseg; k += NT) {
      const uint32_t a = po[(uint64_t)k * (P + 1) + p], e = po[(uint64_t)k * (P + 1) + p + 1];
      cnt += e - a;
      if (k < (uint32_t)NT) {
        ra0 = a;
        c0 = e - a;
      }
    }
    cnt = block_reduce_add<NT, int64_t>(cnt, sm.red);
    uint32_t tcap = 64;
    while (tcap < tmax && (uint64_t)tcap * 5u < (uint64_t)cnt * 8u) tcap <<= 1;
    uint32_t S = 1;  // label-range sub-passes
    while ((uint64_t)tcap * 5u * S < (uint64_t)cnt * 8u) S <<= 1;
    const uint32_t logc = ceil_log2(tcap), mask = tcap - 1, shift = 32 - logc;
    const uint32_t limit = tcap - tcap / 4;  // distinct clusters a sub-pass may hold
    Cand best;
    int64_t own;
    while (true) {
      best = cand_none();
      own = 0;
      bool over = false;
      for (uint32_t sp = 0; sp < S; ++sp) {
        for (uint32_t q = 4 * tid; q < tcap; q += 4 * NT) *(int4*)&keys[q] = make_int4(kEmpty, kEmpty, kEmpty, kEmpty);
        for (uint32_t q = 4 * tid; q < tcap; q += 4 * NT) {
          if constexpr (sizeof(V) == 8) {
            *(int4*)&vals[q] = make_int4(0, 0, 0, 0);
            *(int4*)&vals[q + 2] = make_int4(0, 0, 0, 0);
          } else {
            *(int4*)&vals[q] = make_int4(0, 0, 0, 0);
          }
        }
        if (tid == 0) {
          sm.distinct = 0;
          sm.overflow = 0;
        }
        __syncthreads();
        for (uint32_t kb = 0; kb < nseg; kb += NT) {
          const uint32_t k = kb + tid;
          uint32_t ra = ra0, c = c0;
          if (kb > 0) {
            ra = 0;
            c = 0;
            if (k < nseg) {
              ra = po[(uint64_t)k * (P + 1) + p];
              c = po[(uint64_t)k * (P + 1) + p + 1] - ra;
            }
          } else if (k >= nseg) {
            c = 0;
          }
          int32_t total;
          const int32_t pre = block_incl_scan_add<NT, int32_t>((int32_t)c, sm.scan, &total) - (int32_t)c;
          sm.base[tid] = rb0 + (uint64_t)k * kHubPiece + ra - (uint64_t)pre;
          int32_t carry = 0;
          for (int32_t j0 = 0; j0 < total; j0 += kRedWindow) {
            // owner map of positions [j0, j0 + kRedWindow)
            *(int4*)&sm.own[8 * tid] = make_int4(0, 0, 0, 0);
            __syncthreads();
            if (c > 0 && pre >= j0 && pre < j0 + kRedWindow) sm.own[pre - j0] = (uint16_t)(tid + 1);
            __syncthreads();
            int4 o4 = *(const int4*)&sm.own[8 * tid];
            uint16_t ov[8];
            __builtin_memcpy(ov, &o4, 16);
            int32_t run = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) run = (int32_t)ov[q] > run ? (int32_t)ov[q] : run;
            int32_t blockmax;
            int32_t m = block_incl_scan_max<NT>(run, carry, sm.scan, &blockmax);
            // exclusive prefix of this thread's eight positions
            const int32_t prev = __shfl_up(m, 1, kWave);
            int32_t ex = lane > 0 ? prev : 0;
            if (lane == 0) {
              const int w = tid / kWave;
              ex = carry;
              for (int i = 0; i < w; ++i) ex = sm.scan[i] > ex ? sm.scan[i] : ex;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              ex = (int32_t)ov[q] > ex ? (int32_t)ov[q] : ex;
              ov[q] = (uint16_t)ex;
            }
            __builtin_memcpy(&o4, ov, 16);
            __syncthreads();  // every wave has read the cross-wave maxima
            *(int4*)&sm.own[8 * tid] = o4;
            carry = blockmax;
            __syncthreads();
            int32_t cc[kRedItems];
            V ww[kRedItems];
#pragma unroll
            for (int q = 0; q < kRedItems; ++q) {
              const int32_t j = j0 + q * NT + tid;
              cc[q] = kEmpty;
              ww[q] = 0;
              if (j < total) {
                const uint64_t r = sm.base[sm.own[q * NT + tid] - 1] + (uint64_t)j;
                if (hm.packed) {
                  const uint32_t pw = (uint32_t)hm.rec_c[r];
                  cc[q] = (int32_t)(pw >> hm.rbits);
                  ww[q] = (V)(pw & ((1u << hm.rbits) - 1u));
                } else {
                  cc[q] = hm.rec_c[r];
                  ww[q] = rec_r[r];
                }
              }
            }
#pragma unroll
            for (int q = 0; q < kRedItems; ++q) {
              const int32_t c2 = cc[q];
              if (c2 == kEmpty) continue;
              if (S > 1 && (uint32_t)(((uint64_t)(uint32_t)c2 * S) / (uint64_t)x.g.n) != sp) continue;
              const V w = ww[q];
              // buckets of four slots, read at once: a record finds its
              // cluster or the bucket's first free slot in one LDS read
              uint32_t b = (slot_hash((uint32_t)c2) >> shift) & ~3u;
              // one sub-pass: the table has room for every record, so it
              // cannot fill and the distinct count (one contended LDS atomic
              // per new cluster) is not needed
              bool reserved = S == 1;
              while (true) {
                const int4 k4 = *(const int4*)&keys[b];
                const uint32_t hit = (uint32_t)(k4.x == c2) | ((uint32_t)(k4.y == c2) << 1) |
                                     ((uint32_t)(k4.z == c2) << 2) | ((uint32_t)(k4.w == c2) << 3);
                if (hit) {
                  lds_add(&vals[b + (uint32_t)__ffs(hit) - 1u], w);
                  break;
                }
                const uint32_t fr = (uint32_t)(k4.x == kEmpty) | ((uint32_t)(k4.y == kEmpty) << 1) |
                                    ((uint32_t)(k4.z == kEmpty) << 2) | ((uint32_t)(k4.w == kEmpty) << 3);
                if (fr) {
                  if (!reserved) {
                    if (atomicAdd(&sm.distinct, 1u) >= limit) {
                      sm.overflow = 1;
                      break;
                    }
                    reserved = true;
                  }
                  // slots fill in order, so the first free slot ends the
                  // bucket's occupied prefix; if another record takes it
                  // first, the bucket is read again
                  const uint32_t sl = b + (uint32_t)__ffs(fr) - 1u;
                  const int32_t old = atomicCAS(&keys[sl], kEmpty, c2);
                  if (old == kEmpty || old == c2) {
                    lds_add(&vals[sl], w);
                    break;
                  }
                  continue;
                }
                b = (b + 4u) & mask;
              }
            }
            __syncthreads();  // the owner map is rebuilt by the next window
          }
          __syncthreads();  // sm.base is rewritten by the next batch
        }
        if (sm.overflow) {
          over = true;
          break;
        }
        // one pass over the table: the own cluster's rating and the best
        // other cluster by (rating, smallest tie-break key), keys computed
        // only for slots that reach the thread's best rating
        Cand lb = cand_none();
        for (uint32_t q = 4 * tid; q < tcap; q += 4 * NT) {
          const int4 k4 = *(const int4*)&keys[q];
          int64_t r4[4];
          if constexpr (sizeof(V) == 8) {
            const int4 a = *(const int4*)&vals[q], b = *(const int4*)&vals[q + 2];
            r4[0] = ((int64_t)(uint32_t)a.y << 32) | (uint32_t)a.x;
            r4[1] = ((int64_t)(uint32_t)a.w << 32) | (uint32_t)a.z;
            r4[2] = ((int64_t)(uint32_t)b.y << 32) | (uint32_t)b.x;
            r4[3] = ((int64_t)(uint32_t)b.w << 32) | (uint32_t)b.z;
          } else {
            const int4 a = *(const int4*)&vals[q];
            r4[0] = a.x;
            r4[1] = a.y;
            r4[2] = a.z;
            r4[3] = a.w;
          }
          const int32_t kc[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int32_t c = kc[i];
            if (c == kEmpty) continue;
            if (c == own_c) {
              own = r4[i];
              continue;
            }
            if (r4[i] < lb.r) continue;
            const Cand cd{r4[i], cluster_key(x, vp, c), c};
            if (cand_better(cd, lb)) lb = cd;
          }
        }
        lb = block_best<NT>(lb, sm.best);
        if (lb.c >= 0 && cand_better(lb, best)) {
          if (x.W[lb.c] + wu <= vp.cap) {
            best = lb;
          } else {
            // the best cluster is full: rescan with the cap, the cluster
            // weights of four slots loaded at once
            Cand fb = best;
            for (uint32_t q = 4 * tid; q < tcap; q += 4 * NT) {
              const int4 k4 = *(const int4*)&keys[q];
              const int32_t kc[4] = {k4.x, k4.y, k4.z, k4.w};
              int64_t r4[4], wc[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) r4[i] = (int64_t)vals[q + i];
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const bool cand = kc[i] != kEmpty && kc[i] != own_c && r4[i] >= fb.r;
                wc[i] = cand ? x.W[kc[i]] : INT64_MAX;
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (wc[i] == INT64_MAX || r4[i] < fb.r || wc[i] + wu > vp.cap) continue;
                const Cand cd{r4[i], cluster_key(x, vp, kc[i]), kc[i]};
                if (cand_better(cd, fb)) fb = cd;
              }
            }
            best = block_best<NT>(fb, sm.best);
          }
        }
        __syncthreads();
      }
      if (!over) break;
      __syncthreads();
      S *= 2;
    }
    own = block_reduce_add<NT, int64_t>(own, sm.red);
    if (tid == 0) {
      hm.res_r[t] = best.r;
      hm.res_key[t] = best.key;
      hm.res_c[t] = best.c;
      hm.res_own[t] = own;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_hub_combine(RoundCtx x, HubMeta hm, int32_t nhubs) {
  if (*x.done) return;
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t h = wid; h < nhubs; h += nw) {
    const int32_t P = hm.nparts[h];
    const int32_t tb = hm.task_base[h];
    Cand best = cand_none();
    int64_t own = 0;
    for (int32_t p = lane; p < P; p += kWave) {
      Cand c{hm.res_r[tb + p], hm.res_key[tb + p], hm.res_c[tb + p]};
      if (cand_better(c, best)) best = c;
      own += hm.res_own[tb + p];
    }
    best = wave_best(best);
    own = wave_reduce_add(own);
    if (lane == 0) emit(x, hm.u[h], best, own);
  }
}

// ------------------------------------------------------------ buckets ----
constexpr int kBkThreads = 256;
constexpr int kBkItems = 8;
constexpr int kBkTile = kBkThreads * kBkItems;
constexpr int kNumBuckets = 4;  // lane, small tiles, large tiles, hub

__device__ __forceinline__ int bucket_of(int32_t d, int32_t t_lane, int32_t t_tile, int32_t t_block) {
  if (d <= 0) return -1;
  if (d <= t_lane) return 0;
  if (d <= t_tile) return 1;
  if (d <= t_block) return 2;
  return 3;
}

// Sub-round of a vertex among S: the tie-break mix on a fixed salt and the
// vertex's ID inside its graph, modulo S (fixed for a whole call).
constexpr uint64_t kSubroundSalt = 0x6A09E667F3BCC909ull;
__device__ __forceinline__ uint32_t subround_of(uint32_t u_local, uint32_t S) {
  return (uint32_t)(tiebreak_key(kSubroundSalt, 0, u_local) % S);
}

// Degrees as seen by the plan of sub-round `sr`: vertices of other
// sub-rounds get degree 0 and so fall in no bucket.
__global__ void k_subround_deg(const int32_t* deg, int32_t n, uint32_t S, uint32_t sr, const int32_t* gid,
                               const int32_t* gbase, int32_t* out) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t loc = gid ? (uint32_t)(u - gbase[gid[u]]) : (uint32_t)u;
    out[u] = subround_of(loc, S) == sr ? deg[u] : 0;
  }
}

// Descriptor of every listed (non-hub) vertex: degree and the position of its
// first code (compressed: after the first-edge header; these degrees are
// never chunked) or first edge (plain).
__global__ void k_build_desc(GraphView g, const int32_t* order, const int32_t* deg, int32_t cnt, int4* vdesc,
                             uint32_t* vlen, uint32_t* vnum) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = order[i];
    uint64_t pos;
    uint32_t len = 0;
    if (g.offs) {
      (void)read_header(g, u, pos);
      len = (uint32_t)(g.offs[u + 1] - pos);
    } else {
      pos = g.xadj[u];
    }
    vdesc[i] = make_int4(u, deg[u], (int)(uint32_t)pos, (int)(uint32_t)(pos >> 32));
    vlen[i] = len;
    if (vnum) vnum[i] = count_varints(g.bytes, pos, pos + len);
  }
}

__global__ __launch_bounds__(kBkThreads) void k_bucket_count(const int32_t* deg, int32_t n, int32_t t_lane,
                                                             int32_t t_tile, int32_t t_block, uint32_t* counts,
                                                             uint32_t nb) {
  __shared__ uint32_t c[kNumBuckets];
  if (threadIdx.x < kNumBuckets) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBkTile;
  for (int i = 0; i < kBkItems; ++i) {
    const int64_t u = base + (int64_t)i * kBkThreads + threadIdx.x;
    if (u < n) {
      const int b = bucket_of(deg[u], t_lane, t_tile, t_block);
      if (b >= 0) atomicAdd(&c[b], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < kNumBuckets) counts[(size_t)threadIdx.x * nb + blockIdx.x] = c[threadIdx.x];
}

// Stable: within a block, vertices keep increasing order per bucket.
__global__ __launch_bounds__(kBkThreads) void k_bucket_scatter(const int32_t* deg, int32_t n, int32_t t_lane,
                                                               int32_t t_tile, int32_t t_block,
                                                               const uint32_t* offs, uint32_t nb, int32_t* order) {
  __shared__ uint32_t run[kNumBuckets];
  __shared__ uint32_t wc[kBkThreads / kWave][kNumBuckets];
  const int w = threadIdx.x / kWave;
  if (threadIdx.x < kNumBuckets) run[threadIdx.x] = offs[(size_t)threadIdx.x * nb + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kBkTile;
  const uint64_t lt = lanemask_lt();
  for (int i = 0; i < kBkItems; ++i) {
    const int64_t u = base + (int64_t)i * kBkThreads + threadIdx.x;
    const int b = (u < n) ? bucket_of(deg[u], t_lane, t_tile, t_block) : -1;
    uint64_t m[kNumBuckets];
#pragma unroll
    for (int k = 0; k < kNumBuckets; ++k) m[k] = __ballot(b == k);
    if (lane_id() < kNumBuckets) wc[w][lane_id()] = __popcll(m[lane_id()]);
    __syncthreads();
    if (b >= 0) {
      uint32_t off = run[b] + __popcll(m[b] & lt);
      for (int k = 0; k < w; ++k) off += wc[k][b];
      order[off] = (int32_t)u;
    }
    __syncthreads();
    if (threadIdx.x < kNumBuckets) {
      uint32_t add = 0;
      for (int k = 0; k < kBkThreads / kWave; ++k) add += wc[k][threadIdx.x];
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// Per-bucket adjacency entries and compressed record bytes (statistics).
__global__ __launch_bounds__(256) void k_bucket_sums(const int32_t* deg, int32_t n, int32_t t_lane, int32_t t_tile,
                                                     int32_t t_block, const uint64_t* offs,
                                                     unsigned long long* sums) {
  __shared__ unsigned long long sm[2 * kNumBuckets];
  if (threadIdx.x < 2 * kNumBuckets) sm[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int b = bucket_of(deg[u], t_lane, t_tile, t_block);
    if (b < 0) continue;
    atomicAdd(&sm[b], (unsigned long long)deg[u]);
    if (offs) atomicAdd(&sm[kNumBuckets + b], (unsigned long long)(offs[u + 1] - offs[u]));
  }
  __syncthreads();
  if (threadIdx.x < 2 * kNumBuckets && sm[threadIdx.x]) atomicAdd(&sums[threadIdx.x], sm[threadIdx.x]);
}

// ------------------------------------------------------------ accept -----
constexpr int kCpThreads = 256;
constexpr int kCpItems = 8;
constexpr int kCpTile = kCpThreads * kCpItems;

__global__ __launch_bounds__(kCpThreads) void k_prop_count(const int32_t* ptgt, int32_t n, uint32_t* bc,
                                                           const uint32_t* done) {
  __shared__ uint32_t sm[kCpThreads / kWave];
  if (*done) return;
  const int64_t base = (int64_t)blockIdx.x * kCpTile + (int64_t)threadIdx.x * kCpItems;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kCpItems; ++i)
    if (base + i < n && ptgt[base + i] >= 0) ++c;
  c = block_reduce_add<kCpThreads, uint32_t>(c, sm);
  if (threadIdx.x == 0) bc[blockIdx.x] = c;
}

// Writes the proposals in increasing vertex order: key = target << G |
// (2^G - 1 - gain), value = vertex. With sub-rounds, or when rating a
// reordered copy (which writes proposals only), it clears the proposal slots
// it took; otherwise every rated vertex writes its slot again in the next
// round.
__global__ __launch_bounds__(kCpThreads) void k_prop_write(int32_t* ptgt, const int64_t* pgain, int32_t n,
                                                           const uint32_t* boff, int G, uint64_t* keys,
                                                           uint32_t* vals, const uint32_t* done, int reset) {
  __shared__ uint32_t sm[kCpThreads / kWave];
  __shared__ uint64_t skey[kCpTile];
  __shared__ uint32_t sval[kCpTile];
  if (*done) return;
  const int64_t base = (int64_t)blockIdx.x * kCpTile + (int64_t)threadIdx.x * kCpItems;
  int32_t t8[kCpItems];
  static_assert(kCpItems == 8, "two 16-byte loads per thread");
  if (base + kCpItems <= n && ((uintptr_t)ptgt & 15u) == 0) {
    const int4 a = *(const int4*)(ptgt + base), b = *(const int4*)(ptgt + base + 4);
    t8[0] = a.x, t8[1] = a.y, t8[2] = a.z, t8[3] = a.w, t8[4] = b.x, t8[5] = b.y, t8[6] = b.z, t8[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < kCpItems; ++i) t8[i] = base + i < n ? ptgt[base + i] : -1;
  }
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kCpItems; ++i) c += t8[i] >= 0 ? 1u : 0u;
  uint32_t tot;
  uint32_t incl = block_incl_scan_add<kCpThreads, uint32_t>(c, sm, &tot);
  // the block's proposals in vertex order, staged in LDS and written out by
  // consecutive threads
  uint32_t o = incl - c;
  const uint64_t dmax = (G >= 64) ? ~0ull : ((1ull << G) - 1);
#pragma unroll
  for (int i = 0; i < kCpItems; ++i) {
    const int64_t u = base + i;
    if (t8[i] >= 0) {
      skey[o] = ((uint64_t)(uint32_t)t8[i] << G) | (dmax - (uint64_t)pgain[u]);
      sval[o] = (uint32_t)u;
      ++o;
      if (reset) ptgt[u] = -1;
    }
  }
  __syncthreads();
  const uint32_t ob = boff[blockIdx.x];
  for (uint32_t j = threadIdx.x; j < tot; j += kCpThreads) {
    keys[ob + j] = skey[j];
    vals[ob + j] = sval[j];
  }
}

__global__ void k_admit_prep(const uint64_t* keys, const uint32_t* vals, const uint32_t* count, int G,
                             const int32_t* vwgt, uint32_t* seg, int64_t* wv) {
  const int64_t n = *count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    seg[i] = (uint32_t)(keys[i] >> G);
    wv[i] = vwgt ? vwgt[vals[i]] : 1;
  }
}

__global__ void k_admit(const uint32_t* seg, const int64_t* prefix, const uint32_t* count, const int64_t* W,
                        int64_t cap, const int32_t* gid, const int64_t* gcap, uint8_t* flag) {
  const int64_t n = *count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t t = seg[i];
    const int64_t c = gid ? gcap[gid[t]] : cap;
    flag[i] = (W[t] + prefix[i] <= c) ? 1 : 0;
  }
}

// The admitted proposals of a target are a prefix of its segment (the
// inclusive weight prefix grows along it), so the target's weight grows by
// the prefix at the last admitted one: one atomic per target, not per move.
__global__ __launch_bounds__(256) void k_apply(const uint32_t* seg, const uint32_t* vals, const uint8_t* flag,
                                               const int64_t* wv, const int64_t* prefix, const uint32_t* count,
                                               int32_t* C, int64_t* W, int64_t* stats, int round, int4* mv,
                                               int32_t* Cc, const int32_t* pos) {
  __shared__ int64_t sm[4];
  const int64_t n = *count;
  int64_t moves = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) {
      if (mv) mv[i] = make_int4(-1, 0, 0, 0);
      continue;
    }
    const int32_t u = (int32_t)vals[i];
    const int32_t t = (int32_t)seg[i];
    int32_t old;
    if (Cc) {
      // rating on the degree-ordered copy: only the copy's labels (indexed by
      // its vertices) change during the rounds; the caller's follow after
      // the last round (k_ro_labels)
      const int32_t pu = pos[u];
      old = Cc[pu];
      Cc[pu] = t;
    } else {
      old = C[u];
      C[u] = t;
    }
    if (mv) mv[i] = make_int4(u, old, t, 0);
    if (i + 1 == n || seg[i + 1] != (uint32_t)t || !flag[i + 1])
      atomicAdd((unsigned long long*)&W[t], (unsigned long long)prefix[i]);
    atomicAdd((unsigned long long*)&W[old], (unsigned long long)(-wv[i]));
    ++moves;
  }
  moves = block_reduce_add<256, int64_t>(moves, sm);
  if (threadIdx.x == 0 && moves && round < 64)
    atomicAdd((unsigned long long*)&stats[64 + round], (unsigned long long)moves);
}

// The caller's labels after rounds on the degree-ordered copy: vertex i of
// the copy is original vertex orig[i].
__global__ void k_ro_labels(int32_t n, const int32_t* orig, const int32_t* Cc, int32_t* C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    C[orig[i]] = Cc[i];
}

// End of a sub-round: its proposals count towards the round; after the
// round's last sub-round, a round without any proposal ends the call.
__global__ void k_round_end(const uint32_t* count, uint32_t* done, int64_t* stats, int round, int32_t* rounds_run,
                            unsigned long long* round_props, int last) {
  if (*done) return;
  const uint32_t c = *count;
  if (round < 64) stats[round] += c;
  *round_props += c;
  if (!last) return;
  if (*round_props == 0) *done = 1;
  else *rounds_run = round + 1;
  *round_props = 0;
}

// Bytes of the compressed records of the listed vertices.
__global__ void k_rec_bytes(const uint64_t* offs, const int32_t* idx, int32_t cnt, uint64_t* out) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
    out[i] = offs[idx[i] + 1] - offs[idx[i]];
}

__global__ void k_gather_i32(const int32_t* src, const int32_t* idx, int32_t cnt, int32_t* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = src[idx[i]];
}

__global__ void k_init(int32_t n, const int32_t* vwgt, int32_t* C, int64_t* W, int32_t* ptgt) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    C[u] = (int32_t)u;
    W[u] = vwgt ? vwgt[u] : 1;
    ptgt[u] = -1;
  }
}

// Start of a refinement: the given blocks stay as the labels; W[b] = weight
// of block b (W zeroed before), summed per workgroup in LDS when there are
// few blocks. A block outside [0, k) sets *bad and is not counted.
constexpr int kInitBins = 2048;
__global__ __launch_bounds__(256) void k_init_blocks(int32_t n, const int32_t* vwgt, const int32_t* C, int32_t k,
                                                     int64_t* W, int32_t* ptgt, uint32_t* bad) {
  __shared__ unsigned long long hist[kInitBins];
  const bool local = k <= kInitBins;
  if (local)
    for (int32_t i = threadIdx.x; i < k; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    ptgt[u] = -1;
    const int32_t c = C[u];
    if ((uint32_t)c >= (uint32_t)k) {
      *bad = 1u;
      continue;
    }
    const unsigned long long w = vwgt ? (unsigned long long)vwgt[u] : 1ull;
    if (local) atomicAdd(&hist[c], w);
    else atomicAdd((unsigned long long*)&W[c], w);
  }
  __syncthreads();
  if (local)
    for (int32_t i = threadIdx.x; i < k; i += blockDim.x)
      if (hist[i]) atomicAdd((unsigned long long*)&W[i], hist[i]);
}

int bitlen(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

template <typename F>
lp_status set_lds(F* kern, size_t bytes) {
  LP_CHECK_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return LP_OK;
}

// LDS layout of a rating group for degrees up to dmax.
// Side streams of the current device (created on first use, default
// priority, kept until the process ends). Host threads take sets in turn, so
// calls made at the same time from different threads (up to kSideSets of
// them) do not queue behind each other's side work; threads that share a set
// only add ordering, never a wrong result (every wait is on an event the same
// call recorded before).
constexpr int kSideSets = 4;
lp_status side_stream(int i, hipStream_t* out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static hipStream_t pool[kMaxDev][kSideSets][3] = {};
  static std::atomic<unsigned> next_set{0};
  thread_local const unsigned set = next_set.fetch_add(1) % kSideSets;
  int dev = 0;
  LP_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return LP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(mu);
  hipStream_t& st = pool[dev][set][i];
  if (!st) LP_CHECK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  *out = st;
  return LP_OK;
}

// Width of the LDS ratings of tiles: 16 bits for unit edge weights (a
// rating is at most the vertex's degree, at most 4096 on the tile paths),
// 64 bits when a weighted degree can exceed 2^31 - 1, else 32 bits. The
// narrower the table, the more workgroups share a compute unit.
enum class RateWidth { k16, k32, k64 };
inline RateWidth rate_width(const lp_graph* g) {
  if (g->max_wdeg > 0x7FFFFFFFll) return RateWidth::k64;
  return g->weighted ? RateWidth::k32 : RateWidth::k16;
}

template <class T, typename V, bool COMP, int MODE = kModeRate, bool ITV = false>
lp_status launch_tile(const RoundCtx& x, VDesc vd, const int32_t* tiles, const uint32_t* ntiles, uint32_t* ctr,
                      unsigned grid, bool weighted, hipStream_t s) {
  const TileLayout L = tile_layout<T, V>(COMP, weighted);
  const size_t bytes = (size_t)L.abytes + sizeof(TileShared<T::kThreads, T::kVerts>);
  auto kern = k_rate_tile<T, V, COMP, MODE, ITV>;
  LP_CHECK(set_lds(kern, bytes));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(T::kThreads), bytes, s, x, vd, tiles, ntiles, ctr, L);
  return last_error();
}

template <class T>
lp_status launch_tile_any(bool comp, RateWidth rw, const RoundCtx& x, VDesc vd, const int32_t* tiles,
                          const uint32_t* ntiles, uint32_t* ctr, unsigned grid, bool weighted, hipStream_t s) {
  if (comp && x.g.intervals) {
    if (rw == RateWidth::k16)
      return launch_tile<T, uint16_t, true, kModeRate, true>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
    if (rw == RateWidth::k64)
      return launch_tile<T, int64_t, true, kModeRate, true>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
    return launch_tile<T, int32_t, true, kModeRate, true>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
  }
  if (comp) {
    if (rw == RateWidth::k16) return launch_tile<T, uint16_t, true>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
    if (rw == RateWidth::k64) return launch_tile<T, int64_t, true>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
    return launch_tile<T, int32_t, true>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
  }
  if (rw == RateWidth::k16) return launch_tile<T, uint16_t, false>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
  if (rw == RateWidth::k64) return launch_tile<T, int64_t, false>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
  return launch_tile<T, int32_t, false>(x, vd, tiles, ntiles, ctr, grid, weighted, s);
}

template <class Cfg, typename V>
TileLayout piece_layout_of(bool comp, bool weighted) {
  TileLayout L;
  const uint32_t per = weighted ? 2u : 1u;
  L.table_bytes = (uint32_t)Cfg::kSlots * (4u + (uint32_t)sizeof(V));
  const uint32_t nums = comp ? (per * Cfg::kEdges + 7u * Cfg::kStreams) * 4u : 0u;
  const uint32_t worst = comp ? 5u * per * Cfg::kEdges + 16u * Cfg::kStreams : 0u;
  const uint32_t itv = comp ? (2u * Cfg::kStreams + 2u + 2u * ((uint32_t)Cfg::kEdges / 3u + 1u)) * 4u : 0u;
  uint32_t sb = worst;
  // a whole hub's staged bytes share the table's room: a hub whose record
  // does not fit is cut into pieces instead (whole_fits)
  if (Cfg::kWhole) sb = std::min(worst, L.table_bytes > nums ? L.table_bytes - nums : 0u);
  sb = std::max(sb, itv);
  L.stage_bytes = comp ? ((sb + 15u) & ~15u) : 0u;
  L.nums_off = L.stage_bytes;
  L.abytes = std::max(L.table_bytes, L.stage_bytes + nums);
  L.abytes = (L.abytes + 15u) & ~15u;
  return L;
}

// Whether a hub of degree d whose record takes `bytes` can be rated whole
// with the layout L of shape Cfg (dwords of up to kStreams streams staged).
template <class Cfg>
bool whole_fits(const TileLayout& L, bool comp, int64_t d, uint64_t bytes) {
  if (d > Cfg::kEdges) return false;
  return !comp || bytes + 8u * (uint64_t)Cfg::kStreams + 16u <= (uint64_t)L.stage_bytes;
}

// The lane kernel for the graph's format.
template <int MODE = kModeRate>
lp_status launch_lane(const RoundCtx& x, VDesc vd, int32_t cnt, hipStream_t s) {
  const bool comp = x.g.offs != nullptr;
  if (comp && x.g.intervals)
    hipLaunchKernelGGL((k_rate_lane<true, MODE, true>), dim3(grid_for(cnt, 256)), dim3(256), 0, s, x, vd, cnt);
  else if (comp)
    hipLaunchKernelGGL((k_rate_lane<true, MODE>), dim3(grid_for(cnt, 256)), dim3(256), 0, s, x, vd, cnt);
  else
    hipLaunchKernelGGL((k_rate_lane<false, MODE>), dim3(grid_for(cnt, 256)), dim3(256), 0, s, x, vd, cnt);
  return last_error();
}

template <class Cfg, typename V, int MODE = kModeRate>
lp_status launch_piece_t(const RoundCtx& x, const HubMeta& hm, int32_t npieces, uint32_t* ctr, hipStream_t s) {
  const bool comp = x.g.offs != nullptr;
  const TileLayout L = piece_layout_of<Cfg, V>(comp, x.g.weighted != 0);
  const size_t lds = (size_t)L.abytes + sizeof(PieceShared<Cfg>);
  auto kern = comp ? (x.g.intervals ? k_hub_piece<Cfg, V, true, MODE, true> : k_hub_piece<Cfg, V, true, MODE>)
                   : k_hub_piece<Cfg, V, false, MODE>;
  LP_CHECK(set_lds(kern, lds));
  const unsigned grid = grid_for(npieces, 1, Cfg::kWhole ? 1024 : 2048);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(Cfg::kThreads), lds, s, x, hm, npieces, ctr, L);
  return last_error();
}

// The pieces of the hubs that are cut (ratings of the graph's width).
template <int MODE = kModeRate>
lp_status launch_piece(bool wide, const RoundCtx& x, const HubMeta& hm, int32_t npieces, uint32_t* ctr,
                       hipStream_t s) {
  if (wide) return launch_piece_t<PieceHub, int64_t, MODE>(x, hm, npieces, ctr, s);
  return launch_piece_t<PieceHub, int32_t, MODE>(x, hm, npieces, ctr, s);
}

// The whole hubs: 16-bit ratings for unit edge weights, else 32-bit (graphs
// with 64-bit ratings have none).
template <int MODE = kModeRate>
lp_status launch_whole(bool weighted, const RoundCtx& x, const HubMeta& hw, int32_t nwhole, uint32_t* ctr,
                       hipStream_t s) {
  if (!weighted) return launch_piece_t<PieceWhole16, uint16_t, MODE>(x, hw, nwhole, ctr, s);
  return launch_piece_t<PieceWhole32, int32_t, MODE>(x, hw, nwhole, ctr, s);
}

// Tiles of one tile bucket, planned on the device (the count stays there).
struct TilePlan {
  int32_t* tiles = nullptr;
  uint32_t* ntiles = nullptr;
  unsigned grid = 0;
};

// Device memory of a plan, freed with the plan. For a handle whose buffers
// are stream-ordered the plan is too: taken from the memory cache on the
// building call's stream (which is synchronised before the plan is used
// elsewhere) and released in the order of the handle's stream.
struct PlanMem {
  std::vector<void*> ptrs;
  bool failed = false;
  bool stream_mem = false;
  hipStream_t alloc_stream = nullptr, free_stream = nullptr;
  template <typename T>
  T* alloc(size_t n) {
    void* p = nullptr;
    const size_t bytes = (n ? n : 1) * sizeof(T);
    if (stream_mem) p = cache_alloc(bytes, alloc_stream);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (!p) {
      clear_error();
      failed = true;
      return nullptr;
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  ~PlanMem() {
    for (void* p : ptrs) {
      if (stream_mem) cache_free(p, free_stream);
      else (void)hipFree(p);
    }
  }
};

template <class T>
lp_status plan_tiles(VDesc vd, int32_t cnt, bool comp, RateWidth rw, bool weighted, const int32_t* gid,
                     Scratch& sc, PlanMem& mem, TilePlan& tp) {
  if (cnt <= 0) return LP_OK;
  // the tiles run with the rating layout and, for the cut and the contraction
  // records, with the 32-bit one: the staged bytes must fit both
  TileLayout L = tile_layout<T, int32_t>(comp, weighted);
  const TileLayout Lr = rw == RateWidth::k16   ? tile_layout<T, uint16_t>(comp, weighted)
                        : rw == RateWidth::k64 ? tile_layout<T, int64_t>(comp, weighted)
                                               : L;
  L.stage_bytes = std::min(L.stage_bytes, Lr.stage_bytes);
  const int64_t nseg = ((int64_t)cnt + kTileSeg - 1) / kTileSeg;
  uint32_t* tcnt = sc.alloc<uint32_t>(nseg);
  tp.ntiles = mem.alloc<uint32_t>(1);
  tp.tiles = mem.alloc<int32_t>((size_t)cnt + 1);
  if (sc.failed || mem.failed) return LP_ENOMEM;
  hipStream_t s = sc.stream();
  hipLaunchKernelGGL(k_tile_plan<true>, dim3(grid_for(nseg, 256)), dim3(256), 0, s, vd, cnt, (uint32_t)T::kEdges,
                     (uint32_t)T::kVerts, L.stage_bytes, comp, gid, tcnt, (const uint32_t*)nullptr, (int32_t*)nullptr);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u32(tcnt, tcnt, nseg, tp.ntiles, sc));
  hipLaunchKernelGGL(k_tile_plan<false>, dim3(grid_for(nseg, 256)), dim3(256), 0, s, vd, cnt, (uint32_t)T::kEdges,
                     (uint32_t)T::kVerts, L.stage_bytes, comp, gid, (uint32_t*)nullptr, (const uint32_t*)tcnt, tp.tiles);
  LP_CHECK_LAUNCH();
  tp.grid = (unsigned)std::min<int64_t>(2048, ((int64_t)cnt + 7) / 8 * 8);
  return LP_OK;
}

}  // namespace

}  // namespace lp

using namespace lp;

namespace lp {
namespace {

// Everything about a graph that the rating, cut and record paths need and
// that depends only on the graph and the bucket thresholds: degree buckets
// (one stable vertex list ordered by (bucket, vertex)), vertex descriptors,
// the tiles of both tile buckets, and the hubs' pieces with their code
// streams. Built once per graph for the default thresholds and kept in the
// handle; other thresholds get a plan of their own for one call.
struct Plan {
  int32_t t_lane = 0, t_tile = 0, t_block = 0, hub_part = 0;
  int32_t sub_S = 1, sub_r = 0;  // the vertices of sub-round sub_r of sub_S (all when sub_S == 1)
  // plans of the sub-rounds, per sub-round count (kept by a cached plan; entries are never removed, so
  // pointers handed out stay valid while the handle lives)
  std::map<int32_t, std::vector<std::unique_ptr<Plan>>> subs;
  bool wide = false;
  int32_t bn[kNumBuckets] = {};
  uint32_t bstart[kNumBuckets + 1] = {};
  int32_t* order = nullptr;
  int32_t* deg = nullptr;  // degree of every vertex (also read by the contraction)
  int4* vdesc = nullptr;
  uint32_t* vlen = nullptr;
  TilePlan tps, tpl;
  HubMeta hm{};  // static parts only; per-call buffers are set by the caller
  HubMeta hw{};  // the hubs rated whole (u, deg, pieces, streams)
  int32_t H = 0, npieces = 0, ntasks = 0;  // hubs cut into pieces
  int32_t nwhole = 0;
  uint64_t rsum = 0, psum = 0;
  unsigned long long bsums[2 * kNumBuckets] = {};
  PlanMem mem;
  uint32_t* vnum = nullptr;  // interval-coded graphs: VarInts of every listed vertex
  VDesc vd(int b) const { return VDesc{vdesc + bstart[b], vlen + bstart[b], vnum ? vnum + bstart[b] : nullptr}; }
};

lp_status build_plan(const lp_graph* g, int32_t t_lane, int32_t t_tile, int32_t t_block, int32_t hub_part,
                     hipStream_t s, Plan& P, int32_t sub_S = 1, int32_t sub_r = 0) {
  const int32_t n = g->n;
  // interval-coded records above LP_ITV_CHUNK_THRESHOLD are chunked: the hub
  // path rates them, whatever the tile bucket's bound
  if (g->intervals && t_block > LP_ITV_CHUNK_THRESHOLD) t_block = LP_ITV_CHUNK_THRESHOLD;
  if (t_tile > t_block) t_tile = t_block;
  P.sub_S = sub_S;
  P.sub_r = sub_r;
  P.t_lane = t_lane;
  P.t_tile = t_tile;
  P.t_block = t_block;
  P.hub_part = hub_part;
  P.wide = g->max_wdeg > 0x7FFFFFFFll;
  const bool batch = g->nbatch > 0;
  P.mem.stream_mem = g->stream_mem;
  P.mem.alloc_stream = s;
  P.mem.free_stream = g->mem_stream;
  Scratch sc(s);
  int32_t* deg = sub_S > 1 ? sc.alloc<int32_t>(n) : P.mem.alloc<int32_t>(n);
  if (sub_S == 1) P.deg = deg;
  const unsigned nbk = grid_for(n, kBkTile, 0x7FFFFFFF);
  uint32_t* bcnt = sc.alloc<uint32_t>((size_t)kNumBuckets * nbk);
  uint32_t* btot = sc.alloc<uint32_t>(1);
  unsigned long long* bsums = sc.alloc<unsigned long long>(2 * kNumBuckets);
  P.order = P.mem.alloc<int32_t>(n);
  if (sc.failed || P.mem.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(bsums, 0, 2 * kNumBuckets * sizeof(unsigned long long), s));
  LP_CHECK(compute_degrees(g, deg, s));
  if (sub_S > 1) {  // bucket only this sub-round's vertices; P.deg keeps every degree
    int32_t* dsub = sc.alloc<int32_t>(n);
    if (!dsub) return LP_ENOMEM;
    hipLaunchKernelGGL(k_subround_deg, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, deg, n, (uint32_t)sub_S,
                       (uint32_t)sub_r, batch ? g->gid : nullptr, batch ? g->gbase : nullptr, dsub);
    LP_CHECK_LAUNCH();
    deg = dsub;
  }
  hipLaunchKernelGGL(k_bucket_count, dim3(nbk), dim3(kBkThreads), 0, s, deg, n, t_lane, t_tile, t_block, bcnt, nbk);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u32(bcnt, bcnt, (int64_t)kNumBuckets * nbk, btot, sc));
  hipLaunchKernelGGL(k_bucket_scatter, dim3(nbk), dim3(kBkThreads), 0, s, deg, n, t_lane, t_tile, t_block, bcnt, nbk,
                     P.order);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_bucket_sums, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, deg, n, t_lane, t_tile, t_block,
                     g->compressed ? g->offs : nullptr, bsums);
  LP_CHECK_LAUNCH();
  for (int b = 0; b < kNumBuckets; ++b)
    LP_CHECK_HIP(hipMemcpyAsync(&P.bstart[b], bcnt + (size_t)b * nbk, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipMemcpyAsync(&P.bstart[kNumBuckets], btot, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipMemcpyAsync(P.bsums, bsums, sizeof(P.bsums), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < kNumBuckets; ++b) P.bn[b] = (int32_t)(P.bstart[b + 1] - P.bstart[b]);

  // descriptors of the non-hub buckets
  const int32_t nlisted = (int32_t)P.bstart[3];
  P.vdesc = P.mem.alloc<int4>(nlisted);
  P.vlen = P.mem.alloc<uint32_t>(nlisted);
  if (g->intervals) P.vnum = P.mem.alloc<uint32_t>(nlisted);
  if (P.mem.failed) return LP_ENOMEM;
  if (nlisted > 0) {
    hipLaunchKernelGGL(k_build_desc, dim3(grid_for(nlisted, 256, 65536)), dim3(256), 0, s, g->view(), P.order, deg,
                       nlisted, P.vdesc, P.vlen, P.vnum);
    LP_CHECK_LAUNCH();
  }
  // tiles of the two tile buckets
  const int32_t* gid = batch ? g->gid : nullptr;
  LP_CHECK(plan_tiles<TileSmall>(P.vd(1), P.bn[1], g->compressed, rate_width(g), g->weighted, gid, sc, P.mem, P.tps));
  LP_CHECK(plan_tiles<TileLarge>(P.vd(2), P.bn[2], g->compressed, rate_width(g), g->weighted, gid, sc, P.mem, P.tpl));

  // hubs: metadata (host-built, small) and the code streams of their pieces.
  // A hub whose record fits one workgroup's LDS is rated whole; the others
  // are cut into pieces.
  const int32_t Hall = P.bn[3];
  P.H = 0;
  P.nwhole = 0;
  if (Hall > 0) {
    std::vector<int32_t> au(Hall), ad(Hall);
    std::vector<uint64_t> ab(Hall, 0);
    int32_t* hdeg_dev = sc.alloc<int32_t>(Hall);
    uint64_t* hbytes_dev = sc.alloc<uint64_t>(Hall);
    if (!hdeg_dev || !hbytes_dev) return LP_ENOMEM;
    hipLaunchKernelGGL(k_gather_i32, dim3(grid_for(Hall, 256, 4096)), dim3(256), 0, s, deg, P.order + P.bstart[3],
                       Hall, hdeg_dev);
    LP_CHECK_LAUNCH();
    if (g->compressed) {
      hipLaunchKernelGGL(k_rec_bytes, dim3(grid_for(Hall, 256, 4096)), dim3(256), 0, s, g->offs,
                         P.order + P.bstart[3], Hall, hbytes_dev);
      LP_CHECK_LAUNCH();
      LP_CHECK_HIP(hipMemcpyAsync(ab.data(), hbytes_dev, Hall * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    }
    LP_CHECK_HIP(hipMemcpyAsync(au.data(), P.order + P.bstart[3], Hall * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LP_CHECK_HIP(hipMemcpyAsync(ad.data(), hdeg_dev, Hall * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LP_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> hu, hd, wu, wd;
    const bool comp = g->compressed != 0;
    const TileLayout WL = g->weighted ? piece_layout_of<PieceWhole32, int32_t>(comp, true)
                                      : piece_layout_of<PieceWhole16, uint16_t>(comp, false);
    for (int32_t i = 0; i < Hall; ++i) {
      const bool whole = !P.wide && (g->weighted ? whole_fits<PieceWhole32>(WL, comp, ad[i], ab[i])
                                                 : whole_fits<PieceWhole16>(WL, comp, ad[i], ab[i]));
      (whole ? wu : hu).push_back(au[i]);
      (whole ? wd : hd).push_back(ad[i]);
    }
    const int32_t H = (int32_t)hu.size();
    const int32_t HW = (int32_t)wu.size();
    P.H = H;
    P.nwhole = HW;
    if (HW > 0) {
      HubMeta& hw = P.hw;
      const int NSW = g->weighted ? PieceWhole32::kStreams : PieceWhole16::kStreams;
      std::vector<int32_t> ones(HW, 1), idx(HW);
      std::vector<int2> wp(HW);
      for (int32_t i = 0; i < HW; ++i) {
        idx[i] = i;
        wp[i] = make_int2(i, 0);
      }
      int32_t* d_u = P.mem.alloc<int32_t>(HW);
      int32_t* d_deg = P.mem.alloc<int32_t>(HW);
      int32_t* d_one = P.mem.alloc<int32_t>(HW);
      int32_t* d_idx = P.mem.alloc<int32_t>(HW);
      int2* d_wp = P.mem.alloc<int2>(HW);
      hw.streams = P.mem.alloc<HubStream>((size_t)HW * NSW);
      if (P.mem.failed) return LP_ENOMEM;
      LP_CHECK_HIP(hipMemcpyAsync(d_u, wu.data(), HW * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_deg, wd.data(), HW * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_one, ones.data(), HW * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_idx, idx.data(), HW * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_wp, wp.data(), HW * sizeof(int2), hipMemcpyHostToDevice, s));
      hw.u = d_u;
      hw.deg = d_deg;
      hw.npieces = d_one;
      hw.piece_base = d_idx;
      hw.pieces = d_wp;
      if (g->weighted)
        hipLaunchKernelGGL(k_hub_streams<PieceWhole32>, dim3(grid_for(HW, 4, 4096)), dim3(256), 0, s, g->view(), hw,
                           HW);
      else
        hipLaunchKernelGGL(k_hub_streams<PieceWhole16>, dim3(grid_for(HW, 4, 4096)), dim3(256), 0, s, g->view(), hw,
                           HW);
      LP_CHECK_LAUNCH();
    }
    if (H > 0) {
      // partitions of about hub_part records (at most kMaxParts)
      std::vector<int32_t> np(H), npc(H), pcb(H), tb(H);
      std::vector<uint64_t> rbase(H), pbase(H);
      std::vector<int2> pieces;
      std::vector<HubTask> tasks;
      uint64_t rsum = 0, psum = 0;
      int32_t ntasks = 0;
      for (int h = 0; h < H; ++h) {
        const int64_t d = hd[h];
        np[h] = (int32_t)std::min<int64_t>(kMaxParts, std::max<int64_t>(1, (d + hub_part - 1) / hub_part));
        npc[h] = (int32_t)((d + kHubPiece - 1) / kHubPiece);
        pcb[h] = (int32_t)pieces.size();
        rbase[h] = rsum;
        pbase[h] = psum;
        tb[h] = ntasks;
        rsum += (uint64_t)d;
        psum += (uint64_t)npc[h] * (np[h] + 1);
        ntasks += np[h];
        for (int k = 0; k < npc[h]; ++k) pieces.push_back(make_int2(h, k));
        for (int p = 0; p < np[h]; ++p) tasks.push_back(HubTask{hu[h], np[h], npc[h], p, rbase[h], pbase[h]});
      }
      P.npieces = (int32_t)pieces.size();
      P.ntasks = ntasks;
      P.rsum = rsum;
      P.psum = psum;
      HubMeta& hm = P.hm;
      int32_t* d_u = P.mem.alloc<int32_t>(H);
      int32_t* d_deg = P.mem.alloc<int32_t>(H);
      int32_t* d_np = P.mem.alloc<int32_t>(H);
      int32_t* d_npc = P.mem.alloc<int32_t>(H);
      int32_t* d_pcb = P.mem.alloc<int32_t>(H);
      int32_t* d_tb = P.mem.alloc<int32_t>(H);
      uint64_t* d_rb = P.mem.alloc<uint64_t>(H);
      uint64_t* d_pb = P.mem.alloc<uint64_t>(H);
      int2* d_pieces = P.mem.alloc<int2>(P.npieces);
      HubTask* d_tasks = P.mem.alloc<HubTask>(ntasks);
      hm.streams = P.mem.alloc<HubStream>((size_t)P.npieces * kHubStreams);
      if (P.mem.failed) return LP_ENOMEM;
      LP_CHECK_HIP(hipMemcpyAsync(d_u, hu.data(), H * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_deg, hd.data(), H * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_np, np.data(), H * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_npc, npc.data(), H * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_pcb, pcb.data(), H * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_tb, tb.data(), H * sizeof(int32_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_rb, rbase.data(), H * sizeof(uint64_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_pb, pbase.data(), H * sizeof(uint64_t), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_pieces, pieces.data(), P.npieces * sizeof(int2), hipMemcpyHostToDevice, s));
      LP_CHECK_HIP(hipMemcpyAsync(d_tasks, tasks.data(), ntasks * sizeof(HubTask), hipMemcpyHostToDevice, s));
      hm.u = d_u;
      hm.deg = d_deg;
      hm.nparts = d_np;
      hm.npieces = d_npc;
      hm.piece_base = d_pcb;
      hm.rec_base = d_rb;
      hm.poff_base = d_pb;
      hm.task_base = d_tb;
      hm.pieces = d_pieces;
      hm.tdesc = d_tasks;
      hipLaunchKernelGGL(k_hub_streams<PieceHub>, dim3(grid_for(H, 4, 4096)), dim3(256), 0, s, g->view(), hm, H);
      LP_CHECK_LAUNCH();
    }
  }
  LP_CHECK_HIP(hipStreamSynchronize(s));  // host vectors go out of scope; the plan is complete
  return LP_OK;
}

void plan_delete(void* p) { delete (Plan*)p; }

lp_status get_plan(const lp_graph* g, int32_t t_lane, int32_t t_tile, int32_t t_block, int32_t hub_part,
                   hipStream_t s, const Plan** out, std::unique_ptr<Plan>& tmp);

// Labels of the degree-ordered copy: vertex i of the copy is vertex orig[i].
__global__ void k_permute_labels(int32_t n, const int32_t* orig, const int32_t* C, int32_t* Cp) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Cp[i] = C[orig[i]];
}

__global__ void k_zero_u32(uint32_t* a, int32_t n) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = 0;
}

// One visit of every edge with the default plan: the cut (MODE == kModeCut)
// or the contraction records (kModeRec). The lane, tile and piece kernels
// decode exactly as for rating and stop after the label (or map) gather.
// With `counters` given (32 words of the caller's memory), the visit
// allocates nothing: it uses the plan the handle already holds (LP_EINVAL if
// no earlier call built it) and those counters instead of scratch.
//
// A handle whose degree-ordered copy exists (built by an earlier clustering
// call) is visited on the copy, whose gathers touch fewer lines: the labels
// (map) are permuted to the copy's numbering, and records still go to the
// slices of the original vertices. The allocation-free visit keeps to the
// graph as given.
template <int MODE>
lp_status visit_edges_mode(const lp_graph* g, const int32_t* C, const uint64_t* rbase, const uint64_t* voff, Rec* rec,
                           unsigned long long* cut, hipStream_t s, uint32_t* counters = nullptr) {
  Scratch sc(s);
  const Reorder* ro = counters ? nullptr : existing_reorder(g);
  if (ro) {
    int32_t* Cp = sc.alloc<int32_t>(g->n);
    if (!Cp) return LP_ENOMEM;
    hipLaunchKernelGGL(k_permute_labels, dim3(grid_for(g->n, 256, 65536)), dim3(256), 0, s, g->n, ro->orig, C, Cp);
    LP_CHECK_LAUNCH();
    C = Cp;
    g = ro->g;
  }
  const Plan* plan = nullptr;
  std::unique_ptr<Plan> tmp;
  if (counters) {
    std::lock_guard<std::mutex> lock(g->plan_mu);
    plan = (const Plan*)g->plan;
    if (!plan) return LP_EINVAL;
  } else {
    LP_CHECK(get_plan(g, 16, kTileMaxDeg, TileLarge::kEdges, kDefaultHubPart, s, &plan, tmp));
  }
  // zero[0]: the round's "done" flag (never set here); zero[8..32): hand-out
  // counters of the small tiles, the large tiles and the pieces
  uint32_t* zero = counters ? counters : sc.alloc<uint32_t>(32);
  if (!zero) return LP_ENOMEM;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, zero, 32);
  LP_CHECK_LAUNCH();
  RoundCtx x{};
  x.g = g->view();
  x.C = C;
  x.done = zero;
  x.rbase = rbase;
  x.voff = voff;
  x.rec = rec;
  x.cut = cut;
  x.pmap = ro ? ro->orig : nullptr;
  x.rec_sum = MODE == kModeRec && g->max_wdeg <= 0x7FFFFFFFll ? 1 : 0;
  const bool comp = g->compressed;
  if (plan->bn[0] > 0) {
    const VDesc vd = plan->vd(0);
    const int32_t c = plan->bn[0];
    LP_CHECK(launch_lane<MODE>(x, vd, c, s));
  }
  if (plan->bn[1] > 0) {
    if (comp && g->intervals)
      LP_CHECK((launch_tile<TileSmall, int32_t, true, MODE, true>(x, plan->vd(1), plan->tps.tiles, plan->tps.ntiles,
                                                                  zero + 8, plan->tps.grid, g->weighted, s)));
    else if (comp)
      LP_CHECK((launch_tile<TileSmall, int32_t, true, MODE>(x, plan->vd(1), plan->tps.tiles, plan->tps.ntiles,
                                                            zero + 8, plan->tps.grid, g->weighted, s)));
    else
      LP_CHECK((launch_tile<TileSmall, int32_t, false, MODE>(x, plan->vd(1), plan->tps.tiles, plan->tps.ntiles,
                                                             zero + 8, plan->tps.grid, g->weighted, s)));
  }
  if (plan->bn[2] > 0) {
    if (comp && g->intervals)
      LP_CHECK((launch_tile<TileLarge, int32_t, true, MODE, true>(x, plan->vd(2), plan->tpl.tiles, plan->tpl.ntiles,
                                                                  zero + 16, plan->tpl.grid, g->weighted, s)));
    else if (comp)
      LP_CHECK((launch_tile<TileLarge, int32_t, true, MODE>(x, plan->vd(2), plan->tpl.tiles, plan->tpl.ntiles,
                                                            zero + 16, plan->tpl.grid, g->weighted, s)));
    else
      LP_CHECK((launch_tile<TileLarge, int32_t, false, MODE>(x, plan->vd(2), plan->tpl.tiles, plan->tpl.ntiles,
                                                             zero + 16, plan->tpl.grid, g->weighted, s)));
  }
  if (plan->nwhole > 0) LP_CHECK(launch_whole<MODE>(g->weighted, x, plan->hw, plan->nwhole, zero + 28, s));
  if (plan->H > 0) LP_CHECK(launch_piece<MODE>(false, x, plan->hm, plan->npieces, zero + 24, s));
  return LP_OK;
}

// The plan for these thresholds: the handle's cached one for the defaults
// (built on first use), otherwise a new one owned by `tmp`.
lp_status get_plan(const lp_graph* g, int32_t t_lane, int32_t t_tile, int32_t t_block, int32_t hub_part,
                   hipStream_t s, const Plan** out, std::unique_ptr<Plan>& tmp) {
  const bool dflt = t_lane == 16 && t_tile == kTileMaxDeg && t_block == TileLarge::kEdges &&
                    hub_part == kDefaultHubPart;
  if (!dflt) {
    tmp.reset(new Plan());
    LP_CHECK(build_plan(g, t_lane, t_tile, t_block, hub_part, s, *tmp));
    tmp->mem.free_stream = s;  // used by this call only
    *out = tmp.get();
    return LP_OK;
  }
  std::lock_guard<std::mutex> lock(g->plan_mu);
  if (!g->plan) {
    std::unique_ptr<Plan> p(new Plan());
    LP_CHECK(build_plan(g, t_lane, t_tile, t_block, hub_part, s, *p));
    g->plan = p.release();
    const_cast<lp_graph*>(g)->plan_free = plan_delete;
  }
  *out = (const Plan*)g->plan;
  return LP_OK;
}

}  // namespace

lp_status batch_localize(const lp_graph* b, const int32_t* lab, int32_t* out, int32_t* const* outs_dev,
                         hipStream_t s);

// The plans of a call with S sub-rounds: the plan itself for S == 1, else
// one plan per sub-round over that sub-round's vertices (kept with the
// handle's cached plan for the default thresholds, owned by `tmp` otherwise).
lp_status get_plans(const lp_graph* g, int32_t t_lane, int32_t t_tile, int32_t t_block, int32_t hub_part, int32_t S,
                    hipStream_t s, std::vector<const Plan*>& out, std::unique_ptr<Plan>& tmp) {
  out.clear();
  const Plan* base = nullptr;
  LP_CHECK(get_plan(g, t_lane, t_tile, t_block, hub_part, s, &base, tmp));
  if (S == 1) {
    out.push_back(base);
    return LP_OK;
  }
  Plan* owner = const_cast<Plan*>(base);  // sub-plans only ever get added
  std::unique_lock<std::mutex> lock(g->plan_mu, std::defer_lock);
  if (!tmp) lock.lock();  // the handle's cached plan is shared
  auto& v = owner->subs[S];
  if (v.empty()) {
    std::vector<std::unique_ptr<Plan>> built;
    for (int32_t r = 0; r < S; ++r) {
      std::unique_ptr<Plan> p(new Plan());
      LP_CHECK(build_plan(g, t_lane, t_tile, t_block, hub_part, s, *p, S, r));
      if (tmp) p->mem.free_stream = s;  // used by this call only
      built.push_back(std::move(p));
    }
    v = std::move(built);
  }
  for (auto& p : v) out.push_back(p.get());
  return LP_OK;
}

lp_status plan_degrees(const lp_graph* g, const int32_t** deg, hipStream_t s) {
  const Plan* plan = nullptr;
  std::unique_ptr<Plan> tmp;
  LP_CHECK(get_plan(g, 16, kTileMaxDeg, TileLarge::kEdges, kDefaultHubPart, s, &plan, tmp));
  *deg = plan->deg;
  return LP_OK;
}

lp_status visit_edges_cut(const lp_graph* g, const int32_t* labels, unsigned long long* cut, hipStream_t s) {
  if (g->n == 0) return LP_OK;
  return visit_edges_mode<kModeCut>(g, labels, nullptr, nullptr, nullptr, cut, s);
}

lp_status visit_edges_cut_noalloc(const lp_graph* g, const int32_t* labels, unsigned long long* cut,
                                  uint32_t* counters, hipStream_t s) {
  if (g->n == 0) return LP_OK;
  return visit_edges_mode<kModeCut>(g, labels, nullptr, nullptr, nullptr, cut, s, counters);
}

lp_status visit_edges_records(const lp_graph* g, const int32_t* map, const uint64_t* rbase, const uint64_t* voff,
                              Rec* rec, hipStream_t s) {
  if (g->n == 0) return LP_OK;
  return visit_edges_mode<kModeRec>(g, map, rbase, voff, rec, nullptr, s);
}
}

// One clustering call. For a batch handle, caps / seeds hold one value per
// graph (host arrays) and the labels come out local to each graph: written to
// `labels` (one array over the union) or, if labels_each is given, to each
// graph's own device array.
// init_k == 0: clustering, every vertex starts in its own cluster. init_k > 0:
// refinement, labels hold a partition into init_k blocks on entry.
static lp_status cluster_impl(const lp_graph* g, int64_t cap, const int64_t* caps, int32_t rounds, uint64_t seed,
                              const uint64_t* seeds, int32_t* labels, int32_t* const* labels_each,
                              const lp_config* cfg_in, lp_cluster_stats* stats_out, hipStream_t s,
                              int32_t init_k = 0) {
  const bool batch = g->nbatch > 0;
  if (batch) {
    if (!caps || !seeds) return LP_EINVAL;
    for (int32_t i = 0; i < g->nbatch; ++i)
      if (caps[i] < 1) return LP_EINVAL;
  } else if (cap < 1) {
    return LP_EINVAL;
  }
  if (rounds < 0 || (!labels && !labels_each && g->n > 0)) return LP_EINVAL;
  if (stats_out) memset(stats_out, 0, sizeof(*stats_out));
  const int32_t n = g->n;
  if (init_k < 0 || (init_k > 0 && (batch || init_k > std::max(n, 1)))) return LP_EINVAL;
  if (n == 0) return LP_OK;
  // knobs (results do not depend on them)
  const bool wide = g->max_wdeg > 0x7FFFFFFFll;
  int32_t t_lane = 16, t_tile = kTileMaxDeg, t_block = TileLarge::kEdges, hub_part = kDefaultHubPart;
  int32_t S = 1;  // sub-rounds per round (this one changes the result)
  const bool use_gt = cfg_in && cfg_in->gain_table;  // refinement only: rate from a gain table
  if (use_gt && init_k == 0) return LP_EINVAL;
  if (cfg_in) {
    if (cfg_in->t_lane) t_lane = cfg_in->t_lane;
    if (cfg_in->t_tile) t_tile = cfg_in->t_tile;
    if (cfg_in->t_block) t_block = cfg_in->t_block;
    if (cfg_in->hub_part) hub_part = cfg_in->hub_part;
    if (cfg_in->subrounds) S = cfg_in->subrounds;
  }
  if (t_lane < 0 || t_lane > kMaxLane || t_tile < t_lane || t_tile > kTileMaxDeg || t_block < t_tile ||
      t_block > TileLarge::kEdges || hub_part < 256 || hub_part > 8192 || S < 1 || S > kMaxSubrounds)
    return LP_EINVAL;
  // proposal sort key: target bits + gain bits
  const int G = std::max(1, bitlen((uint64_t)g->max_wdeg));
  const int nbits = std::max(1, bitlen((uint64_t)(n - 1)));
  if (G + nbits > 64) return LP_EUNSUPPORTED;

  Scratch sc(s);
  int32_t* out_labels = labels;
  if (batch) labels = sc.alloc<int32_t>(n);  // global cluster IDs while the rounds run
  int64_t* gcap = batch ? sc.alloc<int64_t>(g->nbatch) : nullptr;
  uint64_t* gseed = batch ? sc.alloc<uint64_t>(g->nbatch) : nullptr;
  int64_t* W = sc.alloc<int64_t>(n);
  int32_t* ptgt = sc.alloc<int32_t>(n);
  int64_t* pgain = sc.alloc<int64_t>(n);
  uint64_t* ka = sc.alloc<uint64_t>(n);
  uint64_t* kb = sc.alloc<uint64_t>(n);
  uint32_t* va = sc.alloc<uint32_t>(n);
  uint32_t* vb = sc.alloc<uint32_t>(n);
  uint32_t* seg = sc.alloc<uint32_t>(n);
  int64_t* wv = sc.alloc<int64_t>(n);
  int64_t* pref = sc.alloc<int64_t>(n);
  uint8_t* flag = sc.alloc<uint8_t>(n);
  int4* mv = use_gt ? sc.alloc<int4>(n) : nullptr;
  const unsigned ncp = grid_for(n, kCpTile, 0x7FFFFFFF);
  uint32_t* pcnt = sc.alloc<uint32_t>(ncp);
  // per sub-round: hand-out counters of the small tiles, large tiles and pieces
  const int64_t nhand = (int64_t)std::max(rounds, 1) * S * 24;
  uint32_t* hand = sc.alloc<uint32_t>(nhand);
  struct Ctl {
    uint32_t done;
    uint32_t count;
    int32_t rounds_run;
    uint32_t bad;  // a refinement block out of range
    uint32_t bucket_tot[4];
    unsigned long long round_props;
    int64_t stats[128];
  };
  Ctl* ctl = sc.alloc<Ctl>(1);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(ctl, 0, sizeof(Ctl), s));
  hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(nhand, 256, 64)), dim3(256), 0, s, hand, (int32_t)nhand);
  LP_CHECK_LAUNCH();
  if (batch) {
    LP_CHECK_HIP(hipMemcpyAsync(gcap, caps, g->nbatch * sizeof(int64_t), hipMemcpyHostToDevice, s));
    LP_CHECK_HIP(hipMemcpyAsync(gseed, seeds, g->nbatch * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  }

  // optional per-phase timing with events on the call's stream
  const bool timing = cfg_in && cfg_in->timing && stats_out;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  struct EventGuard {
    std::vector<Mark>* m;
    ~EventGuard() {
      for (auto& k : *m) {
        (void)hipEventDestroy(k.a);
        (void)hipEventDestroy(k.b);
      }
    }
  } guard{&marks};
  auto begin = [&](int phase, hipStream_t on = nullptr) -> lp_status {
    if (!timing) return LP_OK;
    Mark m{phase, nullptr, nullptr};
    LP_CHECK_HIP(hipEventCreate(&m.a));
    LP_CHECK_HIP(hipEventCreate(&m.b));
    marks.push_back(m);
    LP_CHECK_HIP(hipEventRecord(m.a, on ? on : s));
    return LP_OK;
  };
  auto end = [&](hipStream_t on = nullptr) -> lp_status {
    if (!timing) return LP_OK;
    LP_CHECK_HIP(hipEventRecord(marks.back().b, on ? on : s));
    return LP_OK;
  };
  // a phase that encloses others: closed by the index begin() gave it
  auto end_at = [&](size_t idx, hipStream_t on = nullptr) -> lp_status {
    if (!timing) return LP_OK;
    LP_CHECK_HIP(hipEventRecord(marks[idx].b, on ? on : s));
    return LP_OK;
  };
  // The rating paths of a round are independent (they read the snapshot and
  // write disjoint vertices). By default they run one after another on the
  // call's stream (each kernel already fills the device); with
  // lp_config.overlap they run on side streams forked from and joined back
  // into the call's stream, so that their kernels overlap.
  const bool overlap = cfg_in && cfg_in->overlap;
  hipStream_t side[3] = {s, s, s};
  if (overlap)
    for (int i = 0; i < 3; ++i) LP_CHECK(side_stream(i, &side[i]));
  struct EvGuard {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~EvGuard() {
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  if (overlap)
    for (int i = 0; i < 4; ++i) LP_CHECK_HIP(hipEventCreateWithFlags(&ev.e[i], hipEventDisableTiming));
  // Joins the side streams back into the call's stream when a call returns
  // between fork and join (an error), so that no kernel still running on a
  // side stream outlives the scratch memory released on the call's stream.
  // Declared after the scratch, so it runs before the scratch is released.
  struct JoinGuard {
    hipStream_t s;
    hipStream_t* side;
    hipEvent_t* e;
    bool forked = false;
    void join() {
      if (!forked) return;
      for (int i = 0; i < 3; ++i) {
        (void)hipEventRecord(e[i], side[i]);
        (void)hipStreamWaitEvent(s, e[i], 0);
      }
      forked = false;
    }
    ~JoinGuard() { join(); }
  } jg{s, side, ev.e};

  LP_CHECK(begin(LP_PHASE_SETUP));
  // Rating on a degree-ordered copy of the graph (result-invariant, reorder.h):
  // the copy's labels hold the original cluster IDs (tie-break keys and
  // cluster weights need no translation), proposals land at the original
  // vertices, so acceptance orders them exactly as on the graph as given;
  // apply keeps both label arrays. The handle's own default plan is built as
  // well, for the edge visits (cut, contraction) on the original graph.
  const int32_t ro_mode = cfg_in ? cfg_in->reorder : 0;
  if (ro_mode < 0 || ro_mode > 2) return LP_EINVAL;
  // automatic: large graphs with a skewed degree distribution (a graph whose
  // IDs already follow its geometry, like the cell-ordered RGGs, loses that
  // locality when renumbered by degree), from the second clustering of a
  // handle the caller made (the build costs about as much as 15 rounds: a
  // graph clustered once, like a coarse level, would not repay it)
  const int32_t calls = init_k == 0 && !batch ? g->cluster_calls.fetch_add(1) + 1 : 0;
  const bool skewed = g->max_deg >= 32 * (int64_t)((g->two_m + n - 1) / n);
  const bool use_ro = ro_mode != 2 && init_k == 0 && !batch && !use_gt && S == 1 && reorder_applies(g) &&
                      (ro_mode == 1 || (n >= (1 << 20) && skewed && !g->stream_mem && (calls >= 2 || g->reord)));
  const Reorder* ro = nullptr;
  int32_t* Cc = nullptr;
  if (use_ro) {
    LP_CHECK(get_reorder(g, s, &ro));
    const Plan* p0;
    std::unique_ptr<Plan> t0;
    LP_CHECK(get_plan(g, 16, kTileMaxDeg, TileLarge::kEdges, kDefaultHubPart, s, &p0, t0));
    Cc = sc.alloc<int32_t>(n);
    if (!Cc) return LP_ENOMEM;
  }
  const lp_graph* gr = use_ro ? ro->g : g;  // the graph the rating kernels read
  std::vector<const Plan*> plans;  // one per sub-round
  std::unique_ptr<Plan> plan_tmp;
  LP_CHECK(get_plans(gr, t_lane, t_tile, t_block, hub_part, S, s, plans, plan_tmp));
  uint64_t rsum = 0, psum = 0;
  int32_t tmax = 0, hmax = 0;
  for (const Plan* p : plans) {
    rsum = std::max(rsum, p->rsum);
    psum = std::max(psum, p->psum);
    tmax = std::max(tmax, p->ntasks);
    hmax = std::max(hmax, p->H);
  }
  HubMeta hbuf{};  // per-call hub buffers, shared by the sub-rounds
  if (hmax > 0) {
    // packed records for unit edge weights: a cluster ID below n needs
    // bitlen(n - 1) bits, the rest of the word holds the partial rating
    hbuf.packed = (!g->weighted && !wide) ? 1 : 0;
    hbuf.rbits = (uint32_t)(32 - std::max(1, bitlen((uint64_t)(n - 1))));
    hbuf.rec_c = sc.alloc<int32_t>(rsum);
    hbuf.rec_r = hbuf.packed ? nullptr : wide ? (void*)sc.alloc<int64_t>(rsum) : (void*)sc.alloc<int32_t>(rsum);
    hbuf.poff = sc.alloc<uint32_t>(psum);
    hbuf.res_r = sc.alloc<int64_t>(tmax);
    hbuf.res_key = sc.alloc<uint64_t>(tmax);
    hbuf.res_c = sc.alloc<int32_t>(tmax);
    hbuf.res_own = sc.alloc<int64_t>(tmax);
    if (sc.failed) return LP_ENOMEM;
  }

  struct GtGuard {
    GainTable t;
    hipStream_t s;
    ~GtGuard() {
      if (t.off) gt_release(&t, s);
    }
  } gt{GainTable{}, s};
  if (init_k > 0) {
    LP_CHECK_HIP(hipMemsetAsync(W, 0, (size_t)n * sizeof(int64_t), s));
    hipLaunchKernelGGL(k_init_blocks, dim3(grid_for(n, 256, 512)), dim3(256), 0, s, n, g->vwgt, labels, init_k, W,
                       ptgt, &ctl->bad);
    LP_CHECK_LAUNCH();
    uint32_t bad = 0;
    LP_CHECK_HIP(hipMemcpyAsync(&bad, &ctl->bad, sizeof(bad), hipMemcpyDeviceToHost, s));
    LP_CHECK_HIP(hipStreamSynchronize(s));
    if (bad) return LP_EINVAL;
    if (use_gt) LP_CHECK(gt_create(g, labels, init_k, s, &gt.t));
  } else {
    hipLaunchKernelGGL(k_init, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, g->vwgt, labels, W, ptgt);
    LP_CHECK_LAUNCH();
    // the copy's labels: vertex i starts in the cluster of its original ID
    if (use_ro) LP_CHECK_HIP(hipMemcpyAsync(Cc, ro->orig, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  LP_CHECK(end());

  RoundCtx x;
  x.g = gr->view();
  x.C = use_ro ? Cc : labels;
  x.pmap = use_ro ? ro->orig : nullptr;
  x.W = W;
  x.cap = cap;
  x.seed = seed;
  x.ptgt = ptgt;
  x.pgain = pgain;
  x.done = &ctl->done;
  x.gid = batch ? g->gid : nullptr;
  x.gbase = batch ? g->gbase : nullptr;
  x.gcap = gcap;
  x.gseed = gseed;
  if (hmax > 0) {
    if (wide) LP_CHECK(set_lds(k_hub_reduce<int64_t>, (size_t)hub_table(hub_part, true) * 12 + sizeof(HubReduceSmem)));
    else LP_CHECK(set_lds(k_hub_reduce<int32_t>, (size_t)hub_table(hub_part, false) * 8 + sizeof(HubReduceSmem)));
  }

  for (int32_t r = 0; r < rounds; ++r) {
    x.round = (uint32_t)r;
    const size_t round_mark = marks.size();
    LP_CHECK(begin(LP_PHASE_ROUND));
    for (int32_t sr = 0; sr < S; ++sr) {
      const Plan* plan = plans[sr];
      const int32_t* bn = plan->bn;
      auto vd_of = [&](int b) { return plan->vd(b); };
      const TilePlan& tps = plan->tps;
      const TilePlan& tpl = plan->tpl;
      const int32_t H = plan->H, npieces = plan->npieces, ntasks = plan->ntasks;
      HubMeta hm = plan->hm;
      hm.rec_c = hbuf.rec_c;
      hm.rec_r = hbuf.rec_r;
      hm.packed = hbuf.packed;
      hm.rbits = hbuf.rbits;
      hm.tmax = hub_table(hub_part, wide);
      hm.poff = hbuf.poff;
      hm.res_r = hbuf.res_r;
      hm.res_key = hbuf.res_key;
      hm.res_c = hbuf.res_c;
      hm.res_own = hbuf.res_own;
      uint32_t* hand_r = hand + 24 * ((int64_t)r * S + sr);
      // rating (all buckets) -> ptgt / pgain. The hub pieces run first, alone:
      // they are the head of the longest chain (pieces, then their reduction),
      // which then overlaps with the tiles and lanes on the side streams.
      // With a gain table the ratings are the table's affinities instead.
      if (use_gt) {
        const GtRound gr{labels, W, g->vwgt, cap, seed, (uint32_t)r, ptgt, pgain, &ctl->done};
        LP_CHECK(begin(LP_PHASE_TILE));
        LP_CHECK(gt_select(gt.t, gr, plan->order + plan->bstart[0], bn[0], plan->order + plan->bstart[1],
                           bn[1] + bn[2] + bn[3], s));
        LP_CHECK(end());
      }
      size_t hub_mark = 0;
      if (!use_gt && (H > 0 || plan->nwhole > 0)) {
        hub_mark = marks.size();
        LP_CHECK(begin(LP_PHASE_HUB));
        if (plan->nwhole > 0) {
          LP_CHECK(begin(LP_PHASE_HUB_WHOLE));
          LP_CHECK(launch_whole(g->weighted, x, plan->hw, plan->nwhole, hand_r + 20, s));
          LP_CHECK(end());
        }
        if (H > 0) {
          LP_CHECK(begin(LP_PHASE_HUB_PIECES));
          LP_CHECK(launch_piece(wide, x, hm, npieces, hand_r + 16, s));
          LP_CHECK(end());
        } else {
          LP_CHECK(end_at(hub_mark));
        }
      }
      if (!use_gt) {
        if (overlap) {
          LP_CHECK_HIP(hipEventRecord(ev.e[3], s));
          for (int i = 0; i < 3; ++i) LP_CHECK_HIP(hipStreamWaitEvent(side[i], ev.e[3], 0));
          jg.forked = true;
        }
        if (H > 0) {
          hipStream_t hs = side[0];
          LP_CHECK(begin(LP_PHASE_HUB_REDUCE, hs));
          // as many workgroups as the LDS lets every CU hold, each taking a fixed stride of tasks
          const size_t red_lds = (size_t)hm.tmax * (wide ? 12 : 8) + sizeof(HubReduceSmem);
          const unsigned red_grid = grid_for(ntasks, 1, 256u * (unsigned)std::max<size_t>(1, (160u << 10) / red_lds));
          if (wide)
            hipLaunchKernelGGL(k_hub_reduce<int64_t>, dim3(red_grid), dim3(kHubThreads), red_lds, hs, x, hm, ntasks);
          else
            hipLaunchKernelGGL(k_hub_reduce<int32_t>, dim3(red_grid), dim3(kHubThreads), red_lds, hs, x, hm, ntasks);
          LP_CHECK_LAUNCH();
          hipLaunchKernelGGL(k_hub_combine, dim3(grid_for(H, 4)), dim3(256), 0, hs, x, hm, H);
          LP_CHECK_LAUNCH();
          LP_CHECK(end(hs));
          LP_CHECK(end_at(hub_mark, hs));
        }
        if (bn[2] > 0) {
          LP_CHECK(begin(LP_PHASE_BLOCK, side[1]));
          LP_CHECK(launch_tile_any<TileLarge>(g->compressed, rate_width(g), x, vd_of(2), tpl.tiles, tpl.ntiles,
                                              hand_r + 8, tpl.grid,
                                              g->weighted, side[1]));
          LP_CHECK(end(side[1]));
        }
        if (bn[0] > 0) {
          LP_CHECK(begin(LP_PHASE_LANE, side[2]));
          LP_CHECK(launch_lane(x, vd_of(0), bn[0], side[2]));
          LP_CHECK(end(side[2]));
        }
        if (bn[1] > 0) {
          LP_CHECK(begin(LP_PHASE_TILE));
          LP_CHECK(launch_tile_any<TileSmall>(g->compressed, rate_width(g), x, vd_of(1), tps.tiles, tps.ntiles,
                                              hand_r, tps.grid,
                                              g->weighted, s));
          LP_CHECK(end());
        }
        jg.join();
      }
      // acceptance: compact in vertex order, sort by (target, gain desc)
      LP_CHECK(begin(LP_PHASE_ACCEPT));
      hipLaunchKernelGGL(k_prop_count, dim3(ncp), dim3(kCpThreads), 0, s, ptgt, n, pcnt, &ctl->done);
      LP_CHECK_LAUNCH();
      LP_CHECK(scan_exclusive_u32(pcnt, pcnt, ncp, &ctl->count, sc));
      hipLaunchKernelGGL(k_prop_write, dim3(ncp), dim3(kCpThreads), 0, s, ptgt, pgain, n, pcnt, G, ka, va, &ctl->done,
                         (S > 1 || use_ro) ? 1 : 0);
      LP_CHECK_LAUNCH();
      uint64_t* ks;
      uint32_t* vs;
      LP_CHECK(radix_sort_pairs(ka, va, kb, vb, &ctl->count, n, G + nbits, &ks, &vs, sc));
      const unsigned ga = grid_for(n, 256, 8192);
      hipLaunchKernelGGL(k_admit_prep, dim3(ga), dim3(256), 0, s, ks, vs, &ctl->count, G, g->vwgt, seg, wv);
      LP_CHECK_LAUNCH();
      LP_CHECK(seg_scan_incl_i64(seg, wv, pref, &ctl->count, n, sc));
      hipLaunchKernelGGL(k_admit, dim3(ga), dim3(256), 0, s, seg, pref, &ctl->count, W, cap, x.gid, gcap, flag);
      LP_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_apply, dim3(ga), dim3(256), 0, s, seg, vs, flag, wv, pref, &ctl->count, labels, W,
                         ctl->stats, r, mv, Cc, use_ro ? ro->pos : nullptr);
      LP_CHECK_LAUNCH();
      if (use_gt) LP_CHECK(gt_update(gt.t, mv, &ctl->count, n, labels, s));
      hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1), 0, s, &ctl->count, &ctl->done, ctl->stats, r, &ctl->rounds_run,
                         &ctl->round_props, sr == S - 1 ? 1 : 0);
      LP_CHECK_LAUNCH();
      LP_CHECK(end());
    }
    if (timing) LP_CHECK_HIP(hipEventRecord(marks[round_mark].b, s));
  }
  if (use_ro) {
    hipLaunchKernelGGL(k_ro_labels, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, ro->orig, Cc, labels);
    LP_CHECK_LAUNCH();
  }
  if (batch) LP_CHECK(batch_localize(g, labels, out_labels, labels_each, s));

  if (stats_out) {
    Ctl h;
    LP_CHECK_HIP(hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    LP_CHECK_HIP(hipStreamSynchronize(s));
    stats_out->rounds_run = h.rounds_run;
    for (const Plan* p : plans) {
      stats_out->n_lane += p->bn[0];
      stats_out->n_tile += p->bn[1];
      stats_out->n_block += p->bn[2];
      stats_out->n_hub += p->bn[3];
      for (int b = 0; b < kNumBuckets; ++b) {
        stats_out->bucket_edges[b] += p->bsums[b];
        stats_out->bucket_bytes[b] += p->bsums[kNumBuckets + b];
      }
    }
    for (int i = 0; i < 64; ++i) {
      stats_out->proposals[i] = h.stats[i];
      stats_out->moves[i] = h.stats[64 + i];
    }
    for (auto& m : marks) {
      float ms = 0;
      LP_CHECK_HIP(hipEventElapsedTime(&ms, m.a, m.b));
      if (m.phase == LP_PHASE_ROUND && stats_out->phase_launches[m.phase] < 64)
        stats_out->round_ms[stats_out->phase_launches[m.phase]] = ms;
      stats_out->phase_ms[m.phase] += ms;
      stats_out->phase_launches[m.phase] += 1;
    }
  }
  return LP_OK;
}

extern "C" lp_status lp_cluster_ex(const lp_graph* g, int64_t cap, int32_t rounds, uint64_t seed, int32_t* labels,
                                   const lp_config* cfg, lp_cluster_stats* stats, void* stream) {
  clear_error();
  if (!g || g->nbatch) return LP_EINVAL;
  return cluster_impl(g, cap, nullptr, rounds, seed, nullptr, labels, nullptr, cfg, stats, (hipStream_t)stream);
}

extern "C" lp_status lp_refine_ex(const lp_graph* g, int32_t k, int64_t max_block_weight, int32_t rounds,
                                  uint64_t seed, int32_t* labels, const lp_config* cfg, lp_cluster_stats* stats,
                                  void* stream) {
  clear_error();
  if (!g || g->nbatch || k < 1) return LP_EINVAL;
  return cluster_impl(g, max_block_weight, nullptr, rounds, seed, nullptr, labels, nullptr, cfg, stats,
                      (hipStream_t)stream, k);
}

extern "C" lp_status lp_refine(const lp_graph* g, int32_t k, int64_t max_block_weight, int32_t rounds, uint64_t seed,
                               int32_t* labels, void* stream) {
  clear_error();
  return lp_refine_ex(g, k, max_block_weight, rounds, seed, labels, nullptr, nullptr, stream);
}

extern "C" lp_status lp_batch_cluster_ex(const lp_graph* b, const int64_t* caps, int32_t rounds, const uint64_t* seeds,
                                         int32_t* labels, const lp_config* cfg, lp_cluster_stats* stats,
                                         void* stream) {
  clear_error();
  if (!b || !b->nbatch) return LP_EINVAL;
  return cluster_impl(b, 0, caps, rounds, 0, seeds, labels, nullptr, cfg, stats, (hipStream_t)stream);
}

extern "C" lp_status lp_batch_cluster(int32_t G, const lp_graph* const* gs, const int64_t* caps, int32_t rounds,
                                      const uint64_t* seeds, int32_t* const* labels_each, void* stream) {
  clear_error();
  if (G < 1 || !gs || !caps || !seeds || !labels_each) return LP_EINVAL;
  for (int32_t i = 0; i < G; ++i)
    if (!gs[i] || (gs[i]->n > 0 && !labels_each[i])) return LP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  lp_graph* b = nullptr;
  LP_CHECK(lp_batch_create(G, gs, stream, &b));
  int32_t** outs = nullptr;
  lp_status st = LP_OK;
  outs = (int32_t**)cache_alloc(G * sizeof(int32_t*), s);
  if (!outs) st = LP_ENOMEM;
  if (!st && hipMemcpyAsync(outs, labels_each, G * sizeof(int32_t*), hipMemcpyHostToDevice, s) != hipSuccess)
    st = LP_EDEVICE;
  if (!st) st = cluster_impl(b, 0, caps, rounds, 0, seeds, nullptr, outs, nullptr, nullptr, s);
  if (!st && hipStreamSynchronize(s) != hipSuccess) st = LP_EDEVICE;
  cache_free(outs, s);
  lp_graph_free(b);
  return st;
}

extern "C" lp_status lp_cluster(const lp_graph* g, int64_t cap, int32_t rounds, uint64_t seed, int32_t* labels,
                                void* stream) {
  clear_error();
  return lp_cluster_ex(g, cap, rounds, seed, labels, nullptr, nullptr, stream);
}
