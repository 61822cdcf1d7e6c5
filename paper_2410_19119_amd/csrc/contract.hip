// Cluster contraction (Section IV-B of the paper).
//
// Coarse IDs are the ranks of the nonempty labels (increasing label order);
// members are grouped per coarse vertex. Each coarse neighbourhood (summed
// weights of the fine edges leaving the cluster, keyed by the coarse ID of
// the other end) is built with the paper's two-phase aggregation
// (Section IV-B1), re-planned for gfx950:
//  - light clusters (small total member degree): one wavefront or one
//    workgroup per cluster aggregates into an LDS hash table; short members
//    are walked by one lane each, long members by a whole wavefront; the
//    table is compacted in place, bitonic-sorted in LDS and staged;
//  - heavy clusters: every member neighbourhood is cut into segments of
//    LP_CHUNK_LEN edges; a wavefront per segment writes its (coarse ID,
//    weight) records grouped by coarse-ID range partition; a workgroup per
//    (cluster, partition) aggregates that partition in LDS and emits it
//    sorted. Partitions are ranges, so their outputs concatenate in order.
// A prefix sum over the coarse degrees then places all neighbourhoods.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "decode.h"
#include "graph.h"

namespace lp {

namespace {

constexpr uint32_t kErrLabel = 1, kErrOverflow = 2, kErrFormat = 4;
constexpr uint32_t kShortMember = 32;   // members up to this degree: one lane each
constexpr uint32_t kClassWave = 256;    // total member degree per wavefront-cluster
constexpr uint32_t kClassBlockS = 1024; // ... per workgroup-cluster, small table
constexpr uint32_t kClassBlockL = 4096; // ... per workgroup-cluster, large table
constexpr uint32_t kHeavyTable = 4096;  // LDS entries of a heavy (cluster, partition) task
constexpr uint32_t kHeavyPart = 1024;   // expected distinct coarse IDs per heavy partition
constexpr int kReduceThreads = 256;
constexpr uint32_t kMaxHeavyParts = 1024;
constexpr int kLightThreads = 256;

// ------------------------------------------------------------- setup -----
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

// Class 0: no edges; 1: wavefront; 2, 3: workgroup (small / large table);
// 4: heavy. Light classes get a staging capacity of min(dsum, nc - 1).
__global__ void k_cclass(const unsigned long long* dsum, const unsigned long long* vw, int32_t nc, uint64_t* tcap,
                         uint8_t* cls, int32_t* vwgt_out, uint32_t* err) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nc; a += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t d = dsum[a];
    const uint8_t c = d == 0 ? 0 : d <= kClassWave ? 1 : d <= kClassBlockS ? 2 : d <= kClassBlockL ? 3 : 4;
    cls[a] = c;
    tcap[a] = (c >= 1 && c <= 3) ? std::min<uint64_t>(d, (uint64_t)nc - 1) : 0;
    const unsigned long long w = vw[a];
    if (w > 0x7FFFFFFFull) atomicOr(err, kErrOverflow);
    vwgt_out[a] = (int32_t)w;
  }
}

// Appends every coarse vertex of class 1..4 to its class list; one atomic
// per wavefront and class.
__global__ void k_class_list(const uint8_t* cls, int32_t nc, uint32_t* counters, int32_t* lists, int64_t stride) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += step) {
    const int64_t a = base + threadIdx.x;
    const int c = a < nc ? cls[a] : 0;
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
      const uint64_t m = __ballot(c == k);
      if (!m) continue;
      const int leader = __ffsll((long long)m) - 1;
      uint32_t b = 0;
      if (lane_id() == leader) b = atomicAdd(&counters[k], (uint32_t)__popcll(m));
      b = __shfl(b, leader, kWave);
      if (c == k) lists[(int64_t)(k - 1) * stride + b + __popcll(m & lanemask_lt())] = (int32_t)a;
    }
  }
}

__device__ __forceinline__ uint32_t ceil_log2(uint32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

// ------------------------------------------------------- LDS helpers -----
__device__ __forceinline__ void tbl_add(int32_t* keys, int64_t* vals, uint32_t mask, uint32_t shift, int32_t b,
                                        int64_t w) {
  uint32_t h = slot_hash((uint32_t)b) >> shift;
  while (true) {
    const int32_t k = keys[h];
    if (k == b) {
      atomicAdd((unsigned long long*)&vals[h], (unsigned long long)w);
      return;
    }
    if (k == kEmpty) {
      const int32_t old = atomicCAS(&keys[h], kEmpty, b);
      if (old == kEmpty || old == b) {
        atomicAdd((unsigned long long*)&vals[h], (unsigned long long)w);
        return;
      }
    }
    h = (h + 1) & mask;
  }
}

// Insert with a reservation guard: at most `limit` distinct keys enter the
// table; a further new key sets *overflow instead.
__device__ __forceinline__ void tbl_add_guarded(int32_t* keys, int64_t* vals, uint32_t mask, uint32_t shift,
                                                int32_t b, int64_t w, uint32_t limit, uint32_t* distinct,
                                                uint32_t* overflow) {
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
        if (atomicAdd(distinct, 1u) >= limit) {
          *overflow = 1;
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

// Bitonic sort of (keys, vals)[0..cnt) by key in LDS; cnt is a power of two.
template <int NT>
__device__ __forceinline__ void lds_bitonic(int32_t* keys, int64_t* vals, uint32_t cnt) {
  const int tid = group_tid<NT>();
  for (uint32_t k = 2; k <= cnt; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < cnt; i += NT) {
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

// Compacts the table's entries to its front (in place, NT slots per step:
// every write position is at or before a slot already read in that step),
// sorts them by key and writes them to (ob, ow). Returns the entry count.
template <int NT>
__device__ uint32_t compact_sort_write(int32_t* keys, int64_t* vals, uint32_t cap, int32_t* ob, int64_t* ow,
                                       uint32_t* err, int32_t* scan_sm) {
  const int tid = group_tid<NT>();
  uint32_t cnt = 0;
  for (uint32_t r = 0; r < cap; r += NT) {
    const uint32_t s = r + tid;
    const int32_t k = s < cap ? keys[s] : kEmpty;
    const int64_t v = s < cap ? vals[s] : 0;
    const int32_t f = k != kEmpty;
    int32_t tot;
    const int32_t incl = block_incl_scan_add<NT, int32_t>(f, scan_sm, &tot);
    group_sync<NT>();
    if (f) {
      keys[cnt + incl - 1] = k;
      vals[cnt + incl - 1] = v;
    }
    cnt += (uint32_t)tot;
    group_sync<NT>();
  }
  uint32_t p2 = 1;
  while (p2 < cnt) p2 <<= 1;
  for (uint32_t s = cnt + tid; s < p2; s += NT) keys[s] = 0x7FFFFFFF;
  group_sync<NT>();
  lds_bitonic<NT>(keys, vals, p2);
  for (uint32_t i = tid; i < cnt; i += NT) {
    ob[i] = keys[i];
    ow[i] = vals[i];
    if (vals[i] > 0x7FFFFFFFll) atomicOr(err, kErrOverflow);
  }
  group_sync<NT>();
  return cnt;
}

struct CArgs {
  GraphView g;
  const int32_t* map;
  const int32_t* deg;
  const int32_t* members;
  const uint32_t* mstart;
  const uint64_t* tbase;
  const uint64_t* tcap;
  int32_t* tb;     // light staging: coarse neighbour
  int64_t* tw;     // light staging: weight
  uint64_t* cdeg;  // coarse degree per coarse vertex
  uint32_t* err;
  int32_t nc;
};

// Walks one short neighbourhood with one lane.
template <bool COMP, typename F>
__device__ __forceinline__ void lane_walk(const GraphView& g, int32_t u, uint32_t d, F&& f) {
  if constexpr (COMP) {
    lane_decode(g, u, d, f);
  } else {
    const uint64_t b = g.xadj[u];
    for (uint32_t k = 0; k < d; ++k) f(k, g.adjncy[b + k], g.adjwgt ? g.adjwgt[b + k] : 1);
  }
}

// Walks one neighbourhood with one wavefront.
template <bool COMP, typename F>
__device__ __forceinline__ bool wave_walk(const GraphView& g, int32_t u, uint32_t d, DecodeSmem<kWave>& dsm, F&& f) {
  if constexpr (COMP) {
    const Nbh h = nbh_locate(g, u, d);
    bool ok = true;
    for (uint32_t ch = 0; ch < h.nchunks; ++ch) {
      uint64_t pos = nbh_chunk_pos(g, h, ch);
      const uint32_t first = ch * LP_CHUNK_LEN;
      const uint32_t cnt = (h.nchunks > 1) ? min((uint32_t)LP_CHUNK_LEN, d - first) : d;
      int32_t pv, pw;
      ok &= group_decode<kWave>(g.bytes, pos, u, cnt, g.weighted, true, pv, pw, dsm, f);
    }
    return ok;
  } else {
    const uint64_t b = g.xadj[u];
    for (uint32_t k = lane_id(); k < d; k += kWave) f(k, g.adjncy[b + k], g.adjwgt ? g.adjwgt[b + k] : 1);
    return true;
  }
}

template <int NT>
struct LightSmem {
  DecodeSmem<kWave> dec[NT / kWave];
  int32_t scan[NT / kWave];
  uint32_t distinct;
  uint32_t overflow;
};

// Light clusters. NT = 64: one cluster per wavefront (4 per workgroup);
// NT = 256: one cluster per workgroup. Table capacity = next power of two
// >= 2 * min(dsum, nc - 1), at most tmax. A cluster whose distinct count
// would exceed half the capacity (possible only when the capacity is
// clipped to tmax) is appended to the heavy list (*nheavy entries at
// heavy_list) instead, with its staging capacity cleared.
template <int NT, bool COMP>
__global__ __launch_bounds__(kLightThreads) void k_contract_light(CArgs A, const int32_t* list, int32_t cnt,
                                                                  uint32_t tmax, int32_t* heavy_list,
                                                                  uint32_t* nheavy, uint64_t* tcap_rw) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  constexpr int G = kLightThreads / NT;
  constexpr int NW = NT / kWave;
  const int gi = (int)(threadIdx.x / NT);
  const int tid = group_tid<NT>();
  const int wig = (int)((threadIdx.x % NT) / kWave);  // wave index inside the group
  const size_t per = ((size_t)tmax * 12 + sizeof(LightSmem<NT>) + 15) & ~size_t(15);
  uint8_t* base = smem_raw + gi * per;
  int64_t* vals = (int64_t*)base;
  int32_t* keys = (int32_t*)(base + (size_t)tmax * 8);
  LightSmem<NT>& sm = *(LightSmem<NT>*)(base + (size_t)tmax * 12);
  for (int64_t it = (int64_t)blockIdx.x * G + gi; it < cnt; it += (int64_t)gridDim.x * G) {
    const int32_t a = list[it];
    const uint32_t want = (uint32_t)A.tcap[a];
    const uint32_t logc = min(ceil_log2(tmax), max(6u, ceil_log2(2 * max(want, 1u))));
    const uint32_t cap = 1u << logc, mask = cap - 1, shift = 32 - logc;
    const uint32_t limit = (2 * want > cap) ? cap / 2 : cap;
    for (uint32_t s = tid; s < cap; s += NT) {
      keys[s] = kEmpty;
      vals[s] = 0;
    }
    if (tid == 0) {
      sm.distinct = 0;
      sm.overflow = 0;
    }
    group_sync<NT>();
    const uint32_t m0 = A.mstart[a], m1 = A.mstart[a + 1];
    auto ins = [&](uint32_t, int32_t v, int32_t w) {
      const int32_t b = A.map[v];
      if (b != a) tbl_add_guarded(keys, vals, mask, shift, b, (int64_t)w, limit, &sm.distinct, &sm.overflow);
    };
    // short members: one thread each
    for (uint32_t m = m0 + tid; m < m1; m += NT) {
      const int32_t u = A.members[m];
      const uint32_t d = (uint32_t)A.deg[u];
      if (d > 0 && d <= kShortMember) lane_walk<COMP>(A.g, u, d, ins);
    }
    // long members: one wavefront each
    bool ok = true;
    for (uint32_t mb = m0 + wig * kWave; mb < m1; mb += NW * kWave) {
      const uint32_t m = mb + lane_id();
      const int32_t um = m < m1 ? A.members[m] : 0;
      uint64_t big = __ballot(m < m1 && (uint32_t)A.deg[um] > kShortMember);
      while (big) {
        const int l = __ffsll((long long)big) - 1;
        big &= big - 1;
        const int32_t u = __shfl(um, l, kWave);
        ok &= wave_walk<COMP>(A.g, u, (uint32_t)A.deg[u], sm.dec[wig], ins);
      }
    }
    if (!ok && lane_id() == 0) atomicOr(A.err, kErrFormat);
    group_sync<NT>();
    if (sm.overflow) {
      if (tid == 0) {
        heavy_list[atomicAdd(nheavy, 1u)] = a;
        tcap_rw[a] = 0;
      }
      group_sync<NT>();
      continue;
    }
    const uint32_t k = compact_sort_write<NT>(keys, vals, cap, A.tb + A.tbase[a], A.tw + A.tbase[a], A.err, sm.scan);
    if (tid == 0) A.cdeg[a] = k;
    group_sync<NT>();
  }
}

// Final placement of the light staging (wave per light coarse vertex).
__global__ __launch_bounds__(256) void k_place_light(const uint64_t* cx, const uint64_t* tbase, const uint64_t* tcap,
                                                     const int32_t* tb, const int64_t* tw, int32_t nc,
                                                     int32_t* adjncy, int32_t* adjwgt) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t a = wid; a < nc; a += nw) {
    if (tcap[a] == 0) continue;
    const uint64_t o = cx[a], d = cx[a + 1] - o, t = tbase[a];
    for (uint64_t i = lane; i < d; i += kWave) {
      adjncy[o + i] = tb[t + i];
      adjwgt[o + i] = (int32_t)tw[t + i];
    }
  }
}

// ------------------------------------------------------------ heavy -----
struct Heavy {
  const int32_t* clusters;  // heavy cluster -> coarse vertex
  const int32_t* parts;     // P per heavy cluster
  const uint32_t* mbase;    // first heavy member of each heavy cluster (H + 1)
  const uint32_t* tbase;    // first task of each heavy cluster (H + 1)
  const int32_t* mu;        // heavy member -> fine vertex
  const int32_t* mh;        // heavy member -> heavy cluster
  const uint32_t* sbase;    // first segment of each heavy member (M + 1)
  const uint64_t* rbase;    // first record of each heavy member
  const uint64_t* pbase;    // first partition-table entry of each heavy member
  const int2* pieces;       // (heavy member, first segment of that member)
  uint64_t* seg_rb;         // first record of each segment
  uint64_t* seg_pt;         // partition table of each segment
  int32_t* rec_b;           // records: coarse ID
  int32_t* rec_w;           // records: weight
  uint32_t* ptab;           // per segment: P + 1 partition offsets
  const int2* tasks;        // (heavy cluster, partition)
  uint64_t* tcnt;           // records per task, then (scanned) staging base
  int32_t* ob;              // heavy staging
  int64_t* ow;
  uint64_t* tdeg;           // distinct coarse neighbours per task
};

__global__ void k_heavy_meta(const int32_t* hl, int32_t H, const uint32_t* mstart, const unsigned long long* dsum,
                             int32_t nc, int32_t* parts, uint32_t* mcount, uint32_t* pcount) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = hl[h];
    const uint64_t distinct = std::min<uint64_t>(dsum[a], (uint64_t)nc - 1);
    const uint64_t part = std::max<uint64_t>(kHeavyPart, (distinct + kMaxHeavyParts - 1) / kMaxHeavyParts);
    const int32_t P = (int32_t)std::max<uint64_t>(1, (distinct + part - 1) / part);
    parts[h] = P;
    pcount[h] = (uint32_t)P;
    mcount[h] = mstart[a + 1] - mstart[a];
  }
}

// Heavy members (wave per heavy cluster): vertex, cluster, segments,
// records, partition-table entries and pieces of each member.
__global__ __launch_bounds__(256) void k_heavy_members(const int32_t* hl, int32_t H, const uint32_t* mstart,
                                                       const int32_t* members, const int32_t* deg,
                                                       const int32_t* parts, const uint32_t* mbase, int32_t* mu,
                                                       int32_t* mh, uint32_t* nseg, uint64_t* nrec, uint64_t* npt,
                                                       uint32_t* npiece, int compressed) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t h = wid; h < H; h += nw) {
    const int32_t a = hl[h];
    const uint32_t m0 = mstart[a], cnt = mstart[a + 1] - m0;
    const uint32_t P = (uint32_t)parts[h];
    for (uint32_t i = lane; i < cnt; i += kWave) {
      const int32_t u = members[m0 + i];
      const uint32_t d = (uint32_t)deg[u];
      const uint32_t s = (d + LP_CHUNK_LEN - 1) / LP_CHUNK_LEN;
      const uint32_t o = mbase[h] + i;
      mu[o] = u;
      mh[o] = (int32_t)h;
      nseg[o] = s;
      nrec[o] = d;
      npt[o] = (uint64_t)s * (P + 1);
      npiece[o] = (compressed && d <= LP_CHUNK_THRESHOLD) ? (s ? 1u : 0u) : s;
    }
  }
}

__global__ void k_heavy_pieces(int32_t M, const uint32_t* npiece_scan, const uint32_t* sbase, const uint64_t* rbase,
                               const uint64_t* pbase, const int32_t* mh, const int32_t* parts, const int32_t* mu,
                               const int32_t* deg, int compressed, int2* pieces, uint64_t* seg_rb, uint64_t* seg_pt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t d = (uint32_t)deg[mu[i]];
    const uint32_t b = npiece_scan[i];
    const uint32_t ns = sbase[i + 1] - sbase[i];
    const uint32_t P = (uint32_t)parts[mh[i]];
    for (uint32_t k = 0; k < ns; ++k) {
      seg_rb[sbase[i] + k] = rbase[i] + (uint64_t)k * LP_CHUNK_LEN;
      seg_pt[sbase[i] + k] = pbase[i] + (uint64_t)k * (P + 1);
    }
    if (compressed && d <= LP_CHUNK_THRESHOLD) {
      if (ns) pieces[b] = make_int2((int)i, 0);
    } else {
      for (uint32_t k = 0; k < ns; ++k) pieces[b + k] = make_int2((int)i, (int)k);
    }
  }
}

__global__ void k_heavy_tasks(int32_t H, const int32_t* parts, const uint32_t* tbase, int2* tasks) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x)
    for (int32_t p = 0; p < parts[h]; ++p) tasks[tbase[h] + p] = make_int2((int)h, p);
}

struct ScatterSmem {
  DecodeSmem<kWave> dec;
  int32_t b[LP_CHUNK_LEN];
  int32_t w[LP_CHUNK_LEN];
  uint16_t p[LP_CHUNK_LEN];
  uint32_t hist[kMaxHeavyParts];
  uint32_t cnt;
};

// Range partition of coarse ID b among P parts of [0, nc).
__device__ __forceinline__ uint32_t range_part(int32_t b, uint32_t P, int32_t nc) {
  return (uint32_t)(((uint64_t)(uint32_t)b * P) / (uint64_t)nc);
}

// One wavefront per piece: decode the piece's segment(s), keep edges that
// leave the cluster, group the records of each segment by partition.
template <bool COMP>
__global__ __launch_bounds__(256) void k_heavy_scatter(CArgs A, Heavy hv, int32_t npieces) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  ScatterSmem& sm = ((ScatterSmem*)smem_raw)[threadIdx.x / kWave];
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t pc = wid; pc < npieces; pc += nw) {
    const int2 piece = hv.pieces[pc];
    const int32_t i = piece.x;
    const int32_t u = hv.mu[i];
    const int32_t h = hv.mh[i];
    const int32_t a = hv.clusters[h];
    const uint32_t P = (uint32_t)hv.parts[h];
    const uint32_t d = (uint32_t)A.deg[u];
    const uint32_t nseg_m = hv.sbase[i + 1] - hv.sbase[i];
    bool chunked = true;
    uint32_t nseg_here = 1;
    uint64_t pos = 0;
    if constexpr (COMP) {
      const Nbh hb = nbh_locate(A.g, u, d);
      chunked = hb.nchunks > 1;
      nseg_here = chunked ? 1u : nseg_m;
      pos = chunked ? nbh_chunk_pos(A.g, hb, (uint32_t)piece.y) : hb.codes;
    }
    int32_t pv = 0, pw = 0;
    for (uint32_t s = 0; s < nseg_here; ++s) {
      const uint32_t k = (uint32_t)piece.y + s;
      const uint32_t first = k * LP_CHUNK_LEN;
      const uint32_t cnt = min((uint32_t)LP_CHUNK_LEN, d - first);
      if (lane == 0) sm.cnt = 0;
      wave_sync_lds();
      auto keep = [&](uint32_t, int32_t v, int32_t w) {
        const int32_t b = A.map[v];
        if (b != a) {
          const uint32_t slot = atomicAdd(&sm.cnt, 1u);
          sm.b[slot] = b;
          sm.w[slot] = w;
        }
      };
      if constexpr (COMP) {
        if (!group_decode<kWave>(A.g.bytes, pos, u, cnt, A.g.weighted, chunked || s == 0, pv, pw, sm.dec, keep) &&
            lane == 0)
          atomicOr(A.err, kErrFormat);
      } else {
        const uint64_t e0 = A.g.xadj[u] + first;
        for (uint32_t j = lane; j < cnt; j += kWave) keep(j, A.g.adjncy[e0 + j], A.g.adjwgt ? A.g.adjwgt[e0 + j] : 1);
      }
      for (uint32_t j = lane; j < P; j += kWave) sm.hist[j] = 0;
      wave_sync_lds();
      const uint32_t kept = sm.cnt;
      for (uint32_t j = lane; j < kept; j += kWave) {
        const uint32_t p = range_part(sm.b[j], P, A.nc);
        sm.p[j] = (uint16_t)p;
        atomicAdd(&sm.hist[p], 1u);
      }
      wave_sync_lds();
      uint32_t* pt = hv.ptab + hv.pbase[i] + (uint64_t)k * (P + 1);
      uint32_t carry = 0;
      for (uint32_t b0 = 0; b0 < P; b0 += kWave) {
        const uint32_t j = b0 + lane;
        const uint32_t v = j < P ? sm.hist[j] : 0;
        const uint32_t inc = wave_incl_scan_add(v);
        if (j < P) {
          sm.hist[j] = carry + inc - v;
          pt[j] = carry + inc - v;
        }
        carry += __shfl(inc, kWave - 1, kWave);
      }
      if (lane == 0) pt[P] = kept;
      wave_sync_lds();
      const uint64_t out = hv.rbase[i] + first;
      for (uint32_t j = lane; j < kept; j += kWave) {
        const uint32_t slot = atomicAdd(&sm.hist[sm.p[j]], 1u);
        hv.rec_b[out + slot] = sm.b[j];
        hv.rec_w[out + slot] = sm.w[j];
      }
      wave_sync_lds();
    }
  }
}

// Records per (cluster, partition) task (wave per task).
__global__ __launch_bounds__(256) void k_heavy_count(Heavy hv, int32_t ntasks) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t t = wid; t < ntasks; t += nw) {
    const int2 task = hv.tasks[t];
    const int32_t h = task.x;
    const uint32_t p = (uint32_t)task.y;
    const uint32_t P = (uint32_t)hv.parts[h];
    uint64_t c = 0;
    const uint32_t s0 = hv.sbase[hv.mbase[h]], s1 = hv.sbase[hv.mbase[h + 1]];
    for (uint32_t sg = s0 + lane; sg < s1; sg += kWave) {
      const uint32_t* pt = hv.ptab + hv.seg_pt[sg];
      c += pt[p + 1] - pt[p];
    }
    c = wave_reduce_add(c);
    if (lane == 0) hv.tcnt[t] = c;
  }
}

struct ReduceSmem {
  int32_t scan[kReduceThreads / kWave];
  uint32_t distinct;
  uint32_t overflow;
};

// One workgroup per (cluster, partition): aggregate the partition's records
// in LDS over coarse-ID windows (a window whose distinct count exceeds half
// the table is halved and retried), emitting each window sorted. The table
// is sized by the task's record count.
__global__ __launch_bounds__(kReduceThreads) void k_heavy_reduce(CArgs A, Heavy hv, int32_t ntasks) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  constexpr int NT = kReduceThreads;
  int64_t* vals = (int64_t*)smem_raw;
  int32_t* keys = (int32_t*)(smem_raw + (size_t)kHeavyTable * 8);
  ReduceSmem& sm = *(ReduceSmem*)(smem_raw + (size_t)kHeavyTable * 12);
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  const uint64_t nc = (uint64_t)A.nc;
  for (int64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const int2 task = hv.tasks[t];
    const int32_t h = task.x;
    const uint32_t p = (uint32_t)task.y;
    const uint32_t P = (uint32_t)hv.parts[h];
    const uint64_t lo_p = ((uint64_t)p * nc + P - 1) / P, hi_p = ((uint64_t)(p + 1) * nc + P - 1) / P;
    const uint64_t obase = hv.tcnt[t];
    const uint64_t nrec = hv.tcnt[t + 1] - obase;
    const uint32_t logc =
        min(ceil_log2(kHeavyTable), max(6u, ceil_log2((uint32_t)std::min<uint64_t>(2 * nrec + 2, kHeavyTable))));
    const uint32_t tcap = 1u << logc, mask = tcap - 1, shift = 32 - logc;
    const uint32_t limit = tcap / 2;
    const uint32_t s0 = hv.sbase[hv.mbase[h]], s1 = hv.sbase[hv.mbase[h + 1]];
    uint64_t written = 0;
    uint64_t lo = lo_p, width = hi_p - lo_p;
    while (lo < hi_p) {
      const uint64_t hi = std::min<uint64_t>(hi_p, lo + width);
      for (uint32_t q = tid; q < tcap; q += NT) {
        keys[q] = kEmpty;
        vals[q] = 0;
      }
      if (tid == 0) {
        sm.distinct = 0;
        sm.overflow = 0;
      }
      __syncthreads();
      // one wavefront per segment, lanes over its records of partition p
      for (uint32_t sg = s0 + wv; sg < s1; sg += NT / kWave) {
        const uint32_t* pt = hv.ptab + hv.seg_pt[sg];
        const uint32_t ra = pt[p], rb = pt[p + 1];
        const uint64_t rbase = hv.seg_rb[sg];
        for (uint32_t j = ra + lane; j < rb; j += kWave) {
          const int32_t b = hv.rec_b[rbase + j];
          if ((uint64_t)b >= lo && (uint64_t)b < hi)
            tbl_add_guarded(keys, vals, mask, shift, b, (int64_t)hv.rec_w[rbase + j], limit, &sm.distinct,
                            &sm.overflow);
        }
      }
      __syncthreads();
      if (sm.overflow && hi - lo > 1) {
        width = std::max<uint64_t>(1, (hi - lo) / 2);
        __syncthreads();
        continue;
      }
      const uint32_t k = compact_sort_write<NT>(keys, vals, tcap, hv.ob + obase + written, hv.ow + obase + written,
                                                A.err, sm.scan);
      written += k;
      lo = hi;
      width = hi_p - lo;  // try the rest of the partition in one window again
      __syncthreads();
    }
    if (tid == 0) hv.tdeg[t] = written;
    __syncthreads();
  }
}

__global__ void k_heavy_cdeg(Heavy hv, int32_t H, uint64_t* cdeg) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    uint64_t s = 0;
    for (uint32_t t = hv.tbase[h]; t < hv.tbase[h + 1]; ++t) s += hv.tdeg[t];
    cdeg[hv.clusters[h]] = s;
  }
}

// Places heavy neighbourhoods: task t of cluster h goes after the outputs
// of the cluster's earlier partitions (wave per task).
__global__ __launch_bounds__(256) void k_place_heavy(Heavy hv, int32_t ntasks, const uint64_t* tdeg_scan,
                                                     const uint64_t* cx, int32_t* adjncy, int32_t* adjwgt) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t t = wid; t < ntasks; t += nw) {
    const int32_t h = hv.tasks[t].x;
    const int32_t a = hv.clusters[h];
    const uint64_t dst = cx[a] + (tdeg_scan[t] - tdeg_scan[hv.tbase[h]]);
    const uint64_t src = hv.tcnt[t], d = hv.tdeg[t];
    for (uint64_t j = lane; j < d; j += kWave) {
      adjncy[dst + j] = hv.ob[src + j];
      adjwgt[dst + j] = (int32_t)hv.ow[src + j];
    }
  }
}

__global__ __launch_bounds__(256) void k_wdeg(const uint64_t* xadj, const int32_t* adjwgt, int32_t n,
                                              unsigned long long* max_wdeg, unsigned long long* max_deg) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  unsigned long long mw = 0, md = 0;
  for (int64_t u = wid; u < n; u += nw) {
    const uint64_t b = xadj[u], e = xadj[u + 1];
    int64_t s = 0;
    for (uint64_t k = b + lane; k < e; k += kWave) s += adjwgt[k];
    s = wave_reduce_add(s);
    mw = max(mw, (unsigned long long)s);
    md = max(md, (unsigned long long)(e - b));
  }
  __shared__ unsigned long long sa[4], sb[4];
  mw = wave_reduce_max(mw);
  md = wave_reduce_max(md);
  if (lane == 0) {
    sa[threadIdx.x / kWave] = mw;
    sb[threadIdx.x / kWave] = md;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      mw = max(mw, sa[i]);
      md = max(md, sb[i]);
    }
    atomicMax(max_wdeg, mw);
    atomicMax(max_deg, md);
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

template <int NT, bool COMP>
lp_status launch_light(const CArgs& A, const int32_t* list, uint32_t cnt, uint32_t tmax, int32_t* heavy_list,
                       uint32_t* nheavy, uint64_t* tcap_rw, hipStream_t s) {
  if (cnt == 0) return LP_OK;
  const size_t per = ((size_t)tmax * 12 + sizeof(LightSmem<NT>) + 15) & ~size_t(15);
  const size_t bytes = per * (kLightThreads / NT);
  auto k = k_contract_light<NT, COMP>;
  LP_CHECK(set_lds(k, bytes));
  hipLaunchKernelGGL(k, dim3(grid_for(cnt, kLightThreads / NT, 1u << 20)), dim3(kLightThreads), bytes, s, A, list,
                     (int32_t)cnt, tmax, heavy_list, nheavy, tcap_rw);
  return last_error();
}

// Heavy clusters: metadata, scatter, count, reduce. Fills cdeg of heavy
// clusters and leaves what placement needs in *hv_out.
template <bool COMP>
lp_status contract_heavy(const CArgs& A, const int32_t* hl, int32_t H, const unsigned long long* dsum,
                         Heavy* hv_out, int32_t* ntasks_out, uint64_t** tdeg_scan_out, Scratch& sc) {
  hipStream_t s = sc.stream();
  Heavy hv{};
  int32_t* parts = sc.alloc<int32_t>(H);
  uint32_t* mbase = sc.alloc<uint32_t>((size_t)H + 1);
  uint32_t* tbase = sc.alloc<uint32_t>((size_t)H + 1);
  uint64_t* tot = sc.alloc<uint64_t>(4);
  uint32_t* tot32 = sc.alloc<uint32_t>(4);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(mbase + H, 0, 4, s));
  LP_CHECK_HIP(hipMemsetAsync(tbase + H, 0, 4, s));
  hipLaunchKernelGGL(k_heavy_meta, dim3(grid_for(H, 256, 4096)), dim3(256), 0, s, hl, H, A.mstart, dsum, A.nc, parts,
                     mbase, tbase);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u32(mbase, mbase, (int64_t)H + 1, &tot32[0], sc));
  LP_CHECK(scan_exclusive_u32(tbase, tbase, (int64_t)H + 1, &tot32[1], sc));
  uint32_t ht[2];
  LP_CHECK_HIP(hipMemcpyAsync(ht, tot32, 8, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  const int32_t M = (int32_t)ht[0], T = (int32_t)ht[1];
  int32_t* mu = sc.alloc<int32_t>(M);
  int32_t* mh = sc.alloc<int32_t>(M);
  uint32_t* sbase = sc.alloc<uint32_t>((size_t)M + 1);
  uint64_t* rbase = sc.alloc<uint64_t>((size_t)M + 1);
  uint64_t* pbase = sc.alloc<uint64_t>((size_t)M + 1);
  uint32_t* npiece = sc.alloc<uint32_t>((size_t)M + 1);
  int2* tasks = sc.alloc<int2>(T);
  uint64_t* tcnt = sc.alloc<uint64_t>((size_t)T + 1);
  uint64_t* tdeg = sc.alloc<uint64_t>((size_t)T + 1);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(sbase + M, 0, 4, s));
  LP_CHECK_HIP(hipMemsetAsync(rbase + M, 0, 8, s));
  LP_CHECK_HIP(hipMemsetAsync(pbase + M, 0, 8, s));
  LP_CHECK_HIP(hipMemsetAsync(npiece + M, 0, 4, s));
  LP_CHECK_HIP(hipMemsetAsync(tcnt + T, 0, 8, s));
  hipLaunchKernelGGL(k_heavy_members, dim3(grid_for((int64_t)H * kWave, 256, 16384)), dim3(256), 0, s, hl, H,
                     A.mstart, A.members, A.deg, parts, mbase, mu, mh, sbase, rbase, pbase, npiece, COMP ? 1 : 0);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_heavy_tasks, dim3(grid_for(H, 256, 4096)), dim3(256), 0, s, H, parts, tbase, tasks);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u32(sbase, sbase, (int64_t)M + 1, &tot32[2], sc));
  LP_CHECK(scan_exclusive_u64(rbase, rbase, (int64_t)M + 1, &tot[0], sc));
  LP_CHECK(scan_exclusive_u64(pbase, pbase, (int64_t)M + 1, &tot[1], sc));
  LP_CHECK(scan_exclusive_u32(npiece, npiece, (int64_t)M + 1, &tot32[3], sc));
  uint64_t h64[2];
  uint32_t h32[4];
  LP_CHECK_HIP(hipMemcpyAsync(h64, tot, 16, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipMemcpyAsync(h32, tot32, 16, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  const uint64_t R = h64[0], PT = h64[1];
  const int32_t NP = (int32_t)h32[3];
  if (getenv("LPGPU_DEBUG"))
    fprintf(stderr, "[lpgpu] contract heavy: clusters %d members %d tasks %d segments %u pieces %d records %llu\n", H,
            M, T, h32[2], NP, (unsigned long long)R);
  const uint32_t S = h32[2];
  int2* pieces = sc.alloc<int2>(NP);
  hv.seg_rb = sc.alloc<uint64_t>(S);
  hv.seg_pt = sc.alloc<uint64_t>(S);
  hv.rec_b = sc.alloc<int32_t>(R);
  hv.rec_w = sc.alloc<int32_t>(R);
  hv.ptab = sc.alloc<uint32_t>(PT);
  if (sc.failed) return LP_ENOMEM;
  hipLaunchKernelGGL(k_heavy_pieces, dim3(grid_for(M, 256, 65536)), dim3(256), 0, s, M, npiece, sbase, rbase, pbase,
                     mh, parts, mu, A.deg, COMP ? 1 : 0, pieces, hv.seg_rb, hv.seg_pt);
  LP_CHECK_LAUNCH();
  hv.clusters = hl;
  hv.parts = parts;
  hv.mbase = mbase;
  hv.tbase = tbase;
  hv.mu = mu;
  hv.mh = mh;
  hv.sbase = sbase;
  hv.rbase = rbase;
  hv.pbase = pbase;
  hv.pieces = pieces;
  hv.tasks = tasks;
  hv.tcnt = tcnt;
  hv.tdeg = tdeg;
  if (NP > 0) {
    const size_t sbytes = sizeof(ScatterSmem) * 4;
    LP_CHECK(set_lds(k_heavy_scatter<COMP>, sbytes));
    hipLaunchKernelGGL(k_heavy_scatter<COMP>, dim3(grid_for(NP, 4, 1u << 20)), dim3(256), sbytes, s, A, hv, NP);
    LP_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_heavy_count, dim3(grid_for((int64_t)T, 4, 65536)), dim3(256), 0, s, hv, T);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u64(tcnt, tcnt, (int64_t)T + 1, &tot[2], sc));
  LP_CHECK_HIP(hipMemcpyAsync(h64, tot + 2, 8, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  hv.ob = sc.alloc<int32_t>(h64[0]);
  hv.ow = sc.alloc<int64_t>(h64[0]);
  if (sc.failed) return LP_ENOMEM;
  const size_t rbytes = (size_t)kHeavyTable * 12 + sizeof(ReduceSmem);
  LP_CHECK(set_lds(k_heavy_reduce, rbytes));
  hipLaunchKernelGGL(k_heavy_reduce, dim3(grid_for(T, 1, 1u << 20)), dim3(kReduceThreads), rbytes, s, A, hv, T);
  LP_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_heavy_cdeg, dim3(grid_for(H, 256, 4096)), dim3(256), 0, s, hv, H, A.cdeg);
  LP_CHECK_LAUNCH();
  uint64_t* tscan = sc.alloc<uint64_t>((size_t)T + 1);
  if (!tscan) return LP_ENOMEM;
  LP_CHECK(scan_exclusive_u64(tdeg, tscan, (int64_t)T, nullptr, sc));
  *hv_out = hv;
  *ntasks_out = T;
  *tdeg_scan_out = tscan;
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
    uint32_t ccount[8];
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
    int32_t* lists = sc.alloc<int32_t>((size_t)4 * nc);
    if (sc.failed) { st = LP_ENOMEM; break; }
    if (hipMalloc((void**)&cg->vwgt, (size_t)nc * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&cg->xadj, ((size_t)nc + 1) * sizeof(uint64_t)) != hipSuccess) { st = LP_ENOMEM; break; }
    (void)hipMemsetAsync(cnt, 0, ((size_t)nc + 1) * sizeof(uint32_t), s);
    (void)hipMemsetAsync(cursor, 0, (size_t)nc * sizeof(uint32_t), s);
    (void)hipMemsetAsync(vw, 0, (size_t)nc * 8, s);
    (void)hipMemsetAsync(dsum, 0, (size_t)nc * 8, s);
    (void)hipMemsetAsync(cdeg, 0, ((size_t)nc + 1) * sizeof(uint64_t), s);
    hipLaunchKernelGGL(k_map, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, labels, n, flags, deg, g->vwgt, map, cnt,
                       vw, dsum);
    st = last_error();
    if (st) break;
    st = scan_exclusive_u32(cnt, cnt, (int64_t)nc + 1, nullptr, sc);
    if (st) break;
    hipLaunchKernelGGL(k_members, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, map, n, cnt, cursor, members);
    hipLaunchKernelGGL(k_cclass, dim3(grid_for(nc, 256, 65536)), dim3(256), 0, s, dsum, vw, nc, tcap, cls, cg->vwgt,
                       &ctl->err);
    hipLaunchKernelGGL(k_class_list, dim3(grid_for(nc, 256, 65536)), dim3(256), 0, s, cls, nc, ctl->ccount, lists,
                       (int64_t)nc);
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
    const int64_t stride = nc;
    int32_t* hlist = lists + 3 * stride;
    uint32_t* nheavy = &ctl->ccount[4];
    if (g->compressed) {
      st = launch_light<kWave, true>(A, lists, h.ccount[1], 2 * kClassWave, hlist, nheavy, tcap, s);
      if (!st) st = launch_light<kLightThreads, true>(A, lists + stride, h.ccount[2], 2 * kClassBlockS, hlist, nheavy, tcap, s);
      if (!st) st = launch_light<kLightThreads, true>(A, lists + 2 * stride, h.ccount[3], kClassBlockL, hlist, nheavy, tcap, s);
    } else {
      st = launch_light<kWave, false>(A, lists, h.ccount[1], 2 * kClassWave, hlist, nheavy, tcap, s);
      if (!st) st = launch_light<kLightThreads, false>(A, lists + stride, h.ccount[2], 2 * kClassBlockS, hlist, nheavy, tcap, s);
      if (!st) st = launch_light<kLightThreads, false>(A, lists + 2 * stride, h.ccount[3], kClassBlockL, hlist, nheavy, tcap, s);
    }
    if (st) break;
    // heavy count after the light passes (they may hand clusters over)
    const uint32_t heavy0 = h.ccount[4];
    if (hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = LP_EDEVICE; break; }
    if (getenv("LPGPU_DEBUG"))
      fprintf(stderr, "[lpgpu] contract n=%d nc=%d classes wave %u blockS %u blockL %u heavy %u (+%u handed over)\n",
              n, nc, h.ccount[1], h.ccount[2], h.ccount[3], heavy0, h.ccount[4] - heavy0);
    Heavy hv{};
    int32_t T = 0;
    uint64_t* tscan = nullptr;
    const int32_t H = (int32_t)h.ccount[4];
    if (H > 0) {
      st = g->compressed ? contract_heavy<true>(A, lists + 3 * stride, H, dsum, &hv, &T, &tscan, sc)
                         : contract_heavy<false>(A, lists + 3 * stride, H, dsum, &hv, &T, &tscan, sc);
      if (st) break;
    }
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
    hipLaunchKernelGGL(k_place_light, dim3(grid_for((int64_t)nc * kWave, 256, 65536)), dim3(256), 0, s, cg->xadj,
                       tbase, tcap, tb, tw, nc, cg->adjncy, cg->adjwgt);
    if (T > 0)
      hipLaunchKernelGGL(k_place_heavy, dim3(grid_for((int64_t)T * kWave, 256, 65536)), dim3(256), 0, s, hv, T, tscan,
                         cg->xadj, cg->adjncy, cg->adjwgt);
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
      hipLaunchKernelGGL(k_wdeg, dim3(grid_for((int64_t)cg->n * kWave, 256, 4096)), dim3(256), 0, s, cg->xadj,
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
