// Cluster contraction (Section IV-B of the paper).
//
// Coarse IDs are the ranks of the nonempty labels (increasing label order).
// The coarse neighbourhood of a coarse vertex a is the summed weight of the
// fine edges leaving cluster a, keyed by the coarse ID of the other end,
// sorted by that ID. Re-planned for gfx950 in three passes:
//  1. record pass: every fine vertex reserves a slice of its cluster's record
//     region with one atomic, and the edge visitor of the rating path (lane,
//     tile and hub-piece decoders over the graph's cached plan) writes one
//     (coarse ID, weight) record per neighbour (coarse ID -1 for edges inside
//     the cluster).
//  2. aggregation, following the paper's two-phase aggregation
//     (Section IV-B1): light clusters are aggregated by one wavefront or
//     workgroup from their contiguous records in an LDS hash table, sorted
//     in LDS and written back in place; heavy clusters first group their
//     records by coarse-ID partition (cut at quantiles of a sample of their
//     IDs) in 4096-record chunks, then one workgroup per (cluster, partition)
//     aggregates and sorts that partition. Partitions are ID ranges, so their
//     outputs concatenate in order.
//  3. a prefix sum over the coarse degrees places every neighbourhood.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "decode.h"
#include "graph.h"

namespace lp {
// Degrees of g's vertices, kept in g's cached plan (built here if needed).
lp_status plan_degrees(const lp_graph* g, const int32_t** deg, hipStream_t s);
lp_status visit_edges_records(const lp_graph* g, const int32_t* map, const uint64_t* rbase, const uint64_t* voff,
                              Rec* rec, hipStream_t s);

namespace {

constexpr uint32_t kErrLabel = 1, kErrOverflow = 2, kErrFormat = 4;
constexpr uint32_t kClassWave = 256;     // records per wavefront-cluster
constexpr uint32_t kClassBlockS = 1024;  // records per workgroup-cluster, small table
constexpr uint32_t kClassBlockL = 2048;  // records per workgroup-cluster, large table
constexpr uint32_t kHeavyChunk = 16384;  // records per partitioning chunk (at least)
constexpr uint32_t kMaxChunks = 1024;    // chunks per heavy cluster (at most: larger chunks beyond)
constexpr int kHeavyUnroll = 8;          // records in flight per thread while partitioning
constexpr uint32_t kHeavyTable = 2048;   // LDS entries of a heavy (cluster, partition) task
constexpr uint32_t kHeavyPart = 896;     // records per heavy partition (target; below kHeavyTable / 2)
constexpr uint32_t kMaxHeavyParts = 4096;
constexpr uint32_t kHeavySample = 2048;  // records sampled per heavy cluster for the partition splitters
constexpr int kLightThreads = 256;
constexpr int kReduceThreads = 256;
constexpr uint64_t kBigTask = 16384;  // records of a task reduced by the wide configuration
constexpr int kBigThreads = 1024;
constexpr uint32_t kBigTable = 8192;


// ------------------------------------------------------------- setup -----
__global__ void k_check_mark(const int32_t* C, int32_t n, uint32_t* flags, uint32_t* err) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = C[u];
    if (c < 0 || c >= n) atomicOr(err, kErrLabel);
    else flags[c] = 1;
  }
}

__global__ void k_map(const int32_t* C, int32_t n, const uint32_t* id, const int32_t* deg, const int32_t* vwgt,
                      int32_t* map, unsigned long long* vw, unsigned long long* dsum) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = (int32_t)id[C[u]];
    map[u] = a;
    atomicAdd(&vw[a], (unsigned long long)(vwgt ? vwgt[u] : 1));
    if (deg[u]) atomicAdd(&dsum[a], (unsigned long long)deg[u]);
  }
}

// Reserves each vertex's slice of its cluster's record region.
__global__ void k_reserve(const int32_t* map, const int32_t* deg, int32_t n, unsigned long long* cursor,
                          uint64_t* voff) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t d = deg[u];
    if (d) voff[u] = atomicAdd(&cursor[map[u]], (unsigned long long)d);
  }
}

// Class 0: no records; 1: wavefront; 2, 3: workgroup (small / large table);
// 4: heavy. Staging capacity of light classes = min(dsum, nc - 1).
__global__ void k_cclass(const unsigned long long* dsum, const unsigned long long* vw, int32_t nc, uint64_t* tcap,
                         uint8_t* cls, int32_t* vwgt_out, uint32_t* err) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nc; a += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t d = dsum[a];
    const uint8_t c = d == 0 ? 0 : d <= kClassWave ? 1 : d <= kClassBlockS ? 2 : d <= kClassBlockL ? 3 : 4;
    cls[a] = c;
    tcap[a] = std::min<uint64_t>(d, (uint64_t)nc - 1);
    const unsigned long long w = vw[a];
    if (w > 0x7FFFFFFFull) atomicOr(err, kErrOverflow);
    vwgt_out[a] = (int32_t)w;
  }
}

// Appends every coarse vertex of class 1..4 to its class list: a workgroup
// ranks 2048 vertices per step with wavefront ballots and takes one global
// atomic per class per step.
__global__ __launch_bounds__(256) void k_class_list(const uint8_t* cls, int32_t nc, uint32_t* counters, int32_t* lists,
                                                    int64_t stride) {
  constexpr int kItems = 8;
  __shared__ uint32_t wcnt[4][4];  // [wave][class - 1], then exclusive offsets
  __shared__ uint32_t gbase[4];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (int64_t blk = (int64_t)blockIdx.x * 256 * kItems; blk < nc; blk += (int64_t)gridDim.x * 256 * kItems) {
    int c[kItems];
    uint32_t pos[kItems];
    uint32_t run[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int64_t a = blk + (int64_t)i * 256 + threadIdx.x;
      c[i] = a < nc ? cls[a] : 0;
      pos[i] = 0;
#pragma unroll
      for (int k = 1; k <= 4; ++k) {
        const uint64_t m = __ballot(c[i] == k);
        if (c[i] == k) pos[i] = run[k - 1] + (uint32_t)__popcll(m & lanemask_lt());
        run[k - 1] += (uint32_t)__popcll(m);
      }
    }
    if (lane == 0)
      for (int k = 0; k < 4; ++k) wcnt[w][k] = run[k];
    __syncthreads();
    if (threadIdx.x < 4) {
      const int k = threadIdx.x;
      uint32_t tot = 0;
      for (int v = 0; v < 4; ++v) {
        const uint32_t x = wcnt[v][k];
        wcnt[v][k] = tot;
        tot += x;
      }
      gbase[k] = tot ? atomicAdd(&counters[k + 1], tot) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      if (c[i] == 0) continue;
      const int k = c[i] - 1;
      lists[(int64_t)k * stride + gbase[k] + wcnt[w][k] + pos[i]] = (int32_t)(blk + (int64_t)i * 256 + threadIdx.x);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t ceil_log2(uint32_t x) { return x <= 1 ? 0 : 32 - __clz(x - 1); }

// Table values: 64-bit sums, or 32-bit sums where no sum can reach 2^31 (a
// graph with unit edge weights and fewer than 2^31 directed edges).
__device__ __forceinline__ void tbl_val_add(unsigned long long* v, int64_t w) {
  atomicAdd(v, (unsigned long long)w);
}
__device__ __forceinline__ void tbl_val_add(int64_t* v, int64_t w) {
  atomicAdd((unsigned long long*)v, (unsigned long long)w);
}
__device__ __forceinline__ void tbl_val_add(uint32_t* v, int64_t w) { atomicAdd(v, (uint32_t)w); }

// Adds w to key b's slot. With `guard`, a new key first reserves one of
// `limit` entries (a shared counter) and sets *overflow when none is left;
// without it the caller guarantees that the table cannot fill (at most half
// its slots distinct keys), and the contended counter is skipped.
template <typename V>
__device__ __forceinline__ void tbl_add_guarded(int32_t* keys, V* vals, uint32_t mask, uint32_t shift, int32_t b,
                                                int64_t w, uint32_t limit, uint32_t* distinct, uint32_t* overflow,
                                                bool guard = true) {
  uint32_t h = slot_hash((uint32_t)b) >> shift;
  bool reserved = !guard;
  while (true) {
    const int32_t k = keys[h];
    if (k == b) {
      tbl_val_add(&vals[h], w);
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
        tbl_val_add(&vals[h], w);
        return;
      }
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long x, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)x, m, kWave), hi = __shfl_xor((uint32_t)(x >> 32), m, kWave);
  return ((unsigned long long)hi << 32) | lo;
}

// Sorts k distinct 64-bit values a[0..k) ascending in LDS: every wavefront
// sorts runs of 64 in registers (bitonic network over lane shuffles), then
// runs are merged pairwise, each element placed at its run position plus its
// rank in the partner run (binary search), alternating between a and b.
// Returns the buffer that holds the result; b needs k entries.
template <int NT>
__device__ unsigned long long* lds_sort_u64(unsigned long long* a, unsigned long long* b, uint32_t k) {
  constexpr int NW = NT / kWave;
  const int lane = lane_id();
  const int w = NT == kWave ? 0 : (int)(threadIdx.x / kWave);
  for (uint32_t c = (uint32_t)w * kWave; c < k; c += NW * kWave) {
    const uint32_t i = c + lane;
    unsigned long long x = i < k ? a[i] : ~0ull;
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const unsigned long long y = shfl_xor_u64(x, stride);
        const bool up = (lane & size) == 0;
        const bool lower = (lane & stride) == 0;
        x = (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
      }
    }
    if (i < k) a[i] = x;
  }
  group_sync<NT>();
  const int tid = group_tid<NT>();
  unsigned long long *src = a, *dst = b;
  for (uint32_t R = kWave; R < k; R <<= 1) {
    for (uint32_t i = tid; i < k; i += NT) {
      const unsigned long long x = src[i];
      const uint32_t r = i / R, p = i - r * R;
      const uint32_t ps = (r ^ 1u) * R;
      uint32_t rank = 0;
      if (ps < k) {
        uint32_t lo = 0, hi = min(R, k - ps);
        const unsigned long long* q = src + ps;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (q[mid] < x) lo = mid + 1;
          else hi = mid;
        }
        rank = lo;
      }
      dst[(r & ~1u) * R + p + rank] = x;
    }
    group_sync<NT>();
    unsigned long long* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Writes the k distinct (key << 32 | value) entries of a[] to `out` in key
// order by bucket ranking: entries go to B buckets by a monotone map of their
// key into [0, B) (so bucket order is key order), are scattered into b[] by
// bucket, and each takes its bucket's start plus the number of smaller keys in
// its bucket (ranked into a[], then copied out in order). Needs cnt[B] of LDS
// besides a and b (k entries each). Returns false, having written nothing,
// when the keys are so skewed that ranking inside the buckets would cost more
// than kRankBudget comparisons per entry, so that the caller merge-sorts.
constexpr uint32_t kRankBudget = 32;
constexpr uint32_t kBucketBins = 1024;  // LDS bucket counters of a heavy reduction workgroup

template <int NT>
__device__ bool bucket_rank_write(unsigned long long* a, unsigned long long* b, uint32_t k, uint32_t* cnt,
                                  uint32_t B, Rec* out, int32_t* scan_sm, uint32_t* red) {
  const int tid = group_tid<NT>();
  // key range
  uint32_t mn = 0xFFFFFFFFu, mx = 0;
  for (uint32_t i = tid; i < k; i += NT) {
    const uint32_t key = (uint32_t)(a[i] >> 32);
    mn = min(mn, key);
    mx = max(mx, key);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, d, kWave));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, kWave));
  }
  constexpr int NW = NT / kWave;
  if (lane_id() == 0) {
    red[2 * (tid / kWave)] = mn;
    red[2 * (tid / kWave) + 1] = mx;
  }
  for (uint32_t q = tid; q < B; q += NT) cnt[q] = 0;
  group_sync<NT>();
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    mn = min(mn, red[2 * w]);
    mx = max(mx, red[2 * w + 1]);
  }
  const float scale = (float)B / ((float)(mx - mn) + 1.0f);
  auto bucket = [&](unsigned long long x) {
    const uint32_t q = (uint32_t)((float)((uint32_t)(x >> 32) - mn) * scale);
    return q < B ? q : B - 1;
  };
  for (uint32_t i = tid; i < k; i += NT) atomicAdd(&cnt[bucket(a[i])], 1u);
  group_sync<NT>();
  // ranking costs the sum of the squared bucket sizes; exclusive scan of the
  // counts (B / NT consecutive per thread)
  const uint32_t per = (B + NT - 1) / NT;
  const uint32_t q0 = min(B, (uint32_t)tid * per), q1 = min(B, q0 + per);
  uint32_t sq = 0;
  int32_t sum = 0;
  for (uint32_t q = q0; q < q1; ++q) {
    sq += cnt[q] * cnt[q];
    sum += (int32_t)cnt[q];
  }
  sq = wave_reduce_add(sq);
  group_sync<NT>();
  if (lane_id() == 0) red[tid / kWave] = sq;
  int32_t tot;
  int32_t run = block_incl_scan_add<NT, int32_t>(sum, scan_sm, &tot) - sum;
  sq = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) sq += red[w];
  if (sq > kRankBudget * k) {
    group_sync<NT>();
    return false;
  }
  for (uint32_t q = q0; q < q1; ++q) {
    const uint32_t c = cnt[q];
    cnt[q] = (uint32_t)run;
    run += (int32_t)c;
  }
  group_sync<NT>();
  // scatter by bucket: afterwards cnt[q] is the end of bucket q
  for (uint32_t i = tid; i < k; i += NT) {
    const unsigned long long x = a[i];
    b[atomicAdd(&cnt[bucket(x)], 1u)] = x;
  }
  group_sync<NT>();
  // ranks into a[] (free once scattered), then one coalesced copy out
  unsigned long long* sorted = a;
  for (uint32_t j = tid; j < k; j += NT) {
    const unsigned long long x = b[j];
    const uint32_t q = bucket(x);
    const uint32_t s0 = q ? cnt[q - 1] : 0u, e0 = cnt[q];
    uint32_t r = s0;
    for (uint32_t m = s0; m < e0; ++m) r += b[m] < x;
    sorted[r] = x;
  }
  group_sync<NT>();
  for (uint32_t i = tid; i < k; i += NT) {
    const unsigned long long x = sorted[i];
    out[i] = Rec{(int32_t)(x >> 32), (int32_t)(uint32_t)x};
  }
  group_sync<NT>();
  return true;
}

// Writes the table's entries to `out` sorted by key: every thread takes its
// (strided) slots into registers, a prefix count compacts the entries to pk
// as (key << 32 | value) pairs, which lds_sort_u64 sorts. Returns the entry
// count. cap <= NT * SLOTS and the table never holds more than cap / 2
// entries; pk is the start of the table's LDS region (cap * 8 bytes or more:
// keys and values), so both sort buffers fit in it once the slots are read.
template <int NT, int SLOTS, typename V>
__device__ uint32_t compact_sort_write(int32_t* keys, V* vals, uint32_t cap, Rec* out, uint32_t* err,
                                       int32_t* scan_sm, unsigned long long* pk, uint32_t* bcnt = nullptr,
                                       uint32_t* red = nullptr) {
  const int tid = group_tid<NT>();
  int32_t kk[SLOTS];
  int64_t vv[SLOTS];
  int32_t c = 0;
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) {
    const uint32_t q = (uint32_t)tid + (uint32_t)i * NT;
    kk[i] = kEmpty;
    vv[i] = 0;
    if (q < cap) {
      kk[i] = keys[q];
      vv[i] = (int64_t)vals[q];
      c += kk[i] != kEmpty;
    }
  }
  int32_t tot;
  int32_t o = block_incl_scan_add<NT, int32_t>(c, scan_sm, &tot) - c;
  group_sync<NT>();
#pragma unroll
  for (int i = 0; i < SLOTS; ++i)
    if (kk[i] != kEmpty) {
      if (vv[i] > 0x7FFFFFFFll) atomicOr(err, kErrOverflow);
      pk[o++] = ((unsigned long long)(uint32_t)kk[i] << 32) | (uint32_t)(int32_t)vv[i];
    }
  const uint32_t cnt = (uint32_t)tot;
  group_sync<NT>();
  if (bcnt && cnt > kWave) {
    uint32_t B = 64;
    while (B < cnt && B < kBucketBins) B <<= 1;
    if (bucket_rank_write<NT>(pk, pk + cnt, cnt, bcnt, B, out, scan_sm, red)) return cnt;
  }
  const unsigned long long* sorted = lds_sort_u64<NT>(pk, pk + cnt, cnt);
  for (uint32_t i = tid; i < cnt; i += NT) {
    const unsigned long long x = sorted[i];
    out[i] = Rec{(int32_t)(x >> 32), (int32_t)(uint32_t)x};
  }
  group_sync<NT>();
  return cnt;
}

// Writes the nonzero entries of a direct array over coarse IDs [lo, lo +
// width) in ID order; returns their number.
template <int NT, typename V>
__device__ uint32_t dense_write(const V* vals, uint32_t width, uint64_t lo, Rec* out, uint32_t* err,
                                int32_t* scan_sm) {
  const int tid = group_tid<NT>();
  const uint32_t per = (width + NT - 1) / NT;
  const uint32_t q0 = min(width, (uint32_t)tid * per), q1 = min(width, q0 + per);
  int32_t c = 0;
  for (uint32_t q = q0; q < q1; ++q) c += vals[q] != 0;
  int32_t tot;
  int32_t o = block_incl_scan_add<NT, int32_t>(c, scan_sm, &tot) - c;
  for (uint32_t q = q0; q < q1; ++q) {
    const int64_t v = (int64_t)vals[q];
    if (!v) continue;
    if (v > 0x7FFFFFFFll) atomicOr(err, kErrOverflow);
    out[o++] = Rec{(int32_t)(lo + q), (int32_t)v};
  }
  group_sync<NT>();
  return (uint32_t)tot;
}

// ------------------------------------------------------------- light -----
struct AggArgs {
  const uint64_t* rbase;
  const unsigned long long* dsum;
  const uint64_t* tcap;
  Rec* rec;
  uint64_t* cdeg;  // coarse degree per coarse vertex
  uint32_t* err;
  int32_t nc;
};

template <int NT>
struct LightSmem {
  int32_t scan[NT / kWave];
  uint32_t distinct;
  uint32_t overflow;
};

// Light clusters: NT = 64, one cluster per wavefront (4 per workgroup);
// NT = 256, one cluster per workgroup. The table has the next power of two
// >= 2 * min(dsum, nc - 1) entries, at most tmax; if that capacity was
// clipped and the cluster turns out to have more than half of it distinct
// neighbours, the cluster is appended to the heavy list instead.
template <int NT, typename V>
__global__ __launch_bounds__(kLightThreads) void k_contract_light(AggArgs A, const int32_t* list, int32_t cnt,
                                                                  uint32_t tmax, int32_t* heavy_list,
                                                                  uint32_t* nheavy) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  constexpr int G = kLightThreads / NT;
  const int gi = (int)(threadIdx.x / NT);
  const int tid = group_tid<NT>();
  const size_t per = ((size_t)tmax * (4 + sizeof(V)) + sizeof(LightSmem<NT>) + 15) & ~size_t(15);
  uint8_t* base = smem_raw + gi * per;
  V* vals = (V*)base;
  int32_t* keys = (int32_t*)(base + (size_t)tmax * sizeof(V));
  LightSmem<NT>& sm = *(LightSmem<NT>*)(base + (size_t)tmax * (4 + sizeof(V)));
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
    Rec* r = A.rec + A.rbase[a];
    const uint32_t d = (uint32_t)A.dsum[a];
    for (uint32_t i = tid; i < d; i += NT) {
      const Rec x = r[i];
      if (x.b >= 0)
        tbl_add_guarded(keys, vals, mask, shift, x.b, (int64_t)x.w, limit, &sm.distinct, &sm.overflow, limit < cap);
    }
    group_sync<NT>();
    if (sm.overflow) {
      if (tid == 0) heavy_list[atomicAdd(nheavy, 1u)] = a;
      group_sync<NT>();
      continue;
    }
    constexpr int kSlots = NT == kWave ? 8 : 16;
    const uint32_t k = compact_sort_write<NT, kSlots, V>(keys, vals, cap, r, A.err, sm.scan, (unsigned long long*)base);
    if (tid == 0) A.cdeg[a] = k;
    group_sync<NT>();
  }
}

// ------------------------------------------------------------- heavy -----
struct Heavy {
  const int32_t* clusters;  // heavy cluster -> coarse vertex
  const int32_t* parts;     // P per heavy cluster
  const uint32_t* cbase;    // first chunk of each heavy cluster (H + 1)
  const uint32_t* tbase;    // first task of each heavy cluster (H + 1)
  const uint64_t* pbase;    // first chunk-table entry of each heavy cluster
  const int2* chunks;       // (heavy cluster, chunk index)
  const int2* tasks;        // (heavy cluster, partition)
  Rec* rec2;                // records regrouped by task, at the task's staging base
  uint32_t* ctab;           // per chunk: P counts, then the chunk's first position inside each task
  uint64_t* tcnt;           // records per task, then (scanned) staging base
  Rec* out;                 // heavy staging
  uint64_t* tdeg;           // distinct coarse neighbours per task
  int32_t* bnd;             // P + 1 coarse-ID boundaries per heavy cluster (at tbase[h] + h)
};

// Records per partitioning chunk of a heavy cluster of d records: at least
// kHeavyChunk, and few enough chunks that the (chunk, partition) count table
// of a cluster stays within kMaxChunks rows.
__host__ __device__ inline uint64_t chunk_size(uint64_t d) {
  return std::max<uint64_t>(kHeavyChunk, (d + kMaxChunks - 1) / kMaxChunks);
}

__global__ void k_heavy_meta(const int32_t* hl, int32_t H, const unsigned long long* dsum, int32_t nc, int32_t* parts,
                             uint32_t* ccount, uint32_t* pcount, uint64_t* tabcount) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = hl[h];
    const uint64_t d = dsum[a];
    const uint32_t P = (uint32_t)std::min<uint64_t>(kMaxHeavyParts, std::max<uint64_t>(1, (d + kHeavyPart - 1) / kHeavyPart));
    const uint64_t csz = chunk_size(d);
    const uint32_t nch = (uint32_t)((d + csz - 1) / csz);
    parts[h] = (int32_t)P;
    pcount[h] = P;
    ccount[h] = nch;
    tabcount[h] = (uint64_t)nch * P;
  }
}

__global__ void k_heavy_lists(int32_t H, const int32_t* parts, const uint32_t* cbase, const uint32_t* tbase,
                              int2* chunks, int2* tasks) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    for (uint32_t c = cbase[h]; c < cbase[h + 1]; ++c) chunks[c] = make_int2((int)h, (int)(c - cbase[h]));
    for (int32_t p = 0; p < parts[h]; ++p) tasks[tbase[h] + p] = make_int2((int)h, p);
  }
}

// Partition splitters of every heavy cluster: a sample of up to kHeavySample
// records, 256 per partition (evenly spaced over the cluster's records), is
// sorted and cut at quantiles, so the partitions hold about equal numbers of
// records however skewed the coarse IDs are. Only records with a coarse
// neighbour count: their number is estimated from the sample, and
// partitions beyond about one per kHeavyPart of them stay empty. Partition p
// holds IDs [bnd[p], bnd[p+1]).
__global__ __launch_bounds__(256) void k_heavy_splitters(AggArgs A, Heavy hv, int32_t H) {
  __shared__ unsigned long long sa[kHeavySample], sb[kHeavySample];
  __shared__ int32_t scan[4];
  for (int64_t h = blockIdx.x; h < H; h += gridDim.x) {
    const int32_t a = hv.clusters[h];
    const uint32_t P = (uint32_t)hv.parts[h];
    const uint64_t d = A.dsum[a];
    const uint32_t S = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(kHeavySample, 256ull * P), d);
    const Rec* r = A.rec + A.rbase[a];
    int32_t* bnd = hv.bnd + hv.tbase[h] + h;
    int32_t valid = 0;
    for (uint32_t j = threadIdx.x; j < S; j += 256) {
      const int32_t b = r[(uint64_t)j * d / S].b;
      valid += b >= 0;
      // intra-cluster records (b < 0) sort last and are not counted
      sa[j] = ((unsigned long long)(b >= 0 ? (uint32_t)b : 0xFFFFFFFFu) << 32) | j;
    }
    int32_t V;
    (void)block_incl_scan_add<256, int32_t>(valid, scan, &V);
    __syncthreads();
    const unsigned long long* srt = lds_sort_u64<256>(sa, sb, S);
    // about kHeavyPart records with a coarse neighbour per partition
    const uint64_t want = ((uint64_t)V * d + (uint64_t)S * kHeavyPart - 1) / ((uint64_t)S * kHeavyPart);
    const uint32_t Pe = (uint32_t)std::min<uint64_t>(P, std::max<uint64_t>(1, want));
    for (uint32_t p = threadIdx.x; p <= P; p += 256) {
      int32_t v;
      if (p == 0) v = 0;
      else if (p >= Pe || V == 0) v = A.nc;
      else v = (int32_t)(srt[(uint64_t)p * V / Pe] >> 32);
      bnd[p] = v;
    }
    __syncthreads();
  }
}

// Partition of coarse ID b: the number of inner boundaries <= b.
__device__ __forceinline__ uint32_t split_part(int32_t b, const int32_t* bnd, uint32_t P) {
  uint32_t lo = 1, hi = P;  // first inner boundary > b
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (bnd[mid] <= b) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// One workgroup per chunk: the chunk's records per partition (records inside
// the cluster are not counted), written to the chunk's row of the table.
__global__ __launch_bounds__(256) void k_heavy_hist(AggArgs A, Heavy hv, int32_t nchunks) {
  __shared__ uint32_t hist[kMaxHeavyParts];
  __shared__ int32_t sbnd[kMaxHeavyParts + 1];
  for (int64_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
    const int2 ch = hv.chunks[ci];
    const int32_t h = ch.x;
    const int32_t a = hv.clusters[h];
    const uint32_t P = (uint32_t)hv.parts[h];
    const uint64_t d = A.dsum[a], csz = chunk_size(d);
    const uint64_t off = (uint64_t)ch.y * csz;
    const uint32_t len = (uint32_t)std::min<uint64_t>(csz, d - off);
    const Rec* src = A.rec + A.rbase[a] + off;
    const int32_t* bnd = hv.bnd + hv.tbase[h] + h;
    for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) hist[j] = 0;
    for (uint32_t j = threadIdx.x; j <= P; j += blockDim.x) sbnd[j] = bnd[j];
    __syncthreads();
    for (uint32_t i0 = 0; i0 < len; i0 += 256 * kHeavyUnroll) {
      Rec x[kHeavyUnroll];
#pragma unroll
      for (int u = 0; u < kHeavyUnroll; ++u) {
        const uint32_t i = i0 + u * 256 + threadIdx.x;
        x[u] = i < len ? src[i] : Rec{-1, 0};
      }
#pragma unroll
      for (int u = 0; u < kHeavyUnroll; ++u)
        if (x[u].b >= 0) atomicAdd(&hist[split_part(x[u].b, sbnd, P)], 1u);
    }
    __syncthreads();
    uint32_t* tab = hv.ctab + hv.pbase[h] + (uint64_t)ch.y * P;
    for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) tab[j] = hist[j];
    __syncthreads();
  }
}

// Per (cluster, partition) task (wave per task): its record count, and in
// place of each chunk's count the chunk's first position inside the task
// (exclusive scan over the cluster's chunks).
__global__ __launch_bounds__(256) void k_heavy_count(Heavy hv, int32_t ntasks) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t t = wid; t < ntasks; t += nw) {
    const int2 task = hv.tasks[t];
    const int32_t h = task.x;
    const uint32_t p = (uint32_t)task.y;
    const uint32_t P = (uint32_t)hv.parts[h];
    const uint32_t nch = hv.cbase[h + 1] - hv.cbase[h];
    uint32_t* tab = hv.ctab + hv.pbase[h];
    uint64_t carry = 0;
    for (uint32_t k0 = 0; k0 < nch; k0 += kWave) {
      const uint32_t k = k0 + lane;
      const uint64_t v = k < nch ? tab[(uint64_t)k * P + p] : 0;
      const uint64_t inc = wave_incl_scan_add(v);
      if (k < nch) tab[(uint64_t)k * P + p] = (uint32_t)(carry + inc - v);
      carry += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) hv.tcnt[t] = carry;
  }
}

// One workgroup per chunk: every record of the chunk goes to its task's
// contiguous range of rec2 (task base + the chunk's position inside the task
// + its rank among the chunk's records of that partition). The order inside
// a task varies from run to run; the reduction does not depend on it.
__global__ __launch_bounds__(256) void k_heavy_scatter(AggArgs A, Heavy hv, int32_t nchunks) {
  __shared__ unsigned long long cur[kMaxHeavyParts];
  __shared__ int32_t sbnd[kMaxHeavyParts + 1];
  for (int64_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
    const int2 ch = hv.chunks[ci];
    const int32_t h = ch.x;
    const int32_t a = hv.clusters[h];
    const uint32_t P = (uint32_t)hv.parts[h];
    const uint64_t d = A.dsum[a], csz = chunk_size(d);
    const uint64_t off = (uint64_t)ch.y * csz;
    const uint32_t len = (uint32_t)std::min<uint64_t>(csz, d - off);
    const Rec* src = A.rec + A.rbase[a] + off;
    const int32_t* bnd = hv.bnd + hv.tbase[h] + h;
    const uint32_t* tab = hv.ctab + hv.pbase[h] + (uint64_t)ch.y * P;
    const uint64_t* tb = hv.tcnt + hv.tbase[h];
    for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) cur[j] = tb[j] + tab[j];
    for (uint32_t j = threadIdx.x; j <= P; j += blockDim.x) sbnd[j] = bnd[j];
    __syncthreads();
    for (uint32_t i0 = 0; i0 < len; i0 += 256 * kHeavyUnroll) {
      Rec x[kHeavyUnroll];
#pragma unroll
      for (int u = 0; u < kHeavyUnroll; ++u) {
        const uint32_t i = i0 + u * 256 + threadIdx.x;
        x[u] = i < len ? src[i] : Rec{-1, 0};
      }
#pragma unroll
      for (int u = 0; u < kHeavyUnroll; ++u)
        if (x[u].b >= 0) hv.rec2[atomicAdd(&cur[split_part(x[u].b, sbnd, P)], 1ull)] = x[u];
    }
    __syncthreads();
  }
}

template <int NT>
struct ReduceSmem {
  int32_t scan[NT / kWave];
  uint32_t red[2 * (NT / kWave)];
  uint32_t distinct;
  uint32_t overflow;
  uint32_t bcnt[kBucketBins];
};

// One workgroup of NT threads per (cluster, partition): aggregate the
// partition's records in an LDS table of TABLE entries over coarse-ID windows
// (a window whose distinct count exceeds half the table is halved and
// retried), emitting each window sorted. The table is sized by the task's
// record count. With `list`, the workgroups take the listed tasks; without,
// every task of at most max_rec records (larger ones are listed for the wide
// configuration).
template <int NT, uint32_t TABLE, typename V>
__global__ __launch_bounds__(NT) void k_heavy_reduce(AggArgs A, Heavy hv, const int32_t* list, int32_t ntasks,
                                                     uint64_t max_rec) {
  extern __shared__ __align__(16) uint8_t smem_raw[];
  V* vals = (V*)smem_raw;
  int32_t* keys = (int32_t*)(smem_raw + (size_t)TABLE * sizeof(V));
  ReduceSmem<NT>& sm = *(ReduceSmem<NT>*)(smem_raw + (size_t)TABLE * (4 + sizeof(V)));
  const int tid = threadIdx.x;
  for (int64_t i = blockIdx.x; i < ntasks; i += gridDim.x) {
    const int64_t t = list ? (int64_t)list[i] : i;
    const uint64_t obase = hv.tcnt[t];
    const uint64_t nrec = hv.tcnt[t + 1] - obase;
    if (!list && nrec > max_rec) continue;
    if (nrec == 0) {
      if (tid == 0) hv.tdeg[t] = 0;
      continue;
    }
    const int2 task = hv.tasks[t];
    const int32_t h = task.x;
    const uint32_t p = (uint32_t)task.y;
    const int32_t* bnd = hv.bnd + hv.tbase[h] + h;
    const uint64_t lo_p = (uint64_t)bnd[p], hi_p = (uint64_t)bnd[p + 1];
    const uint32_t logc =
        min(ceil_log2(TABLE), max(6u, ceil_log2((uint32_t)std::min<uint64_t>(2 * nrec + 2, TABLE))));
    const uint32_t tcap = 1u << logc, mask = tcap - 1, shift = 32 - logc;
    const uint32_t limit = tcap / 2;
    const Rec* src = hv.rec2 + obase;
    uint64_t written = 0;
    uint64_t lo = lo_p, width = hi_p - lo_p;
    while (lo < hi_p) {
      const uint64_t hi = std::min<uint64_t>(hi_p, lo + width);
      // a window at most TABLE IDs wide is summed in a direct array
      // indexed by b - lo: no hashing, no overflow, no sort
      const bool dense = hi - lo <= TABLE;
      if (dense) {
        for (uint32_t q = tid; q < (uint32_t)(hi - lo); q += NT) vals[q] = 0;
      } else {
        for (uint32_t q = tid; q < tcap; q += NT) {
          keys[q] = kEmpty;
          vals[q] = 0;
        }
      }
      if (tid == 0) {
        sm.distinct = 0;
        sm.overflow = 0;
      }
      __syncthreads();
      // kHeavyUnroll records in flight per thread; each thread sums a run of
      // equal coarse IDs in registers and adds it to the table when the ID
      // changes, so records of one hot neighbour cost few LDS atomics
      const bool guard = 2 * nrec + 2 > tcap;
      int32_t rk = -1;
      int64_t rs = 0;
      auto flush = [&]() {
        if (rk < 0) return;
        if (dense)
          tbl_val_add(&vals[(uint64_t)rk - lo], rs);
        else
          tbl_add_guarded(keys, vals, mask, shift, rk, rs, limit, &sm.distinct, &sm.overflow, guard);
      };
      for (uint64_t j0 = 0; j0 < nrec; j0 += (uint64_t)NT * kHeavyUnroll) {
        Rec x[kHeavyUnroll];
#pragma unroll
        for (int u = 0; u < kHeavyUnroll; ++u) {
          const uint64_t j = j0 + (uint64_t)u * NT + tid;
          x[u] = j < nrec ? src[j] : Rec{-1, 0};
        }
#pragma unroll
        for (int u = 0; u < kHeavyUnroll; ++u) {
          if ((uint64_t)x[u].b >= lo && (uint64_t)x[u].b < hi) {
            if (x[u].b == rk) {
              rs += x[u].w;
            } else {
              flush();
              rk = x[u].b;
              rs = x[u].w;
            }
          }
        }
        if (!dense && *(volatile uint32_t*)&sm.overflow) break;
      }
      flush();
      __syncthreads();
      if (!dense && sm.overflow) {
        width = std::max<uint64_t>(TABLE, (hi - lo) / 2);
        __syncthreads();
        continue;
      }
      Rec* dst = hv.out + obase + written;
      const uint32_t k = dense ? dense_write<NT, V>(vals, (uint32_t)(hi - lo), lo, dst, A.err, sm.scan)
                               : compact_sort_write<NT, TABLE / NT, V>(keys, vals, tcap, dst, A.err, sm.scan,
                                                                             (unsigned long long*)smem_raw, sm.bcnt,
                                                                             sm.red);
      written += k;
      // the next window keeps the width that fitted, twice as wide when it
      // used under a quarter of the table
      width = (hi - lo) * (k < limit / 4 ? 2 : 1);
      lo = hi;
      __syncthreads();
    }
    if (tid == 0) hv.tdeg[t] = written;
    __syncthreads();
  }
}

// Tasks of more than thr records, in any order (they go to the wide
// reduction configuration).
__global__ void k_heavy_big(const uint64_t* tcnt, int32_t T, uint64_t thr, int32_t* list, uint32_t* cnt) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += (int64_t)gridDim.x * blockDim.x)
    if (tcnt[t + 1] - tcnt[t] > thr) list[atomicAdd(cnt, 1u)] = (int32_t)t;
}

__global__ void k_heavy_cdeg(Heavy hv, int32_t H, uint64_t* cdeg) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    uint64_t s = 0;
    for (uint32_t t = hv.tbase[h]; t < hv.tbase[h + 1]; ++t) s += hv.tdeg[t];
    cdeg[hv.clusters[h]] = s;
  }
}

// ---------------------------------------------------------- placement ----
// Light clusters: their aggregated neighbourhood sits at the start of their
// record region (wave per coarse vertex; heavy clusters are skipped). Also
// gathers the largest weighted degree and degree of the light coarse vertices
// (mx[0], mx[1]).
__global__ __launch_bounds__(256) void k_place_light(const uint64_t* cx, const uint64_t* rbase, const uint8_t* heavy,
                                                     const Rec* rec, int32_t nc, int32_t* adjncy, int32_t* adjwgt,
                                                     unsigned long long* mx) {
  __shared__ unsigned long long sa[4], sb[4];
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  unsigned long long mw = 0, md = 0;
  for (int64_t a = wid; a < nc; a += nw) {
    const uint64_t o = cx[a], d = cx[a + 1] - o;
    if (d == 0 || heavy[a]) continue;
    const Rec* r = rec + rbase[a];
    int64_t sw = 0;
    for (uint64_t i = lane; i < d; i += kWave) {
      const Rec x = r[i];
      adjncy[o + i] = x.b;
      adjwgt[o + i] = x.w;
      sw += x.w;
    }
    sw = wave_reduce_add(sw);
    mw = max(mw, (unsigned long long)sw);
    md = max(md, (unsigned long long)d);
  }
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
    if (mw) atomicMax(&mx[0], mw);
    if (md) atomicMax(&mx[1], md);
  }
}

__global__ void k_mark_heavy(const int32_t* hl, int32_t H, uint8_t* heavy) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x)
    heavy[hl[h]] = 1;
}

// Heavy clusters: task t of cluster h goes after the outputs of the
// cluster's earlier partitions (wave per task); the task's weight sum is
// added to its cluster's (hsum).
__global__ __launch_bounds__(256) void k_place_heavy(Heavy hv, int32_t ntasks, const uint64_t* tdeg_scan,
                                                     const uint64_t* cx, int32_t* adjncy, int32_t* adjwgt,
                                                     unsigned long long* hsum) {
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t t = wid; t < ntasks; t += nw) {
    const int32_t h = hv.tasks[t].x;
    const int32_t a = hv.clusters[h];
    const uint64_t dst = cx[a] + (tdeg_scan[t] - tdeg_scan[hv.tbase[h]]);
    const uint64_t src = hv.tcnt[t], d = hv.tdeg[t];
    int64_t sw = 0;
    for (uint64_t j = lane; j < d; j += kWave) {
      const Rec x = hv.out[src + j];
      adjncy[dst + j] = x.b;
      adjwgt[dst + j] = x.w;
      sw += x.w;
    }
    sw = wave_reduce_add(sw);
    if (lane == 0 && sw) atomicAdd(&hsum[h], (unsigned long long)sw);
  }
}

// Largest weighted degree and degree over the heavy coarse vertices.
__global__ void k_heavy_max(Heavy hv, int32_t H, const unsigned long long* hsum, const uint64_t* cx,
                            unsigned long long* mx) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < H; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = hv.clusters[h];
    atomicMax(&mx[0], hsum[h]);
    atomicMax(&mx[1], (unsigned long long)(cx[a + 1] - cx[a]));
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

template <int NT, typename V>
lp_status launch_light(const AggArgs& A, const int32_t* list, uint32_t cnt, uint32_t tmax, int32_t* heavy_list,
                       uint32_t* nheavy, hipStream_t s) {
  if (cnt == 0) return LP_OK;
  const size_t per = ((size_t)tmax * (4 + sizeof(V)) + sizeof(LightSmem<NT>) + 15) & ~size_t(15);
  const size_t bytes = per * (kLightThreads / NT);
  auto k = k_contract_light<NT, V>;
  LP_CHECK(set_lds(k, bytes));
  hipLaunchKernelGGL(k, dim3(grid_for(cnt, kLightThreads / NT, 1u << 20)), dim3(kLightThreads), bytes, s, A, list,
                     (int32_t)cnt, tmax, heavy_list, nheavy);
  return last_error();
}

template <int NT, uint32_t TABLE, typename V>
lp_status launch_reduce(const AggArgs& A, const Heavy& hv, const int32_t* list, int32_t ntasks, uint64_t max_rec,
                        hipStream_t s) {
  const size_t bytes = (size_t)TABLE * (4 + sizeof(V)) + sizeof(ReduceSmem<NT>);
  auto k = k_heavy_reduce<NT, TABLE, V>;
  LP_CHECK(set_lds(k, bytes));
  // the listed tasks are few and long: at most as many workgroups as fit
  const uint32_t grid = list ? (uint32_t)std::min<int64_t>(ntasks, 2048) : grid_for(ntasks, 1, 1u << 20);
  hipLaunchKernelGGL(k, dim3(grid), dim3(NT), bytes, s, A, hv, list, ntasks, max_rec);
  return last_error();
}

// Diagnostics of the heavy path (LPGPU_DEBUG): reduction time, the spread of
// records over tasks, the largest tasks with their ID width and distinct
// count. Synchronises the stream.
void heavy_debug(const Heavy& hv, int32_t H, int32_t T, uint32_t nbig, hipEvent_t* ev, hipStream_t s) {
  (void)hipEventRecord(ev[2], s);
  std::vector<uint64_t> tc((size_t)T + 1), td((size_t)T);
  std::vector<int2> tk((size_t)T);
  std::vector<int32_t> bnd((size_t)T + H), parts((size_t)H);
  std::vector<uint32_t> tb((size_t)H + 1);
  (void)hipMemcpyAsync(tc.data(), hv.tcnt, tc.size() * 8, hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(td.data(), hv.tdeg, td.size() * 8, hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(tk.data(), hv.tasks, tk.size() * sizeof(int2), hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(bnd.data(), hv.bnd, bnd.size() * 4, hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(parts.data(), hv.parts, parts.size() * 4, hipMemcpyDeviceToHost, s);
  (void)hipMemcpyAsync(tb.data(), hv.tbase, tb.size() * 4, hipMemcpyDeviceToHost, s);
  (void)hipStreamSynchronize(s);
  float ms = 0.f, ms_big = 0.f;
  (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
  (void)hipEventElapsedTime(&ms_big, ev[1], ev[2]);
  for (int i = 0; i < 3; ++i) (void)hipEventDestroy(ev[i]);
  std::vector<uint64_t> nr((size_t)T);
  uint64_t tot = 0, big = 0, bigrec = 0, huge = 0, hugerec = 0, single = 0, singlerec = 0, dist = 0;
  for (int32_t t = 0; t < T; ++t) {
    nr[t] = tc[t + 1] - tc[t];
    tot += nr[t];
    dist += td[t];
    if (nr[t] > 2048) big++, bigrec += nr[t];
    if (nr[t] > 65536) huge++, hugerec += nr[t];
    const int32_t h = tk[t].x, p = tk[t].y;
    const int32_t* b = bnd.data() + tb[h] + h;
    if (b[p + 1] - b[p] == 1) single++, singlerec += nr[t];
  }
  int32_t capped = 0;
  for (int32_t h = 0; h < H; ++h) capped += parts[h] == (int32_t)kMaxHeavyParts;
  std::vector<int32_t> ord((size_t)T);
  for (int32_t t = 0; t < T; ++t) ord[t] = t;
  const int32_t top = std::min<int32_t>(T, 8);
  std::partial_sort(ord.begin(), ord.begin() + top, ord.end(), [&](int32_t a, int32_t b) { return nr[a] > nr[b]; });
  fprintf(stderr,
          "[lpgpu] heavy reduce %.3f ms, %u large tasks %.3f ms: tasks %d records %llu distinct %llu; >2048: %llu "
          "tasks %llu records; >65536: %llu tasks %llu records; single-ID tasks %llu with %llu records; clusters at "
          "the part cap %d\n",
          ms, nbig, ms_big, T, (unsigned long long)tot, (unsigned long long)dist, (unsigned long long)big,
          (unsigned long long)bigrec, (unsigned long long)huge, (unsigned long long)hugerec,
          (unsigned long long)single, (unsigned long long)singlerec, capped);
  for (int32_t i = 0; i < top; ++i) {
    const int32_t t = ord[i], h = tk[t].x, p = tk[t].y;
    const int32_t* b = bnd.data() + tb[h] + h;
    fprintf(stderr, "[lpgpu]   task %d: cluster %d part %d/%d records %llu distinct %llu ids [%d, %d)\n", t, h, p,
            parts[h], (unsigned long long)nr[t], (unsigned long long)td[t], b[p], b[p + 1]);
  }
}

// Heavy clusters: metadata, partitioning, counts, reduction. Fills the coarse
// degrees of heavy clusters and leaves what placement needs in *hv_out.
// rec2 has the layout of the record buffer.
lp_status contract_heavy(const AggArgs& A, const int32_t* hl, int32_t H, Rec* rec2, bool narrow, Heavy* hv_out,
                         int32_t* ntasks_out, uint64_t** tdeg_scan_out, Scratch& sc) {
  hipStream_t s = sc.stream();
  Heavy hv{};
  int32_t* parts = sc.alloc<int32_t>(H);
  uint32_t* cbase = sc.alloc<uint32_t>((size_t)H + 1);
  uint32_t* tbase = sc.alloc<uint32_t>((size_t)H + 1);
  uint64_t* pbase = sc.alloc<uint64_t>((size_t)H + 1);
  uint64_t* tot = sc.alloc<uint64_t>(4);
  uint32_t* tot32 = sc.alloc<uint32_t>(4);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(cbase + H, 0, 4, s));
  LP_CHECK_HIP(hipMemsetAsync(tbase + H, 0, 4, s));
  LP_CHECK_HIP(hipMemsetAsync(pbase + H, 0, 8, s));
  hipLaunchKernelGGL(k_heavy_meta, dim3(grid_for(H, 256, 4096)), dim3(256), 0, s, hl, H, A.dsum, A.nc, parts, cbase,
                     tbase, pbase);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u32(cbase, cbase, (int64_t)H + 1, &tot32[0], sc));
  LP_CHECK(scan_exclusive_u32(tbase, tbase, (int64_t)H + 1, &tot32[1], sc));
  LP_CHECK(scan_exclusive_u64(pbase, pbase, (int64_t)H + 1, &tot[0], sc));
  uint32_t ht[2];
  uint64_t hp = 0;
  LP_CHECK_HIP(hipMemcpyAsync(ht, tot32, 8, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipMemcpyAsync(&hp, tot, 8, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  const int32_t NCH = (int32_t)ht[0], T = (int32_t)ht[1];
  int2* chunks = sc.alloc<int2>(NCH);
  int2* tasks = sc.alloc<int2>(T);
  uint64_t* tcnt = sc.alloc<uint64_t>((size_t)T + 1);
  uint64_t* tdeg = sc.alloc<uint64_t>((size_t)T + 1);
  hv.ctab = sc.alloc<uint32_t>(hp);
  hv.bnd = sc.alloc<int32_t>((size_t)T + H);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(tcnt + T, 0, 8, s));
  hipLaunchKernelGGL(k_heavy_lists, dim3(grid_for(H, 256, 4096)), dim3(256), 0, s, H, parts, cbase, tbase, chunks,
                     tasks);
  LP_CHECK_LAUNCH();
  hv.clusters = hl;
  hv.parts = parts;
  hv.cbase = cbase;
  hv.tbase = tbase;
  hv.pbase = pbase;
  hv.chunks = chunks;
  hv.tasks = tasks;
  hv.tcnt = tcnt;
  hv.tdeg = tdeg;
  hv.rec2 = rec2;
  hipLaunchKernelGGL(k_heavy_splitters, dim3(grid_for(H, 1, 1u << 20)), dim3(256), 0, s, A, hv, H);
  LP_CHECK_LAUNCH();
  if (NCH > 0) {
    hipLaunchKernelGGL(k_heavy_hist, dim3(grid_for(NCH, 1, 1u << 20)), dim3(256), 0, s, A, hv, NCH);
    LP_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_heavy_count, dim3(grid_for((int64_t)T, 4, 65536)), dim3(256), 0, s, hv, T);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_u64(tcnt, tcnt, (int64_t)T + 1, &tot[2], sc));
  int32_t* big = sc.alloc<int32_t>((size_t)T + 1);
  if (!big) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(tot32 + 2, 0, 4, s));
  hipLaunchKernelGGL(k_heavy_big, dim3(grid_for(T, 256, 4096)), dim3(256), 0, s, tcnt, T, (uint64_t)kBigTask, big,
                     tot32 + 2);
  LP_CHECK_LAUNCH();
  if (NCH > 0) {
    hipLaunchKernelGGL(k_heavy_scatter, dim3(grid_for(NCH, 1, 1u << 20)), dim3(256), 0, s, A, hv, NCH);
    LP_CHECK_LAUNCH();
  }
  uint64_t nout = 0;
  uint32_t nbig = 0;
  LP_CHECK_HIP(hipMemcpyAsync(&nout, tot + 2, 8, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipMemcpyAsync(&nbig, tot32 + 2, 4, hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  const bool debug = getenv("LPGPU_DEBUG") != nullptr;
  if (debug)
    fprintf(stderr, "[lpgpu] contract heavy: clusters %d chunks %d tasks %d records %llu\n", H, NCH, T,
            (unsigned long long)nout);
  hv.out = sc.alloc<Rec>(nout);
  if (sc.failed) return LP_ENOMEM;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  if (debug) {
    for (int i = 0; i < 3; ++i) (void)hipEventCreate(&ev[i]);
    (void)hipEventRecord(ev[0], s);
  }
  // tasks of up to kBigTask records by 256-thread workgroups; the larger
  // ones (partitions of the largest clusters, or many records of few coarse
  // neighbours) by 1024-thread workgroups with four times the table
  if (narrow) LP_CHECK((launch_reduce<kReduceThreads, kHeavyTable, uint32_t>(A, hv, nullptr, T, kBigTask, s)));
  else LP_CHECK((launch_reduce<kReduceThreads, kHeavyTable, int64_t>(A, hv, nullptr, T, kBigTask, s)));
  if (debug) (void)hipEventRecord(ev[1], s);
  if (nbig && narrow) LP_CHECK((launch_reduce<kBigThreads, kBigTable, uint32_t>(A, hv, big, (int32_t)nbig, 0, s)));
  else if (nbig) LP_CHECK((launch_reduce<kBigThreads, kBigTable, int64_t>(A, hv, big, (int32_t)nbig, 0, s)));
  if (debug) heavy_debug(hv, H, T, nbig, ev, s);
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
  const bool debug = getenv("LPGPU_DEBUG") != nullptr;
  Scratch sc(s);
  struct Ctl {
    uint32_t err;
    uint32_t nc;
    uint32_t ccount[8];
    uint32_t npieces;
    uint32_t pad;
    uint64_t two_mc;
    uint64_t nrec;
  };
  Ctl* ctl = sc.alloc<Ctl>(1);
  const int32_t* deg = nullptr;
  uint32_t* flags = sc.alloc<uint32_t>(n);
  int32_t* map = map_out ? map_out : sc.alloc<int32_t>(n);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(ctl, 0, sizeof(Ctl), s));
  lp_graph* cg = new lp_graph();
  (void)hipGetDevice(&cg->device);
  cg->stream_mem = true;
  cg->mem_stream = s;
  lp_status st = LP_OK;
  unsigned long long* mx = nullptr;
  unsigned long long mxh[2] = {0, 0};
  do {
    if (n == 0) {
      if (graph_alloc(cg, (void**)&cg->xadj, sizeof(uint64_t)) != hipSuccess) { st = LP_ENOMEM; break; }
      if (hipMemsetAsync(cg->xadj, 0, sizeof(uint64_t), s) != hipSuccess) { st = LP_EDEVICE; break; }
      break;
    }
    st = plan_degrees(g, &deg, s);
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
    unsigned long long* vw = sc.alloc<unsigned long long>(nc);
    unsigned long long* dsum = sc.alloc<unsigned long long>(nc);
    unsigned long long* cursor = sc.alloc<unsigned long long>(nc);
    uint64_t* voff = sc.alloc<uint64_t>(n);
    uint64_t* rbase = sc.alloc<uint64_t>((size_t)nc + 1);
    uint64_t* tcap = sc.alloc<uint64_t>(nc);
    uint64_t* cdeg = sc.alloc<uint64_t>((size_t)nc + 1);
    uint8_t* cls = sc.alloc<uint8_t>(nc);
    uint8_t* heavy = sc.alloc<uint8_t>(nc);
    int32_t* lists = sc.alloc<int32_t>((size_t)4 * nc);
    if (graph_alloc(cg, (void**)&cg->vwgt, (size_t)nc * sizeof(int32_t)) != hipSuccess ||
        graph_alloc(cg, (void**)&cg->xadj, ((size_t)nc + 1) * sizeof(uint64_t)) != hipSuccess) { st = LP_ENOMEM; break; }
    (void)hipMemsetAsync(vw, 0, (size_t)nc * 8, s);
    (void)hipMemsetAsync(dsum, 0, (size_t)nc * 8, s);
    (void)hipMemsetAsync(cursor, 0, (size_t)nc * 8, s);
    (void)hipMemsetAsync(cdeg, 0, ((size_t)nc + 1) * sizeof(uint64_t), s);
    (void)hipMemsetAsync(heavy, 0, (size_t)nc, s);
    hipLaunchKernelGGL(k_map, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, labels, n, flags, deg, g->vwgt, map, vw,
                       dsum);
    st = last_error();
    if (st) break;
    st = scan_exclusive_u64((const uint64_t*)dsum, rbase, nc, &ctl->nrec, sc);
    if (st) break;
    hipLaunchKernelGGL(k_reserve, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, map, deg, n, cursor, voff);
    hipLaunchKernelGGL(k_cclass, dim3(grid_for(nc, 256, 65536)), dim3(256), 0, s, dsum, vw, nc, tcap, cls, cg->vwgt,
                       &ctl->err);
    hipLaunchKernelGGL(k_class_list, dim3(grid_for(nc, 256 * 8, 65536)), dim3(256), 0, s, cls, nc, ctl->ccount, lists,
                       (int64_t)nc);
    st = last_error();
    if (st) break;
    // record pass: the edge visitor shared with rating and the cut
    Rec* rec = sc.alloc<Rec>(g->two_m);
    if (sc.failed) { st = LP_ENOMEM; break; }
    st = visit_edges_records(g, map, rbase, voff, rec, s);
    if (st) break;
    if (hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = LP_EDEVICE; break; }
    if (h.err & kErrFormat) { st = LP_EINVAL; break; }
    if (h.err) { st = LP_EOVERFLOW; break; }
    // aggregation
    AggArgs A;
    A.rbase = rbase;
    A.dsum = dsum;
    A.tcap = tcap;
    A.rec = rec;
    A.cdeg = cdeg;
    A.err = &ctl->err;
    A.nc = nc;
    const int64_t stride = nc;
    int32_t* hlist = lists + 3 * stride;
    uint32_t* nheavy = &ctl->ccount[4];
    // 32-bit table sums where no coarse edge weight can reach 2^31: unit
    // weights and fewer than 2^32 adjacency entries (a coarse edge counts
    // fine edges of one direction, at most half of them)
    const bool narrow = !g->weighted && g->two_m < (1ull << 32);
    if (narrow) {
      st = launch_light<kWave, uint32_t>(A, lists, h.ccount[1], 2 * kClassWave, hlist, nheavy, s);
      if (!st)
        st = launch_light<kLightThreads, uint32_t>(A, lists + stride, h.ccount[2], 2 * kClassBlockS, hlist, nheavy, s);
      if (!st)
        st = launch_light<kLightThreads, uint32_t>(A, lists + 2 * stride, h.ccount[3], 2 * kClassBlockL, hlist, nheavy,
                                                   s);
    } else {
      st = launch_light<kWave, int64_t>(A, lists, h.ccount[1], 2 * kClassWave, hlist, nheavy, s);
      if (!st)
        st = launch_light<kLightThreads, int64_t>(A, lists + stride, h.ccount[2], 2 * kClassBlockS, hlist, nheavy, s);
      if (!st)
        st = launch_light<kLightThreads, int64_t>(A, lists + 2 * stride, h.ccount[3], 2 * kClassBlockL, hlist, nheavy,
                                                  s);
    }
    if (st) break;
    const uint32_t heavy0 = h.ccount[4];
    if (hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = LP_EDEVICE; break; }
    if (debug)
      fprintf(stderr,
              "[lpgpu] contract n=%d nc=%d records %llu pieces %u classes wave %u blockS %u blockL %u heavy %u "
              "(+%u handed over)\n",
              n, nc, (unsigned long long)h.nrec, h.npieces, h.ccount[1], h.ccount[2], h.ccount[3], heavy0,
              h.ccount[4] - heavy0);
    Heavy hv{};
    int32_t T = 0;
    uint64_t* tscan = nullptr;
    const int32_t H = (int32_t)h.ccount[4];
    if (H > 0) {
      Rec* rec2 = sc.alloc<Rec>(g->two_m);
      if (!rec2) { st = LP_ENOMEM; break; }
      st = contract_heavy(A, hlist, H, rec2, narrow, &hv, &T, &tscan, sc);
      if (st) break;
      hipLaunchKernelGGL(k_mark_heavy, dim3(grid_for(H, 256, 4096)), dim3(256), 0, s, hlist, H, heavy);
      st = last_error();
      if (st) break;
    }
    st = scan_exclusive_u64(cdeg, cg->xadj, (int64_t)nc + 1, &ctl->two_mc, sc);
    if (st) break;
    if (hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { st = LP_EDEVICE; break; }
    if (h.err) { st = LP_EOVERFLOW; break; }
    cg->two_m = h.two_mc;
    cg->weighted = 1;
    if (graph_alloc(cg, (void**)&cg->adjncy, (h.two_mc ? h.two_mc : 1) * sizeof(int32_t)) != hipSuccess ||
        graph_alloc(cg, (void**)&cg->adjwgt, (h.two_mc ? h.two_mc : 1) * sizeof(int32_t)) != hipSuccess) { st = LP_ENOMEM; break; }
    mx = sc.alloc<unsigned long long>(2);
    unsigned long long* hsum = H > 0 ? sc.alloc<unsigned long long>(H) : nullptr;
    if (!mx || (H > 0 && !hsum)) { st = LP_ENOMEM; break; }
    if (hipMemsetAsync(mx, 0, 16, s) != hipSuccess ||
        (H > 0 && hipMemsetAsync(hsum, 0, (size_t)H * sizeof(unsigned long long), s) != hipSuccess)) {
      st = LP_EDEVICE;
      break;
    }
    hipLaunchKernelGGL(k_place_light, dim3(grid_for((int64_t)nc * kWave, 256, 65536)), dim3(256), 0, s, cg->xadj,
                       rbase, heavy, rec, nc, cg->adjncy, cg->adjwgt, mx);
    if (T > 0) {
      hipLaunchKernelGGL(k_place_heavy, dim3(grid_for((int64_t)T * kWave, 256, 65536)), dim3(256), 0, s, hv, T, tscan,
                         cg->xadj, cg->adjncy, cg->adjwgt, hsum);
      hipLaunchKernelGGL(k_heavy_max, dim3(grid_for(H, 256, 4096)), dim3(256), 0, s, hv, H, hsum, cg->xadj, mx);
    }
    st = last_error();
    if (st) break;
    if (hipMemcpyAsync(mxh, mx, 16, hipMemcpyDeviceToHost, s) != hipSuccess) { st = LP_EDEVICE; break; }
  } while (0);
  if (st == LP_OK && hipStreamSynchronize(s) != hipSuccess) st = LP_EDEVICE;
  if (st != LP_OK) {
    lp_graph_free(cg);
    return st;
  }
  // coarse metadata used by later calls: total weight, degree maxima
  cg->max_wdeg = (int64_t)mxh[0];
  cg->max_deg = (int64_t)mxh[1];
  cg->total_vwgt = g->total_vwgt;
  *coarse_out = cg;
  return LP_OK;
}
