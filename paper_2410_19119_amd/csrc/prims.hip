#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

// Device-wide primitives written for wave64 / gfx950: reduce-then-scan prefix
// sums (plain and segmented) and a stable LSD radix sort of (key, value)
// pairs with 8-bit digits. The LP acceptance step and contraction use them.
#include "lp_device.h"
#include "prims.h"

namespace lp {

lp_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return LP_OK;
  static const bool debug = getenv("LPGPU_DEBUG") != nullptr;
  if (debug) fprintf(stderr, "[lpgpu] %s failed at %s:%d: %s\n", what, file, line, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? LP_ENOMEM : LP_EDEVICE;
}

// ----------------------------------------------------------- memory cache --
namespace {

struct CBlock {
  void* p;
  hipStream_t s;   // stream of the release
  hipEvent_t ev;   // recorded on s at the release
};

struct DevCache {
  std::mutex mu;
  std::multimap<size_t, CBlock> free_;    // by size
  std::unordered_map<void*, size_t> live;  // handed-out blocks
  std::vector<hipEvent_t> spare;           // events of reused blocks
  size_t cached = 0, limit = 0, live_bytes = 0;
};

constexpr int kCacheDevices = 64;

DevCache* cache_of(int* dev_out) {
  static DevCache caches[kCacheDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kCacheDevices) {
    clear_error();
    return nullptr;
  }
  if (dev_out) *dev_out = dev;
  return &caches[dev];
}

// LPGPU_CACHE_LOG set: every HIP allocation and release of the cache is
// reported on stderr.
bool cache_log() {
  static const bool on = getenv("LPGPU_CACHE_LOG") != nullptr;
  return on;
}

// Sizes are rounded up to eight classes per power of two (at least 512
// bytes), so a block serves later requests of the same class.
size_t size_class(size_t b) {
  if (b <= 512) return 512;
  const int e = 63 - __builtin_clzll((unsigned long long)(b - 1));  // 2^e < b <= 2^(e+1)
  const size_t step = (size_t)1 << (e - 3);
  return (b + step - 1) / step * step;
}

// Frees cached blocks (largest first) whose release has completed until at
// most `keep` bytes stay cached. Caller holds c.mu.
void trim_locked(DevCache& c, size_t keep) {
  for (auto it = c.free_.end(); c.cached > keep && it != c.free_.begin();) {
    --it;
    if (hipEventQuery(it->second.ev) != hipSuccess) continue;
    if (cache_log()) fprintf(stderr, "[lpgpu-cache] hipFree %zu (cached %zu)\n", it->first, c.cached);
    (void)hipFree(it->second.p);
    (void)hipEventDestroy(it->second.ev);
    c.cached -= it->first;
    it = c.free_.erase(it);
  }
  clear_error();
}

// The caller's allocator (lp_set_allocator): when set, every scratch block
// and every buffer of a handle made inside a call comes from it. Blocks keep
// the allocator that made them, so switching allocators never mixes them up.
// The caller's functions are called without any lock of the library held.
struct ExtBlock {
  size_t bytes;
  lp_allocator a;
};
std::mutex g_ext_mu;
lp_allocator g_ext{};
bool g_ext_on = false;
std::unordered_map<void*, ExtBlock> g_ext_live;
uint64_t g_ext_bytes = 0;

}  // namespace

void* cache_alloc(size_t bytes, hipStream_t s) {
  lp_allocator a{};
  bool ext = false;
  {
    std::lock_guard<std::mutex> lock(g_ext_mu);
    ext = g_ext_on;
    a = g_ext;
  }
  if (ext) {
    void* p = a.alloc(bytes ? bytes : 1, (void*)s, a.ctx);
    if (!p) return nullptr;
    std::lock_guard<std::mutex> lock(g_ext_mu);
    g_ext_live[p] = ExtBlock{bytes, a};
    g_ext_bytes += bytes;
    return p;
  }
  DevCache* c = cache_of(nullptr);
  if (!c) return nullptr;
  const size_t need = size_class(bytes);
  std::lock_guard<std::mutex> lock(c->mu);
  if (!c->limit) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = 0;
    clear_error();
    // keep up to half of the device: the working set of one call (a
    // contraction of 4e9 edges takes two record buffers of 33 GB) must stay
    // cached between calls, or every call pays for mapping it again
    c->limit = std::max<size_t>(tot / 2, (size_t)2 << 30);
  }
  for (auto it = c->free_.lower_bound(need); it != c->free_.end() && it->first <= need + need / 4; ++it) {
    CBlock& b = it->second;
    const bool done = hipEventQuery(b.ev) == hipSuccess;
    clear_error();
    if (!done && b.s != s) continue;
    // on the releasing stream the wait is implied by stream order; it is
    // enqueued anyway so that a recycled stream handle stays safe
    if (!done && hipStreamWaitEvent(s, b.ev, 0) != hipSuccess) {
      clear_error();
      continue;
    }
    void* p = b.p;
    c->spare.push_back(b.ev);
    c->cached -= it->first;
    c->live[p] = it->first;
    c->live_bytes += it->first;
    c->free_.erase(it);
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    clear_error();
    // out of memory: wait for the device, empty the cache, try once more
    if (cache_log()) fprintf(stderr, "[lpgpu-cache] out of memory for %zu bytes: emptying %zu cached\n", need, c->cached);
    (void)hipDeviceSynchronize();
    trim_locked(*c, 0);
    if (hipMalloc(&p, need) != hipSuccess) {
      clear_error();
      return nullptr;
    }
  }
  if (cache_log()) fprintf(stderr, "[lpgpu-cache] hipMalloc %zu (cached %zu)\n", need, c->cached);
  c->live[p] = need;
  c->live_bytes += need;
  return p;
}

void cache_free(void* p, hipStream_t s) {
  if (!p) return;
  {
    ExtBlock b{};
    bool ext = false;
    {
      std::lock_guard<std::mutex> lock(g_ext_mu);
      auto it = g_ext_live.find(p);
      if (it != g_ext_live.end()) {
        b = it->second;
        ext = true;
        g_ext_bytes -= b.bytes;
        g_ext_live.erase(it);
      }
    }
    if (ext) {
      b.a.free(p, (void*)s, b.a.ctx);
      return;
    }
  }
  DevCache* c = cache_of(nullptr);
  if (!c) return;
  std::lock_guard<std::mutex> lock(c->mu);
  auto lv = c->live.find(p);
  if (lv == c->live.end()) return;  // not a cache block
  const size_t size = lv->second;
  c->live.erase(lv);
  c->live_bytes -= size;
  hipEvent_t ev = nullptr;
  if (!c->spare.empty()) {
    ev = c->spare.back();
    c->spare.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    clear_error();
    (void)hipStreamSynchronize(s);  // no event: release synchronously
    (void)hipFree(p);
    clear_error();
    return;
  }
  if (hipEventRecord(ev, s) != hipSuccess) {
    clear_error();
    c->spare.push_back(ev);
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    clear_error();
    return;
  }
  c->free_.insert({size, CBlock{p, s, ev}});
  c->cached += size;
  if (c->cached > c->limit) trim_locked(*c, c->limit);
}

lp_status set_allocator(const lp_allocator* a) {
  if (a && (!a->alloc || !a->free)) return LP_EINVAL;
  std::lock_guard<std::mutex> lock(g_ext_mu);
  g_ext_on = a != nullptr;
  g_ext = a ? *a : lp_allocator{};
  return LP_OK;
}

void memory_info(uint64_t* live, uint64_t* cached, uint64_t* external) {
  DevCache* c = cache_of(nullptr);
  uint64_t l = 0, k = 0, e = 0;
  if (c) {
    std::lock_guard<std::mutex> lock(c->mu);
    l = c->live_bytes;
    k = c->cached;
  }
  {
    std::lock_guard<std::mutex> lock(g_ext_mu);
    e = g_ext_bytes;
  }
  if (live) *live = l;
  if (cached) *cached = k;
  if (external) *external = e;
}

void cache_trim_all() {
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) {
    clear_error();
    return;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
  clear_error();
  for (int d = 0; d < ndev && d < kCacheDevices; ++d) {
    if (hipSetDevice(d) != hipSuccess) {
      clear_error();
      continue;
    }
    DevCache* c = cache_of(nullptr);
    if (!c) continue;
    std::lock_guard<std::mutex> lock(c->mu);
    if (c->free_.empty()) continue;
    (void)hipDeviceSynchronize();
    trim_locked(*c, 0);
  }
  (void)hipSetDevice(cur);
  clear_error();
}

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T shfl_up_any(T x, int d) {
  static_assert(sizeof(T) % 4 == 0, "word-sized types only");
  union U {
    T t;
    uint32_t w[sizeof(T) / 4];
  } a, b;
  a.t = x;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) b.w[i] = __shfl_up(a.w[i], d, kWave);
  return b.t;
}

template <typename T>
__device__ __forceinline__ T shfl_any(T x, int src) {
  union U {
    T t;
    uint32_t w[sizeof(T) / 4];
  } a, b;
  a.t = x;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) b.w[i] = __shfl(a.w[i], src, kWave);
  return b.t;
}

// In-order (non-commutative safe) block inclusive scan of one value per thread.
template <typename T, typename Op>
__device__ __forceinline__ T block_scan_incl(T x, T* sm, T* total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = shfl_up_any(x, d);
    if (lane >= d) x = Op::op(y, x);
  }
  if (lane == kWave - 1) sm[w] = x;
  __syncthreads();
  T pre = Op::id();
  T tot = Op::id();
#pragma unroll
  for (int i = 0; i < kScanThreads / kWave; ++i) {
    if (i < w) pre = Op::op(pre, sm[i]);
    tot = Op::op(tot, sm[i]);
  }
  __syncthreads();
  *total = tot;
  return Op::op(pre, x);
}

template <typename T>
struct SumOp {
  __device__ static T id() { return T(0); }
  __device__ static T op(T a, T b) { return a + b; }
};

struct SegElem {
  int64_t v;
  uint32_t f;  // 1 = a run starts inside this element's range
  uint32_t pad;
};

struct SegOp {
  __device__ static SegElem id() { return SegElem{0, 0, 0}; }
  __device__ static SegElem op(SegElem a, SegElem b) {
    return SegElem{b.f ? b.v : a.v + b.v, a.f | b.f, 0};
  }
};

// ---- plain sums --------------------------------------------------------
template <typename T>
struct LoadArr {
  const T* in;
  __device__ T operator()(int64_t i) const { return in[i]; }
};

template <typename T, typename Op, typename Load>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Load load, int64_t n, T* aggs) {
  __shared__ T sm[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T acc = Op::id();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) acc = Op::op(acc, load(base + i));
  T tot;
  (void)block_scan_incl<T, Op>(acc, sm, &tot);
  if (threadIdx.x == 0) aggs[blockIdx.x] = tot;
}

// Exclusive sum scan of one tile with a carry-in from block_off.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_excl_down(const T* in, T* out, int64_t n,
                                                                 const T* block_off, T* total_dev) {
  __shared__ T sm[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T x[kScanItems];
  T acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    x[i] = (base + i < n) ? in[base + i] : T(0);
    acc += x[i];
  }
  T tot;
  T incl = block_scan_incl<T, SumOp<T>>(acc, sm, &tot);
  T run = incl - acc + (block_off ? block_off[blockIdx.x] : T(0));
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += x[i];
  }
  if (total_dev && block_off == nullptr && threadIdx.x == 0) *total_dev = tot;
}

template <typename T>
lp_status scan_exclusive_t(const T* in, T* out, int64_t n, T* total_dev, Scratch& sc) {
  hipStream_t s = sc.stream();
  if (n <= 0) {
    if (total_dev) LP_CHECK_HIP(hipMemsetAsync(total_dev, 0, sizeof(T), s));
    return LP_OK;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_excl_down<T>, dim3(1), dim3(kScanThreads), 0, s, in, out, n, (const T*)nullptr,
                       total_dev);
    LP_CHECK_LAUNCH();
    return LP_OK;
  }
  T* aggs = sc.alloc<T>(nb);
  if (!aggs) return LP_ENOMEM;
  hipLaunchKernelGGL((k_scan_reduce<T, SumOp<T>, LoadArr<T>>), dim3((unsigned)nb), dim3(kScanThreads), 0, s,
                     LoadArr<T>{in}, n, aggs);
  LP_CHECK_LAUNCH();
  LP_CHECK(scan_exclusive_t<T>(aggs, aggs, nb, total_dev, sc));
  hipLaunchKernelGGL(k_scan_excl_down<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                     (const T*)aggs, (T*)nullptr);
  LP_CHECK_LAUNCH();
  return LP_OK;
}

// ---- segmented sums ----------------------------------------------------
struct LoadSeg {
  const uint32_t* seg;
  const int64_t* val;
  __device__ SegElem operator()(int64_t i) const {
    uint32_t f = (i == 0) || (seg[i] != seg[i - 1]);
    return SegElem{val[i], f, 0};
  }
};

struct LoadAggs {
  const SegElem* a;
  __device__ SegElem operator()(int64_t i) const { return a[i]; }
};

// Inclusive segmented scan of one tile, carry-in = exclusive prefix of the
// block aggregates (carry[b]).
template <typename Load>
__global__ __launch_bounds__(kScanThreads) void k_seg_down(Load load, int64_t n, const SegElem* carry,
                                                           SegElem* out_elems, int64_t* out_vals) {
  __shared__ SegElem sm[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  SegElem x[kScanItems];
  SegElem acc = SegOp::id();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    x[i] = (base + i < n) ? load(base + i) : SegOp::id();
    acc = SegOp::op(acc, x[i]);
  }
  SegElem tot;
  SegElem incl = block_scan_incl<SegElem, SegOp>(acc, sm, &tot);
  // exclusive prefix of this thread = everything before it in the block,
  // preceded by the block's carry-in
  SegElem pre = shfl_up_any(incl, 1);
  {
    // lane 0 of each wave takes the previous wave's total
    __shared__ SegElem wl[kScanThreads / kWave];
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wl[w] = incl;
    __syncthreads();
    if (lane_id() == 0) pre = (w == 0) ? SegOp::id() : wl[w - 1];
  }
  SegElem run = SegOp::op(carry ? carry[blockIdx.x] : SegOp::id(), pre);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    run = SegOp::op(run, x[i]);
    if (base + i < n) {
      if (out_vals) out_vals[base + i] = run.v;
      if (out_elems) out_elems[base + i] = run;
    }
  }
}

// Exclusive segmented scan of an array of aggregates, in place (recursive).
lp_status seg_scan_aggs_excl(SegElem* a, int64_t n, Scratch& sc) {
  hipStream_t s = sc.stream();
  // inclusive into tmp, then shift by one
  SegElem* incl = sc.alloc<SegElem>(n);
  if (!incl) return LP_ENOMEM;
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  SegElem* carry = nullptr;
  if (nb > 1) {
    carry = sc.alloc<SegElem>(nb);
    if (!carry) return LP_ENOMEM;
    hipLaunchKernelGGL((k_scan_reduce<SegElem, SegOp, LoadAggs>), dim3((unsigned)nb), dim3(kScanThreads), 0, s,
                       LoadAggs{a}, n, carry);
    LP_CHECK_LAUNCH();
    LP_CHECK(seg_scan_aggs_excl(carry, nb, sc));
  }
  hipLaunchKernelGGL(k_seg_down<LoadAggs>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, LoadAggs{a}, n,
                     (const SegElem*)carry, incl, (int64_t*)nullptr);
  LP_CHECK_LAUNCH();
  // a[i] = incl[i-1], a[0] = identity
  LP_CHECK_HIP(hipMemcpyAsync(a + 1, incl, (size_t)(n - 1) * sizeof(SegElem), hipMemcpyDeviceToDevice, s));
  LP_CHECK_HIP(hipMemsetAsync(a, 0, sizeof(SegElem), s));
  return LP_OK;
}

__global__ void k_read_count(const uint32_t* count_dev, int64_t* n_out) { *n_out = *count_dev; }

template <typename Load>
__global__ __launch_bounds__(kScanThreads) void k_seg_reduce_dyn(Load load, const uint32_t* count_dev,
                                                                 SegElem* aggs) {
  __shared__ SegElem sm[kScanThreads / kWave];
  const int64_t n = *count_dev;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  SegElem acc = SegOp::id();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) acc = SegOp::op(acc, load(base + i));
  SegElem tot;
  (void)block_scan_incl<SegElem, SegOp>(acc, sm, &tot);
  if (threadIdx.x == 0) aggs[blockIdx.x] = tot;
}

template <typename Load>
__global__ __launch_bounds__(kScanThreads) void k_seg_down_dyn(Load load, const uint32_t* count_dev,
                                                               const SegElem* carry, int64_t* out_vals) {
  const int64_t n = *count_dev;
  if ((int64_t)blockIdx.x * kScanTile >= n) return;
  // identical to k_seg_down with a device-side count
  __shared__ SegElem sm[kScanThreads / kWave];
  __shared__ SegElem wl[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  SegElem x[kScanItems];
  SegElem acc = SegOp::id();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    x[i] = (base + i < n) ? load(base + i) : SegOp::id();
    acc = SegOp::op(acc, x[i]);
  }
  SegElem tot;
  SegElem incl = block_scan_incl<SegElem, SegOp>(acc, sm, &tot);
  SegElem pre = shfl_up_any(incl, 1);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) wl[w] = incl;
  __syncthreads();
  if (lane_id() == 0) pre = (w == 0) ? SegOp::id() : wl[w - 1];
  SegElem run = SegOp::op(carry ? carry[blockIdx.x] : SegOp::id(), pre);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    run = SegOp::op(run, x[i]);
    if (base + i < n) out_vals[base + i] = run.v;
  }
}

// ---- radix sort ----------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRsBins = 256;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t* __restrict__ keys,
                                                        const uint32_t* count_dev, int shift,
                                                        uint32_t* __restrict__ hist, uint32_t nblocks) {
  __shared__ uint32_t h[kRsBins];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t n = *count_dev;
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int i = 0; i < kRsItems; ++i) {
    int64_t j = base + (int64_t)i * kRsThreads + t;
    if (j < n) atomicAdd(&h[(uint32_t)(keys[j] >> shift) & (kRsBins - 1)], 1u);
  }
  __syncthreads();
  hist[(size_t)t * nblocks + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout,
                                                           const uint32_t* count_dev, int shift,
                                                           const uint32_t* __restrict__ offs,
                                                           uint32_t nblocks) {
  constexpr int kW = kRsThreads / kWave;
  __shared__ uint32_t running[kRsBins];
  __shared__ uint32_t wcnt[kW][kRsBins];
  const int t = threadIdx.x;
  const int w = t / kWave;
  const int64_t n = *count_dev;
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  if (base >= n) return;
  running[t] = offs[(size_t)t * nblocks + blockIdx.x];
  const uint64_t lt = lanemask_lt();
  for (int i = 0; i < kRsItems; ++i) {
    const int64_t j = base + (int64_t)i * kRsThreads + t;
    const bool valid = j < n;
    uint64_t key = valid ? kin[j] : 0;
    uint32_t val = valid ? vin[j] : 0;
    uint32_t d = (uint32_t)(key >> shift) & (kRsBins - 1);
#pragma unroll
    for (int k = 0; k < kW; ++k) wcnt[k][t] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    uint32_t rank = __popcll(peers & lt);
    uint32_t cnt = __popcll(peers);
    if (valid && rank == cnt - 1) wcnt[w][d] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t off = running[d] + rank;
#pragma unroll
      for (int k = 0; k < kW; ++k)
        if (k < w) off += wcnt[k][d];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) add += wcnt[k][t];
    running[t] += add;
    __syncthreads();
  }
}

}  // namespace

lp_status scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total_dev, Scratch& sc) {
  return scan_exclusive_t<uint64_t>(in, out, n, total_dev, sc);
}

lp_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, Scratch& sc) {
  return scan_exclusive_t<uint32_t>(in, out, n, total_dev, sc);
}

lp_status seg_scan_incl_i64(const uint32_t* seg, const int64_t* val, int64_t* out, const uint32_t* count_dev,
                            int64_t max_n, Scratch& sc) {
  if (max_n <= 0) return LP_OK;
  hipStream_t s = sc.stream();
  int64_t nb = (max_n + kScanTile - 1) / kScanTile;
  SegElem* carry = nullptr;
  if (nb > 1) {
    carry = sc.alloc<SegElem>(nb);
    if (!carry) return LP_ENOMEM;
    hipLaunchKernelGGL(k_seg_reduce_dyn<LoadSeg>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, LoadSeg{seg, val},
                       count_dev, carry);
    LP_CHECK_LAUNCH();
    LP_CHECK(seg_scan_aggs_excl(carry, nb, sc));
  }
  hipLaunchKernelGGL(k_seg_down_dyn<LoadSeg>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, LoadSeg{seg, val},
                     count_dev, (const SegElem*)carry, out);
  LP_CHECK_LAUNCH();
  return LP_OK;
}

lp_status radix_sort_pairs(uint64_t* keys_a, uint32_t* vals_a, uint64_t* keys_b, uint32_t* vals_b,
                           const uint32_t* count_dev, int64_t max_n, int bits, uint64_t** keys_out,
                           uint32_t** vals_out, Scratch& sc) {
  hipStream_t s = sc.stream();
  *keys_out = keys_a;
  *vals_out = vals_a;
  if (max_n <= 0 || bits <= 0) return LP_OK;
  if (max_n > 0xFFFFFFFFll) return LP_EUNSUPPORTED;
  const uint32_t nb = (uint32_t)((max_n + kRsTile - 1) / kRsTile);
  uint32_t* hist = sc.alloc<uint32_t>((size_t)kRsBins * nb);
  if (!hist) return LP_ENOMEM;
  uint64_t *kin = keys_a, *kout = keys_b;
  uint32_t *vin = vals_a, *vout = vals_b;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kRsThreads), 0, s, kin, count_dev, shift, hist, nb);
    LP_CHECK_LAUNCH();
    LP_CHECK(scan_exclusive_u32(hist, hist, (int64_t)kRsBins * nb, nullptr, sc));
    hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kRsThreads), 0, s, kin, vin, kout, vout, count_dev, shift,
                       hist, nb);
    LP_CHECK_LAUNCH();
    uint64_t* tk = kin;
    kin = kout;
    kout = tk;
    uint32_t* tv = vin;
    vin = vout;
    vout = tv;
  }
  *keys_out = kin;
  *vals_out = vin;
  return LP_OK;
}

}  // namespace lp
