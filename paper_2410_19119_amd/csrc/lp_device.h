// Device-side building blocks shared by the library's kernels: the graph view
// passed to kernels, the VarInt / zigzag decoders of the compressed format
// (Section III-A of the paper), the tie-break priority, wave and block
// reductions / scans, and the LDS rating table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lp_common.h"

namespace lp {

constexpr int kWave = 64;

// ------------------------------------------------------------ graph view --
// Everything a kernel needs to walk a neighbourhood. Compressed graphs use
// offs/bytes; plain graphs use xadj/adjncy/adjwgt. vwgt == nullptr means unit
// vertex weights, adjwgt == nullptr (or !weighted) unit edge weights.
struct GraphView {
  int32_t n;
  int32_t weighted;  // edge weights present
  int32_t intervals; // compressed with interval encoding
  uint64_t two_m;
  const uint64_t* offs;
  const uint8_t* bytes;
  const uint64_t* xadj;
  const int32_t* adjncy;
  const int32_t* adjwgt;
  const int32_t* vwgt;
};

// Degree above which a compressed neighbourhood is split into chunks of
// LP_CHUNK_LEN (Section III-A); interval-coded graphs split earlier.
__host__ __device__ __forceinline__ uint32_t chunk_threshold(bool intervals) {
  return intervals ? LP_ITV_CHUNK_THRESHOLD : LP_CHUNK_THRESHOLD;
}

__device__ __forceinline__ int64_t vweight(const GraphView& g, int32_t u) {
  return g.vwgt ? (int64_t)g.vwgt[u] : 1;
}

// ---------------------------------------------------------- integer mix --
// Tie-break priority of cluster c in round r: SplitMix64's output function
// (Steele, Lea, Flood 2014) on seed ^ (r << 32) ^ c. A bijection of c, so
// distinct clusters never tie; the smaller value wins.
__device__ __forceinline__ uint64_t tiebreak_key(uint64_t seed, uint32_t round, uint32_t c) {
  uint64_t z = seed ^ ((uint64_t)round << 32) ^ (uint64_t)c;
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Hash for table slots and partitions (multiplicative, Knuth).
__device__ __forceinline__ uint32_t slot_hash(uint32_t c) { return c * 0x9E3779B1u; }
__device__ __forceinline__ uint32_t part_hash(uint32_t c) {
  uint32_t x = c * 0x85EBCA6Bu;
  return x ^ (x >> 15);
}

__device__ __forceinline__ int64_t unzigzag(uint64_t z) { return (int64_t)(z >> 1) ^ -(int64_t)(z & 1); }
__device__ __forceinline__ int32_t unzigzag32(uint32_t z) { return (int32_t)(z >> 1) ^ -(int32_t)(z & 1); }

// Serial VarInt read (one lane), LEB128 order: low 7-bit group first, high bit
// of a byte = another byte follows.
__device__ __forceinline__ uint64_t varint_read(const uint8_t* __restrict__ b, uint64_t& pos) {
  uint64_t x = 0;
  int shift = 0;
  while (true) {
    uint32_t c = b[pos++];
    x |= (uint64_t)(c & 0x7F) << shift;
    if (!(c & 0x80)) break;
    shift += 7;
  }
  return x;
}

// First edge ID header of vertex u and the byte position right after it.
__device__ __forceinline__ uint64_t read_header(const GraphView& g, int32_t u, uint64_t& pos) {
  pos = g.offs[u];
  return varint_read(g.bytes, pos);
}

// One contraction record per fine edge: the coarse vertex of the neighbour
// (-1 for an edge inside the cluster) and the edge weight.
struct Rec {
  int32_t b;
  int32_t w;
};

// ------------------------------------------------------------ wave ops ----
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << lane_id()) - 1ull;  // lane 0 -> 0
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP moves of a 32-bit value between lanes (VALU, no LDS round trip); lanes
// that receive nothing (outside the row, or a row not in ROW_MASK) get 0.
// CTRL: row_shr:n = 0x110 + n within rows of 16 lanes; row_bcast:15 = 0x142
// (lane 15 of each row to the next row); row_bcast:31 = 0x143 (lane 31 to
// rows 2 and 3); wave_shr:1 = 0x138 (one lane up across the wave).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int32_t dpp_i32(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive wave64 sum of a 32-bit value: shifts by 1, 2, 4, 8 inside rows of
// 16 lanes, then each row's total passed on by the two row broadcasts.
__device__ __forceinline__ int32_t wave_incl_scan_add_i32(int32_t v) {
  v += dpp_i32<0x111>(v);
  v += dpp_i32<0x112>(v);
  v += dpp_i32<0x114>(v);
  v += dpp_i32<0x118>(v);
  v += dpp_i32<0x142, 0xa>(v);
  v += dpp_i32<0x143, 0xc>(v);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan_add(T x) {
  if constexpr (sizeof(T) == 4) {
    return (T)wave_incl_scan_add_i32((int32_t)x);
  } else {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      T y = __shfl_up(x, d, kWave);
      if (lane_id() >= d) x += y;
    }
    return x;
  }
}

template <typename T>
__device__ __forceinline__ T wave_reduce_add(T x) {
  if constexpr (sizeof(T) == 4) {
    return (T)__builtin_amdgcn_readlane(wave_incl_scan_add_i32((int32_t)x), kWave - 1);
  } else {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
  }
}

template <typename T>
__device__ __forceinline__ T wave_reduce_max(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    T y = __shfl_xor(x, d, kWave);
    x = y > x ? y : x;
  }
  return x;
}

// ------------------------------------------------------ best candidate ----
// A candidate move: rating r (higher wins), tie-break key (lower wins),
// cluster c. r < 0 means "none".
struct Cand {
  int64_t r;
  uint64_t key;
  int32_t c;
};

__device__ __forceinline__ bool cand_better(const Cand& a, const Cand& b) {
  return a.r > b.r || (a.r == b.r && a.r >= 0 && a.key < b.key);
}

__device__ __forceinline__ Cand cand_none() { return Cand{-1, ~0ull, -1}; }

__device__ __forceinline__ Cand wave_best(Cand x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    Cand y;
    y.r = __shfl_xor(x.r, d, kWave);
    y.key = __shfl_xor(x.key, d, kWave);
    y.c = __shfl_xor(x.c, d, kWave);
    if (cand_better(y, x)) x = y;
  }
  return x;
}

// Block-wide best; `sm` needs one Cand per wave. All threads get the result.
template <int NT>
__device__ __forceinline__ Cand block_best(Cand x, Cand* sm) {
  x = wave_best(x);
  if constexpr (NT == kWave) return x;
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) sm[w] = x;
  __syncthreads();
  Cand b = sm[0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i)
    if (cand_better(sm[i], b)) b = sm[i];
  return b;
}

template <int NT, typename T>
__device__ __forceinline__ T block_reduce_add(T x, T* sm) {
  x = wave_reduce_add(x);
  if constexpr (NT == kWave) return x;
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) sm[w] = x;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) s += sm[i];
  return s;
}

// Block-wide inclusive scan (sum). `sm` needs NT/64 + 1 elements. Returns the
// inclusive prefix; *total gets the block total.
template <int NT, typename T>
__device__ __forceinline__ T block_incl_scan_add(T x, T* sm, T* total) {
  T s = wave_incl_scan_add(x);
  if constexpr (NT == kWave) {
    *total = __shfl(s, kWave - 1, kWave);
    return s;
  }
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == kWave - 1) sm[w] = s;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) {
    T v = sm[i];
    if (i < w) off += v;
    tot += v;
  }
  *total = tot;
  return s + off;
}

}  // namespace lp
