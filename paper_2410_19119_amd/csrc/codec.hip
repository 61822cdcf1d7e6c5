// Graph handles: validation, GPU compression into the gap + VarInt format
// (Section III-A), decompression, degree extraction from the first-edge-ID
// headers, and the plain-CSR handle.
#include <string.h>

#include "decode.h"
#include "graph.h"

namespace lp {

namespace {

constexpr int kWavesPerBlock = 4;

enum : uint32_t {
  kErrRange = 1,
  kErrSelf = 2,
  kErrWeight = 4,
  kErrOrder = 8,
  kErrXadj = 16,
  kErrVwgt = 32,
};

__device__ __forceinline__ uint32_t varint_len(uint64_t x) {
  uint32_t k = 1;
  while (x >= 0x80) {
    x >>= 7;
    ++k;
  }
  return k;
}

__device__ __forceinline__ uint64_t zigzag(int64_t x) { return ((uint64_t)x << 1) ^ (uint64_t)(x >> 63); }

__device__ __forceinline__ uint32_t varint_put(uint8_t* out, uint64_t x) {
  uint32_t k = 0;
  while (x >= 0x80) {
    out[k++] = (uint8_t)((x & 0x7F) | 0x80);
    x >>= 7;
  }
  out[k++] = (uint8_t)x;
  return k;
}

struct CsrIn {
  int32_t n;
  const uint64_t* xadj;
  const int32_t* adjncy;
  const int32_t* adjwgt;
  const int32_t* vwgt;
};

// Block-wide maxima of two values, then one atomic per block (256 threads).
__device__ __forceinline__ void block_max2(unsigned long long a, unsigned long long b, unsigned long long* ga,
                                           unsigned long long* gb) {
  __shared__ unsigned long long sa[4], sb[4];
  a = wave_reduce_max(a);
  b = wave_reduce_max(b);
  if (lane_id() == 0) {
    sa[threadIdx.x / kWave] = a;
    sb[threadIdx.x / kWave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      a = max(a, sa[i]);
      b = max(b, sb[i]);
    }
    atomicMax(ga, a);
    atomicMax(gb, b);
  }
}

// The wave-per-vertex kernels below take their vertices in blocks, in order,
// from a counter (one per launch). A vertex u costs its degree plus one, so
// it starts at key(u) = xadj[u] + u (increasing in u), and block c holds the
// vertices whose key lies in [c * kCodecWork, (c + 1) * kCodecWork), i.e.
// vertices blk[c] .. blk[c + 1] - 1: at most kCodecWork vertices, and the
// adjacency of those plus the rest of the last one. The resident waves then
// read a window of the adjacency that slides over it, a run of high-degree
// vertices (a degree-ordered graph starts with one) spreads over as many
// blocks as its entries fill, and a run of isolated vertices (such a graph
// ends with one) over as many as its count fills. With a static stride,
// waves that met high-degree vertices fell behind and the reads spread over
// the whole adjacency (R-MAT scale 26 in its given order compressed 30x
// slower than the same graph numbered by degree).
constexpr uint64_t kCodecWork = 16384;
constexpr unsigned kCodecGrid = 2048;  // workgroups of 256 threads

struct CodecBlocks {
  const int64_t* blk;        // nb + 1 entries
  int64_t nb;
  unsigned long long* ctr;   // hand-out counter (zero before the launch)
};

// blk[c] = the smallest u with key(u) >= c * kCodecWork (c < nb), blk[nb] =
// n. xadj must be non-decreasing from 0 (a decrease sets *err and leaves blk
// incomplete).
__global__ void k_codec_blocks(const uint64_t* xadj, int64_t n, int64_t nb, int64_t* blk, uint32_t* err) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += (int64_t)gridDim.x * blockDim.x) {
    if (u > 0 && xadj[u] < xadj[u - 1]) {
      atomicOr(err, 1u);
      continue;
    }
    const uint64_t hi = xadj[u] + (uint64_t)u;
    // blocks c with key(u - 1) < c * kCodecWork <= key(u) (u > 0), or c = 0
    const int64_t c0 = u ? (int64_t)((xadj[u - 1] + (uint64_t)(u - 1)) / kCodecWork) + 1 : 0;
    const int64_t c1 = min((int64_t)(hi / kCodecWork), nb - 1);
    for (int64_t c = c0; c <= c1; ++c) blk[c] = u;
    if (u == n) blk[nb] = n;
  }
}

__device__ __forceinline__ int64_t next_block(const CodecBlocks& cb) {
  uint32_t c = 0;
  if (lane_id() == 0) c = (uint32_t)atomicAdd(cb.ctr, 1ull);
  return (int64_t)(uint32_t)__shfl((int)c, 0, kWave);
}

// One wave per vertex: range / self-loop / weight / order checks, weighted
// degree and degree maxima.
__global__ __launch_bounds__(256) void k_validate(CsrIn g, uint32_t* err, unsigned long long* max_wdeg,
                                                  unsigned long long* max_deg, CodecBlocks cb) {
  const int lane = lane_id();
  uint32_t bad = 0;
  unsigned long long mw = 0, md = 0;
  for (int64_t c = next_block(cb); c < cb.nb; c = next_block(cb))
  for (int64_t u = cb.blk[c]; u < cb.blk[c + 1]; ++u) {
    const uint64_t b = g.xadj[u], e = g.xadj[u + 1];
    if (e < b) {
      bad |= kErrXadj;
      continue;
    }
    int64_t wsum = 0;
    for (uint64_t k = b + lane; k < e; k += kWave) {
      const int32_t v = g.adjncy[k];
      const int32_t w = g.adjwgt ? g.adjwgt[k] : 1;
      if (v < 0 || v >= g.n) bad |= kErrRange;
      if (v == u) bad |= kErrSelf;
      if (w < 1) bad |= kErrWeight;
      if (k > b) {
        const int32_t pv = g.adjncy[k - 1];
        const int32_t pw = g.adjwgt ? g.adjwgt[k - 1] : 1;
        if (pv > v || (pv == v && pw > w)) bad |= kErrOrder;
      }
      wsum += w;
    }
    wsum = wave_reduce_add(wsum);
    mw = max(mw, (unsigned long long)wsum);
    md = max(md, (unsigned long long)(e - b));
  }
  if (bad) atomicOr(err, bad);
  block_max2(mw, md, max_wdeg, max_deg);
}

__global__ __launch_bounds__(256) void k_vwgt_check(const int32_t* vwgt, int32_t n, uint32_t* err,
                                                    unsigned long long* total) {
  __shared__ int64_t sm[4];
  int64_t s = 0;
  uint32_t bad = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = vwgt ? vwgt[u] : 1;
    if (w < 1) bad = kErrVwgt;
    s += w;
  }
  s = block_reduce_add<256, int64_t>(s, sm);
  if (threadIdx.x == 0) atomicAdd(total, (unsigned long long)s);
  if (bad) atomicOr(err, bad);
}

// Record size of each vertex (wave per vertex).
__global__ __launch_bounds__(256) void k_record_size(CsrIn g, uint64_t* size, CodecBlocks cb) {
  const int lane = lane_id();
  for (int64_t c = next_block(cb); c < cb.nb; c = next_block(cb))
  for (int64_t u = cb.blk[c]; u < cb.blk[c + 1]; ++u) {
    const uint64_t b = g.xadj[u], e = g.xadj[u + 1];
    const uint64_t d = e - b;
    const uint64_t nch = d > LP_CHUNK_THRESHOLD ? (d + LP_CHUNK_LEN - 1) / LP_CHUNK_LEN : 1;
    uint64_t len = 0;
    for (uint64_t k = b + lane; k < e; k += kWave) {
      const uint64_t i = k - b;
      const bool st = (nch > 1) ? (i % LP_CHUNK_LEN == 0) : (i == 0);
      const int32_t v = g.adjncy[k];
      const uint64_t code = st ? zigzag((int64_t)v - (int64_t)u) : (uint64_t)((int64_t)v - (int64_t)g.adjncy[k - 1]);
      len += varint_len(code);
      if (g.adjwgt) {
        const int64_t w = g.adjwgt[k];
        const int64_t pw = st ? 0 : g.adjwgt[k - 1];
        len += varint_len(zigzag(w - pw));
      }
    }
    len = wave_reduce_add(len);
    if (lane == 0) size[u] = len + varint_len(b) + (nch > 1 ? 4 * (nch - 1) : 0);
  }
}

// Writes every record at offs[u] (wave per vertex).
__global__ __launch_bounds__(256) void k_encode(CsrIn g, const uint64_t* offs, uint8_t* out, CodecBlocks cb) {
  const int lane = lane_id();
  for (int64_t c = next_block(cb); c < cb.nb; c = next_block(cb))
  for (int64_t u = cb.blk[c]; u < cb.blk[c + 1]; ++u) {
    const uint64_t b = g.xadj[u], e = g.xadj[u + 1];
    const uint64_t d = e - b;
    const uint64_t nch = d > LP_CHUNK_THRESHOLD ? (d + LP_CHUNK_LEN - 1) / LP_CHUNK_LEN : 1;
    uint8_t* rec = out + offs[u];
    const uint32_t hdr = varint_len(b);
    if (lane == 0) varint_put(rec, b);
    const uint64_t table = hdr;
    uint64_t pos = hdr + (nch > 1 ? 4 * (nch - 1) : 0);
    for (uint64_t k0 = b; k0 < e; k0 += kWave) {
      const uint64_t k = k0 + lane;
      const bool valid = k < e;
      uint64_t code = 0, wcode = 0;
      uint32_t len = 0;
      bool st = false;
      uint64_t i = k - b;
      if (valid) {
        st = (nch > 1) ? (i % LP_CHUNK_LEN == 0) : (i == 0);
        const int32_t v = g.adjncy[k];
        code = st ? zigzag((int64_t)v - (int64_t)u) : (uint64_t)((int64_t)v - (int64_t)g.adjncy[k - 1]);
        len = varint_len(code);
        if (g.adjwgt) {
          const int64_t w = g.adjwgt[k];
          const int64_t pw = st ? 0 : g.adjwgt[k - 1];
          wcode = zigzag(w - pw);
          len += varint_len(wcode);
        }
      }
      const uint64_t incl = wave_incl_scan_add((uint64_t)len);
      const uint64_t my = pos + incl - len;
      if (valid) {
        uint32_t o = varint_put(rec + my, code);
        if (g.adjwgt) varint_put(rec + my + o, wcode);
        if (st && i > 0) {
          const uint32_t rel = (uint32_t)my;
          uint8_t* t = rec + table + 4 * (i / LP_CHUNK_LEN - 1);
          t[0] = (uint8_t)rel;
          t[1] = (uint8_t)(rel >> 8);
          t[2] = (uint8_t)(rel >> 16);
          t[3] = (uint8_t)(rel >> 24);
        }
      }
      pos += __shfl(incl, kWave - 1, kWave);
    }
  }
}

// ------------------------------------------------- interval encoding ----
// Interval-coded records (Section III-A; layout in lp.h): one lane writes a
// whole record, chunk by chunk, in four passes over each chunk's sorted
// neighbours: the interval count, the (start, length - 3) pairs, the weights
// of the interval neighbours, and the remaining neighbours gap encoded.
// A run is a maximal stretch of IDs each one above the previous neighbour's,
// found left to right; runs of three or more are intervals.
__device__ __forceinline__ uint32_t put_or_len(uint8_t* out, uint64_t pos, uint64_t x) {
  return out ? varint_put(out + pos, x) : varint_len(x);
}

__device__ __forceinline__ uint64_t run_end(const int32_t* a, uint64_t i, uint64_t e) {
  uint64_t j = i + 1;
  while (j < e && (int64_t)a[j] == (int64_t)a[j - 1] + 1) ++j;
  return j;
}

// Size of u's record (out == nullptr) or the record written at out.
__device__ uint64_t itv_record(const CsrIn& g, int64_t u, uint8_t* out) {
  const uint64_t b = g.xadj[u], e = g.xadj[u + 1], d = e - b;
  const int32_t* a = g.adjncy;
  const uint64_t nch = d > LP_ITV_CHUNK_THRESHOLD ? (d + LP_CHUNK_LEN - 1) / LP_CHUNK_LEN : 1;
  uint64_t k = put_or_len(out, 0, b);
  const uint64_t table = k;
  if (nch > 1) k += 4 * (nch - 1);
  for (uint64_t ch = 0; ch < nch; ++ch) {
    const uint64_t cb = nch > 1 ? b + ch * LP_CHUNK_LEN : b;
    const uint64_t ce = nch > 1 ? min(e, cb + LP_CHUNK_LEN) : e;
    if (ch > 0 && out) {
      const uint32_t rel = (uint32_t)k;
      uint8_t* t = out + table + 4 * (ch - 1);
      t[0] = (uint8_t)rel;
      t[1] = (uint8_t)(rel >> 8);
      t[2] = (uint8_t)(rel >> 16);
      t[3] = (uint8_t)(rel >> 24);
    }
    uint64_t cnt = 0;
    for (uint64_t i = cb; i < ce;) {
      const uint64_t j = run_end(a, i, ce);
      if (j - i >= 3) {
        ++cnt;
        i = j;
      } else {
        ++i;
      }
    }
    k += put_or_len(out, k, cnt);
    for (uint64_t i = cb; i < ce;) {
      const uint64_t j = run_end(a, i, ce);
      if (j - i >= 3) {
        k += put_or_len(out, k, zigzag((int64_t)a[i] - u));
        k += put_or_len(out, k, j - i - 3);
        i = j;
      } else {
        ++i;
      }
    }
    int64_t wprev = 0;
    if (g.adjwgt)
      for (uint64_t i = cb; i < ce;) {
        const uint64_t j = run_end(a, i, ce);
        if (j - i >= 3) {
          for (uint64_t t = i; t < j; ++t) {
            k += put_or_len(out, k, zigzag((int64_t)g.adjwgt[t] - wprev));
            wprev = g.adjwgt[t];
          }
          i = j;
        } else {
          ++i;
        }
      }
    bool first = true;
    int64_t rprev = 0;
    for (uint64_t i = cb; i < ce;) {
      const uint64_t j = run_end(a, i, ce);
      if (j - i >= 3) {
        i = j;
        continue;
      }
      k += put_or_len(out, k, first ? zigzag((int64_t)a[i] - u) : (uint64_t)((int64_t)a[i] - rprev));
      if (g.adjwgt) {
        k += put_or_len(out, k, zigzag((int64_t)g.adjwgt[i] - wprev));
        wprev = g.adjwgt[i];
      }
      rprev = a[i];
      first = false;
      ++i;
    }
  }
  return k;
}

__global__ void k_record_size_itv(CsrIn g, uint64_t* size) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x)
    size[u] = itv_record(g, u, nullptr);
}

__global__ void k_encode_itv(CsrIn g, const uint64_t* offs, uint8_t* out) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x)
    (void)itv_record(g, u, out + offs[u]);
}

// Bounded VarInt read for decompression: false past `end` or beyond 64 bits.
__device__ __forceinline__ bool varint_read_to(const uint8_t* b, uint64_t end, uint64_t& pos, uint64_t& x) {
  x = 0;
  for (int shift = 0; shift < 64; shift += 7) {
    if (pos >= end) return false;
    const uint32_t c = b[pos++];
    x |= (uint64_t)(c & 0x7F) << shift;
    if (!(c & 0x80)) return true;
  }
  return false;
}

// One chunk of an interval-coded record written in (ID, weight) order: the
// interval neighbours and the other neighbours are each increasing in that
// order, so one lane merges the two on the fly. False on a malformed chunk.
__device__ bool itv_chunk_sorted(const GraphView& g, int32_t u, uint64_t pos, uint64_t end, uint32_t cnt,
                                 int32_t* ids, int32_t* wts) {
  const uint8_t* B = g.bytes;
  uint64_t kk, x;
  if (!varint_read_to(B, end, pos, kk) || kk > cnt) return false;
  const uint64_t pairs = pos;
  uint64_t L = 0;
  for (uint64_t j = 0; j < kk; ++j) {
    uint64_t len;
    if (!varint_read_to(B, end, pos, x) || !varint_read_to(B, end, pos, len)) return false;
    L += len + 3;
  }
  if (L > cnt) return false;
  // interval weights start at pos; the residuals after them
  const uint64_t wstart = pos;
  int64_t wlast = 0;
  if (g.weighted)
    for (uint64_t t = 0; t < L; ++t) {
      if (!varint_read_to(B, end, pos, x)) return false;
      wlast += unzigzag(x);
    }
  uint64_t pa = pairs, pw = wstart, pr = pos;
  // cursor A: interval neighbours; cursor B: the other neighbours
  uint64_t ja = 0, rema = 0, nb_left = cnt - L;
  int64_t va = 0, wa = 0, vb = 0, wb = wlast;
  bool has_a = false, has_b = false, first_b = true;
  auto next_a = [&]() -> bool {
    if (rema == 0) {
      if (ja == kk) {
        has_a = false;
        return true;
      }
      uint64_t zs, len;
      if (!varint_read_to(B, end, pa, zs) || !varint_read_to(B, end, pa, len)) return false;
      va = (int64_t)u + unzigzag(zs);
      rema = len + 3;
      ++ja;
    } else {
      ++va;
    }
    --rema;
    if (g.weighted) {
      uint64_t c;
      if (!varint_read_to(B, end, pw, c)) return false;
      wa += unzigzag(c);
    } else {
      wa = 1;
    }
    has_a = true;
    return va >= 0 && va < g.n;
  };
  auto next_b = [&]() -> bool {
    if (nb_left == 0) {
      has_b = false;
      return true;
    }
    uint64_t c;
    if (!varint_read_to(B, end, pr, c)) return false;
    vb = first_b ? (int64_t)u + unzigzag(c) : vb + (int64_t)c;
    first_b = false;
    if (g.weighted) {
      if (!varint_read_to(B, end, pr, c)) return false;
      wb += unzigzag(c);
    } else {
      wb = 1;
    }
    --nb_left;
    has_b = true;
    return vb >= 0 && vb < g.n;
  };
  if (!next_a() || !next_b()) return false;
  for (uint32_t i = 0; i < cnt; ++i) {
    const bool take_a = has_a && (!has_b || va < vb || (va == vb && wa <= wb));
    if (take_a) {
      ids[i] = (int32_t)va;
      if (wts) wts[i] = (int32_t)wa;
      if (!next_a()) return false;
    } else {
      if (!has_b) return false;
      ids[i] = (int32_t)vb;
      if (wts) wts[i] = (int32_t)wb;
      if (!next_b()) return false;
    }
  }
  return pr == end;
}

// Decompression of an interval-coded graph: one lane per vertex, chunk by
// chunk; the whole record must be consumed.
__global__ void k_decode_all_itv(GraphView g, const uint64_t* xadj, int32_t* adjncy, int32_t* adjwgt,
                                 uint32_t* err) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t fe = xadj[u];
    const uint32_t deg = (uint32_t)(xadj[u + 1] - fe);
    if (deg == 0) continue;
    const Nbh h = nbh_locate(g, (int32_t)u, deg);
    for (uint32_t ch = 0; ch < h.nchunks; ++ch) {
      const uint64_t p0 = nbh_chunk_pos(g, h, ch);
      const uint64_t p1 = ch + 1 < h.nchunks ? nbh_chunk_pos(g, h, ch + 1) : g.offs[u + 1];
      const uint32_t first = ch * LP_CHUNK_LEN;
      const uint32_t cnt = (h.nchunks > 1) ? min((uint32_t)LP_CHUNK_LEN, deg - first) : deg;
      if (p1 < p0 || p1 > g.offs[u + 1] ||
          !itv_chunk_sorted(g, (int32_t)u, p0, p1, cnt, adjncy + fe + first, adjwgt ? adjwgt + fe + first : nullptr)) {
        atomicOr(err, 1u);
        break;
      }
      if (adjwgt && !g.weighted)
        for (uint32_t i = 0; i < cnt; ++i) adjwgt[fe + first + i] = 1;
    }
  }
}

__global__ void k_degrees_comp(GraphView g, int32_t* deg) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x) {
    uint64_t p;
    const uint64_t a = read_header(g, (int32_t)u, p);
    const uint64_t b = (u + 1 < g.n) ? read_header(g, (int32_t)(u + 1), p) : g.two_m;
    deg[u] = (int32_t)(b - a);
  }
}

__global__ void k_degrees_plain(GraphView g, int32_t* deg) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x)
    deg[u] = (int32_t)(g.xadj[u + 1] - g.xadj[u]);
}

// Decompression: xadj from the first-edge headers, then one wave per vertex
// decodes its chunks with the cooperative decoder.
__global__ void k_xadj_from_headers(GraphView g, uint64_t* xadj) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= g.n; u += (int64_t)gridDim.x * blockDim.x) {
    uint64_t p;
    xadj[u] = (u < g.n) ? read_header(g, (int32_t)u, p) : g.two_m;
  }
}

__global__ __launch_bounds__(256) void k_decode_all(GraphView g, const uint64_t* xadj, int32_t* adjncy,
                                                    int32_t* adjwgt, uint32_t* err, CodecBlocks cb) {
  __shared__ DecodeSmem<kWave> smem[kWavesPerBlock];
  const int w = threadIdx.x / kWave;
  for (int64_t c = next_block(cb); c < cb.nb; c = next_block(cb))
  for (int64_t u = cb.blk[c]; u < cb.blk[c + 1]; ++u) {
    const uint64_t fe = xadj[u];
    const uint32_t deg = (uint32_t)(xadj[u + 1] - fe);
    if (deg == 0) continue;
    const Nbh h = nbh_locate(g, (int32_t)u, deg);
    for (uint32_t ch = 0; ch < h.nchunks; ++ch) {
      uint64_t pos = nbh_chunk_pos(g, h, ch);
      const uint32_t first = ch * LP_CHUNK_LEN;
      const uint32_t cnt = (h.nchunks > 1) ? min((uint32_t)LP_CHUNK_LEN, deg - first) : deg;
      int32_t pv = 0, pw = 0;
      const uint64_t out = fe + first;
      bool ok = group_decode<kWave>(g.bytes, pos, (int32_t)u, cnt, g.weighted, true, pv, pw, smem[w],
                                    [&](uint32_t i, int32_t v, int32_t wt) {
                                      adjncy[out + i] = v;
                                      if (adjwgt) adjwgt[out + i] = wt;
                                    });
      if (!ok) {
        if (lane_id() == 0) atomicOr(err, 1u);
        break;
      }
    }
  }
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

// The hand-out blocks of a CSR whose offsets xadj[0..n] (xadj[n] = two_m)
// are on the device, with nctr zeroed counters (one per launch that uses
// them: cb.ctr + i). LP_EINVAL if xadj decreases somewhere. Synchronises the
// scratch stream.
lp_status codec_blocks(const uint64_t* xadj, int64_t n, uint64_t two_m, int nctr, Scratch& sc, CodecBlocks* cb) {
  hipStream_t s = sc.stream();
  const int64_t nb = (int64_t)((two_m + (uint64_t)n) / kCodecWork) + 1;
  int64_t* blk = sc.alloc<int64_t>((size_t)nb + 1);
  unsigned long long* ctr = sc.alloc<unsigned long long>((size_t)nctr + 1);  // counters, then an error word
  if (!blk || !ctr) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(ctr, 0, ((size_t)nctr + 1) * sizeof(unsigned long long), s));
  uint32_t* err = (uint32_t*)(ctr + nctr);
  hipLaunchKernelGGL(k_codec_blocks, dim3(grid_for(n + 1, 256, 65536)), dim3(256), 0, s, xadj, n, nb, blk, err);
  LP_CHECK_LAUNCH();
  uint32_t h = 0;
  LP_CHECK_HIP(hipMemcpyAsync(&h, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  if (h) return LP_EINVAL;
  *cb = CodecBlocks{blk, nb, ctr};
  return LP_OK;
}

// Input checks of a CSR; also the codec hand-out blocks (counters for
// validation, record sizes and encoding).
lp_status check_csr(const CsrIn& in, hipStream_t s, uint64_t* two_m, int64_t* max_wdeg, int64_t* max_deg,
                    int64_t* total_vwgt, Scratch& sc, CodecBlocks* cb) {
  uint64_t x0 = 0, xn = 0;
  LP_CHECK_HIP(hipMemcpyAsync(&x0, in.xadj, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipMemcpyAsync(&xn, in.xadj + in.n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  if (x0 != 0) return LP_EINVAL;
  LP_CHECK(codec_blocks(in.xadj, in.n, xn, 3, sc, cb));
  struct Acc {
    uint32_t err;
    uint32_t pad;
    unsigned long long wdeg, deg, tot;
  };
  Acc* acc = sc.alloc<Acc>(1);
  if (!acc) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(acc, 0, sizeof(Acc), s));
  if (in.n > 0) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for((int64_t)in.n * kWave, 256, kCodecGrid)), dim3(256), 0, s, in,
                       &acc->err, &acc->wdeg, &acc->deg, *cb);
    LP_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_vwgt_check, dim3(grid_for(in.n, 256, 4096)), dim3(256), 0, s, in.vwgt, in.n, &acc->err,
                       &acc->tot);
    LP_CHECK_LAUNCH();
  }
  Acc h;
  LP_CHECK_HIP(hipMemcpyAsync(&h, acc, sizeof(Acc), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  if (h.err) return LP_EINVAL;
  *two_m = xn;
  *max_wdeg = (int64_t)h.wdeg;
  *max_deg = (int64_t)h.deg;
  *total_vwgt = (int64_t)h.tot;
  return LP_OK;
}

template <typename T>
lp_status dev_copy(T** dst, const T* src, size_t count, hipStream_t s, size_t pad = 0) {
  *dst = nullptr;
  size_t bytes = count * sizeof(T) + pad;
  LP_CHECK_HIP(hipMalloc((void**)dst, bytes ? bytes : 1));
  if (count) LP_CHECK_HIP(hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyDeviceToDevice, s));
  if (pad) LP_CHECK_HIP(hipMemsetAsync((uint8_t*)*dst + count * sizeof(T), 0, pad, s));
  return LP_OK;
}

}  // namespace

lp_status compute_degrees(const lp_graph* g, int32_t* deg, hipStream_t s) {
  if (g->n == 0) return LP_OK;
  if (g->deg) {
    LP_CHECK_HIP(hipMemcpyAsync(deg, g->deg, (size_t)g->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    return LP_OK;
  }
  if (g->compressed)
    hipLaunchKernelGGL(k_degrees_comp, dim3(grid_for(g->n, 256, 65536)), dim3(256), 0, s, g->view(), deg);
  else
    hipLaunchKernelGGL(k_degrees_plain, dim3(grid_for(g->n, 256, 65536)), dim3(256), 0, s, g->view(), deg);
  return last_error();
}

}  // namespace lp

using namespace lp;

static lp_status make_handle(int32_t n, const uint64_t* xadj, const int32_t* adjncy, const int32_t* adjwgt,
                             const int32_t* vwgt, void* stream, bool compress, lp_graph** out,
                             bool intervals = false) {
  if (!out || n < 0 || (n > 0 && (!xadj || !adjncy)) || (n == 0 && !xadj)) return LP_EINVAL;
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  CsrIn in{n, xadj, adjncy, adjwgt, vwgt};
  uint64_t two_m = 0;
  int64_t max_wdeg = 0, max_deg = 0, total = 0;
  CodecBlocks cb{};
  LP_CHECK(check_csr(in, s, &two_m, &max_wdeg, &max_deg, &total, sc, &cb));
  if (max_deg > 0x7FFFFFFF) return LP_EUNSUPPORTED;
  lp_graph* g = new lp_graph();
  (void)hipGetDevice(&g->device);
  g->n = n;
  g->two_m = two_m;
  g->weighted = adjwgt != nullptr;
  g->total_vwgt = total;
  g->max_wdeg = max_wdeg;
  g->max_deg = max_deg;
  lp_status st = LP_OK;
  do {
    if (vwgt) {
      st = dev_copy(&g->vwgt, vwgt, (size_t)n, s);
      if (st) break;
    }
    if (!compress) {
      st = dev_copy(&g->xadj, xadj, (size_t)n + 1, s);
      if (st) break;
      st = dev_copy(&g->adjncy, adjncy, (size_t)two_m, s);
      if (st) break;
      if (adjwgt) {
        st = dev_copy(&g->adjwgt, adjwgt, (size_t)two_m, s);
        if (st) break;
      }
      break;
    }
    g->compressed = 1;
    g->intervals = intervals ? 1 : 0;
    uint64_t* size = sc.alloc<uint64_t>((size_t)n + 1);
    uint64_t* total_dev = sc.alloc<uint64_t>(1);
    if (!size || !total_dev) {
      st = LP_ENOMEM;
      break;
    }
    if (hipMalloc((void**)&g->offs, ((size_t)n + 1) * sizeof(uint64_t)) != hipSuccess) {
      st = LP_ENOMEM;
      break;
    }
    if (n > 0) {
      if (intervals)
        hipLaunchKernelGGL(k_record_size_itv, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, in, size);
      else
        hipLaunchKernelGGL(k_record_size, dim3(grid_for((int64_t)n * kWave, 256, kCodecGrid)), dim3(256), 0, s, in,
                           size, CodecBlocks{cb.blk, cb.nb, cb.ctr + 1});
      st = last_error();
      if (st) break;
    }
    st = scan_exclusive_u64(size, g->offs, n, total_dev, sc);
    if (st) break;
    uint64_t nbytes = 0;
    if (hipMemcpyAsync(&nbytes, total_dev, sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = LP_EDEVICE;
      break;
    }
    if (hipMemcpyAsync(g->offs + n, total_dev, sizeof(uint64_t), hipMemcpyDeviceToDevice, s) != hipSuccess) {
      st = LP_EDEVICE;
      break;
    }
    g->nbytes = nbytes;
    if (hipMalloc((void**)&g->bytes, nbytes + kBytePad) != hipSuccess) {
      st = LP_ENOMEM;
      break;
    }
    if (hipMemsetAsync(g->bytes + nbytes, 0, kBytePad, s) != hipSuccess) {
      st = LP_EDEVICE;
      break;
    }
    if (n > 0) {
      if (intervals)
        hipLaunchKernelGGL(k_encode_itv, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, in, g->offs, g->bytes);
      else
        hipLaunchKernelGGL(k_encode, dim3(grid_for((int64_t)n * kWave, 256, kCodecGrid)), dim3(256), 0, s, in,
                           g->offs, g->bytes, CodecBlocks{cb.blk, cb.nb, cb.ctr + 2});
      st = last_error();
    }
  } while (0);
  if (st == LP_OK && hipStreamSynchronize(s) != hipSuccess) st = LP_EDEVICE;
  if (st != LP_OK) {
    lp_graph_free(g);
    return st;
  }
  *out = g;
  return LP_OK;
}

extern "C" lp_status lp_compress(int32_t n, const uint64_t* xadj, const int32_t* adjncy, const int32_t* adjwgt,
                                 const int32_t* vwgt, void* stream, lp_graph** out) {
  clear_error();
  return make_handle(n, xadj, adjncy, adjwgt, vwgt, stream, true, out);
}

extern "C" lp_status lp_compress_ex(int32_t n, const uint64_t* xadj, const int32_t* adjncy, const int32_t* adjwgt,
                                    const int32_t* vwgt, int32_t flags, void* stream, lp_graph** out) {
  clear_error();
  if (flags & ~LP_COMPRESS_INTERVALS) return LP_EINVAL;
  return make_handle(n, xadj, adjncy, adjwgt, vwgt, stream, true, out, (flags & LP_COMPRESS_INTERVALS) != 0);
}

extern "C" lp_status lp_graph_from_csr(int32_t n, const uint64_t* xadj, const int32_t* adjncy,
                                       const int32_t* adjwgt, const int32_t* vwgt, void* stream, lp_graph** out) {
  clear_error();
  return make_handle(n, xadj, adjncy, adjwgt, vwgt, stream, false, out);
}

extern "C" lp_status lp_graph_export(const lp_graph* g, uint64_t* offs_dev, uint8_t* bytes_dev, void* stream) {
  clear_error();
  if (!g || !g->compressed || !offs_dev || (!bytes_dev && g->nbytes)) return LP_EINVAL;
  if (g->nbatch) return LP_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  LP_CHECK_HIP(hipMemcpyAsync(offs_dev, g->offs, ((size_t)g->n + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
  if (g->nbytes) LP_CHECK_HIP(hipMemcpyAsync(bytes_dev, g->bytes, g->nbytes, hipMemcpyDeviceToDevice, s));
  return LP_OK;
}

extern "C" lp_status lp_decompress(const lp_graph* g, uint64_t* xadj, int32_t* adjncy, int32_t* adjwgt,
                                   int32_t* vwgt, void* stream) {
  clear_error();
  if (!g || !xadj || (!adjncy && g->two_m)) return LP_EINVAL;
  if (g->nbatch) return LP_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  if (vwgt) {
    if (g->vwgt) {
      if (g->n) LP_CHECK_HIP(hipMemcpyAsync(vwgt, g->vwgt, (size_t)g->n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    } else if (g->n) {
      hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(g->n, 256, 65536)), dim3(256), 0, s, vwgt, (int64_t)g->n, 1);
      LP_CHECK_LAUNCH();
    }
  }
  if (!g->compressed) {
    LP_CHECK_HIP(hipMemcpyAsync(xadj, g->xadj, ((size_t)g->n + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    if (g->two_m) {
      LP_CHECK_HIP(hipMemcpyAsync(adjncy, g->adjncy, g->two_m * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      if (adjwgt) {
        if (g->adjwgt)
          LP_CHECK_HIP(hipMemcpyAsync(adjwgt, g->adjwgt, g->two_m * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        else {
          hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)g->two_m, 256, 65536)), dim3(256), 0, s, adjwgt,
                             (int64_t)g->two_m, 1);
          LP_CHECK_LAUNCH();
        }
      }
    }
    return LP_OK;
  }
  uint32_t* err = sc.alloc<uint32_t>(1);
  if (!err) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s));
  GraphView v = g->view();
  hipLaunchKernelGGL(k_xadj_from_headers, dim3(grid_for((int64_t)g->n + 1, 256, 65536)), dim3(256), 0, s, v, xadj);
  LP_CHECK_LAUNCH();
  CodecBlocks cb{};
  if (g->n && !g->intervals) LP_CHECK(codec_blocks(xadj, g->n, g->two_m, 1, sc, &cb));
  if (g->n) {
    if (g->intervals)
      hipLaunchKernelGGL(k_decode_all_itv, dim3(grid_for(g->n, 256, 65536)), dim3(256), 0, s, v, xadj, adjncy, adjwgt,
                         err);
    else
      hipLaunchKernelGGL(k_decode_all, dim3(grid_for((int64_t)g->n * kWave, 256, kCodecGrid)), dim3(256), 0, s, v,
                         xadj, adjncy, adjwgt, err, cb);
    LP_CHECK_LAUNCH();
  }
  uint32_t h = 0;
  LP_CHECK_HIP(hipMemcpyAsync(&h, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  return h ? LP_EINVAL : LP_OK;
}

extern "C" lp_status lp_graph_info(const lp_graph* g, int32_t* n, uint64_t* two_m, uint64_t* nbytes,
                                   int32_t* is_compressed, int32_t* has_edge_weights, int64_t* total_vwgt) {
  clear_error();
  if (!g) return LP_EINVAL;
  if (n) *n = g->n;
  if (two_m) *two_m = g->two_m;
  if (nbytes) *nbytes = g->nbytes;
  if (is_compressed) *is_compressed = g->compressed ? (g->intervals ? 2 : 1) : 0;
  if (has_edge_weights) *has_edge_weights = g->weighted;
  if (total_vwgt) *total_vwgt = g->total_vwgt;
  return LP_OK;
}

extern "C" void lp_graph_free(lp_graph* g) {
  if (!g) return;
  void* bufs[] = {g->offs, g->bytes, g->xadj, g->adjncy, g->adjwgt, g->vwgt, g->gid, g->gbase, g->deg};
  if (g->stream_mem) {
    // released in the order of the stream that made the handle, to the
    // memory cache of the handle's device
    int cur = g->device;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    if (g->plan && g->plan_free) g->plan_free(g->plan);
    if (g->reord && g->reord_free) g->reord_free(g->reord);
    for (void* p : bufs) cache_free(p, g->mem_stream);
    if (cur != g->device) (void)hipSetDevice(cur);
    clear_error();
  } else {
    (void)hipDeviceSynchronize();
    if (g->plan && g->plan_free) g->plan_free(g->plan);
    if (g->reord && g->reord_free) g->reord_free(g->reord);
    for (void* p : bufs) (void)hipFree(p);
  }
  delete g;
}

extern "C" void lp_trim_memory(void) { cache_trim_all(); }

extern "C" lp_status lp_set_allocator(const lp_allocator* a) { return set_allocator(a); }

extern "C" lp_status lp_memory_info(uint64_t* live_bytes, uint64_t* cached_bytes, uint64_t* external_bytes) {
  memory_info(live_bytes, cached_bytes, external_bytes);
  return LP_OK;
}

extern "C" const char* lp_strerror(lp_status s) {
  switch (s) {
    case LP_OK: return "ok";
    case LP_EINVAL: return "invalid argument or malformed graph";
    case LP_ENOMEM: return "device out of memory";
    case LP_EOVERFLOW: return "coarse weight exceeds INT32_MAX";
    case LP_EDEVICE: return "HIP device error";
    case LP_EUNSUPPORTED: return "input outside the supported range";
    default: return "unknown status";
  }
}

extern "C" const char* lp_version(void) { return "lpgpu 0.1 gfx950"; }
