// Neighbourhood decoders for the gap + VarInt compressed format
// (Section III-A of the paper; layout documented in lp.h):
//  - lane_decode: one lane walks one short neighbourhood byte by byte;
//  - group_decode: a wavefront (NT = 64) or a whole workgroup (NT > 64)
//    decodes one code stream cooperatively, NT * 4 bytes per step: every
//    thread loads one dword, the group finds the VarInt terminator bytes
//    (bit 7 clear), assembles each number from the at most five bytes that
//    precede its terminator, compacts the numbers into LDS in stream order by
//    a prefix count of terminators, and turns gaps into neighbour IDs with a
//    group-wide prefix sum (gap-only format);
//  - LaneDec / lane_decode_chunk: one lane walks one chunk of either format,
//    the interval neighbours of an interval-coded chunk first.
#pragma once

#include "lp_device.h"

namespace lp {

// Where the codes of vertex u start, and how its neighbourhood is chunked.
struct Nbh {
  uint64_t rec;     // offs[u]
  uint64_t codes;   // first code of chunk 0
  uint32_t nchunks; // 1 unless deg > chunk_threshold(intervals)
};

__device__ __forceinline__ Nbh nbh_locate(const GraphView& g, int32_t u, uint32_t deg) {
  Nbh h;
  uint64_t pos;
  (void)read_header(g, u, pos);
  h.rec = g.offs[u];
  h.nchunks = deg > chunk_threshold(g.intervals) ? (deg + LP_CHUNK_LEN - 1) / LP_CHUNK_LEN : 1;
  h.codes = pos + (h.nchunks > 1 ? 4ull * (h.nchunks - 1) : 0ull);
  return h;
}

// Byte position of chunk k of a split neighbourhood (k = 0 is h.codes).
__device__ __forceinline__ uint64_t nbh_chunk_pos(const GraphView& g, const Nbh& h, uint32_t k) {
  if (k == 0) return h.codes;
  const uint8_t* t = g.bytes + (h.codes - 4ull * (h.nchunks - 1)) + 4ull * (k - 1);
  uint32_t rel = (uint32_t)t[0] | ((uint32_t)t[1] << 8) | ((uint32_t)t[2] << 16) | ((uint32_t)t[3] << 24);
  return h.rec + rel;
}

// Thread index inside the cooperating group.
template <int NT>
__device__ __forceinline__ int group_tid() {
  return NT == kWave ? lane_id() : (int)threadIdx.x;
}

template <int NT>
__device__ __forceinline__ void group_sync() {
  if constexpr (NT == kWave) wave_sync_lds();
  else __syncthreads();
}

// Group-wide inclusive sum of one int per thread; *total = group total.
// `sm` must hold NT/64 ints (unused for NT == 64).
template <int NT>
__device__ __forceinline__ int32_t group_scan(int32_t x, int32_t* sm, int32_t* total) {
  return block_incl_scan_add<NT, int32_t>(x, sm, total);
}

// LDS scratch of one decoding group.
template <int NT>
struct DecodeSmem {
  uint32_t codes[4 * NT];
  int32_t scan[NT / kWave > 0 ? NT / kWave : 1];
  uint64_t newpos;
};

// Decodes `count` neighbours whose codes start at byte `pos`. If `start` is
// true the first code is zigzag(v0 - u) (a chunk start) and the weight
// differences restart from 0; otherwise decoding continues from prev_v /
// prev_w. For every decoded neighbour i (0-based within this call) one
// thread calls f(i, v, w). All NT threads must call this function.
// On return pos points after the last consumed code, prev_v / prev_w hold
// the last neighbour and weight. Returns false on a malformed stream.
template <int NT, typename F>
__device__ bool group_decode(const uint8_t* __restrict__ bytes, uint64_t& pos, int32_t u, uint32_t count,
                             bool weighted, bool start, int32_t& prev_v, int32_t& prev_w, DecodeSmem<NT>& sm,
                             F&& f) {
  const int tid = group_tid<NT>();
  const uint32_t per = weighted ? 2u : 1u;
  if (start) {
    prev_v = 0;
    prev_w = 0;
  }
  bool first_pending = start;
  uint32_t done = 0;
  while (done < count) {
    const uint32_t need = (count - done) * per;
    const uint64_t base = pos & ~3ull;
    const int skip = (int)(pos - base);
    const uint32_t cur = *(const uint32_t*)(bytes + base + 4ull * tid);
    uint32_t prv;
    if constexpr (NT == kWave) {
      prv = __shfl_up(cur, 1, kWave);
      if (tid == 0) prv = 0;
    } else {
      prv = tid ? *(const uint32_t*)(bytes + base + 4ull * tid - 4) : 0u;
    }
    const uint64_t win = ((uint64_t)cur << 32) | prv;
    // bit i of cont / term describes byte i of win (bytes 0..3 = previous
    // thread's dword, 4..7 = this thread's); bytes before `pos` are ignored
    uint32_t cont = 0, term = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = 4 * tid - 4 + i;
      const bool valid = j >= skip;
      const uint32_t b = (uint32_t)(win >> (8 * i)) & 0xFFu;
      if (valid && (b & 0x80u)) cont |= 1u << i;
      if (i >= 4 && valid && !(b & 0x80u)) term |= 1u << i;
    }
    int32_t nterm = __popc(term);
    int32_t total;
    int32_t incl = group_scan<NT>(nterm, sm.scan, &total);
    int32_t idx = incl - nterm;
    uint32_t take = (uint32_t)total < need ? (uint32_t)total : need;
    if (weighted) take &= ~1u;
    if (take == 0) return false;  // no complete number in a full window
#pragma unroll
    for (int i = 4; i < 8; ++i) {
      if (term & (1u << i)) {
        int s = i;
        while (s > 0 && ((cont >> (s - 1)) & 1u)) --s;
        uint64_t value = 0;
        for (int k = s; k <= i; ++k) value |= ((win >> (8 * k)) & 0x7Full) << (7 * (k - s));
        if ((uint32_t)idx < take) sm.codes[idx] = (uint32_t)value;
        if ((uint32_t)idx == take - 1) sm.newpos = base + 4ull * tid + (uint64_t)(i - 4) + 1ull;
        ++idx;
      }
    }
    group_sync<NT>();
    const uint64_t npos = sm.newpos;
    const uint32_t nb = take / per;
    for (uint32_t b0 = 0; b0 < nb; b0 += NT) {
      const uint32_t i = b0 + (uint32_t)tid;
      const bool valid = i < nb;
      int32_t dv = 0, dw = 0;
      if (valid) {
        const uint32_t code = sm.codes[i * per];
        dv = (first_pending && i == 0) ? u + unzigzag32(code) : (int32_t)code;
        if (weighted) dw = unzigzag32(sm.codes[i * per + 1]);
      }
      int32_t tv, tw = 0;
      const int32_t sv = group_scan<NT>(dv, sm.scan, &tv);
      int32_t sw = 0;
      if (weighted) sw = group_scan<NT>(dw, sm.scan, &tw);
      if (valid) f(done + i, prev_v + sv, weighted ? prev_w + sw : 1);
      prev_v += tv;
      prev_w += tw;
      first_pending = false;
    }
    done += nb;
    pos = npos;
    group_sync<NT>();
  }
  return true;
}

// One lane's decoder of one chunk (a whole unsplit neighbourhood, or one
// chunk of a split one) whose codes start at byte pos: next() yields the
// chunk's neighbours one by one with their weights (1 for unit weights). In
// an interval-coded chunk it first walks the (start, length) pairs and the
// interval weights (a second cursor), then the gap-coded residuals, whose
// codes follow the interval weights.
struct LaneDec {
  const uint8_t* b;
  uint64_t pos;   // next pair, then next residual code
  uint64_t wpos;  // next interval weight
  int32_t u, x, v, w;
  uint32_t kleft, rem;
  bool weighted, itv, first_res;

  __device__ __forceinline__ void init(const GraphView& g, int32_t u_, uint64_t p) {
    b = g.bytes;
    u = u_;
    pos = p;
    weighted = g.weighted != 0;
    itv = g.intervals != 0;
    x = v = w = 0;
    rem = 0;
    kleft = 0;
    first_res = true;
    if (itv) {
      kleft = (uint32_t)varint_read(b, pos);
      wpos = pos;
      for (uint32_t j = 0; j < 2 * kleft; ++j) (void)varint_read(b, wpos);
      if (kleft == 0) pos = wpos;
    }
  }

  __device__ __forceinline__ void next(int32_t& ov, int32_t& ow) {
    if (rem > 0 || kleft > 0) {
      if (rem == 0) {
        x = u + (int32_t)unzigzag(varint_read(b, pos));
        rem = 3 + (uint32_t)varint_read(b, pos);
        --kleft;
      }
      ov = x++;
      --rem;
      if (weighted) w += (int32_t)unzigzag(varint_read(b, wpos));
      if (rem == 0 && kleft == 0) pos = wpos;  // residuals follow the interval weights
    } else {
      const uint64_t code = varint_read(b, pos);
      v = first_res ? u + (int32_t)unzigzag(code) : v + (int32_t)code;
      first_res = false;
      ov = v;
      if (weighted) w += (int32_t)unzigzag(varint_read(b, pos));
    }
    ow = weighted ? w : 1;
  }
};

// Serial decode of one chunk of cnt neighbours by one lane: f(i, v, w) for
// i = 0..cnt-1 in decoding order.
template <typename F>
__device__ __forceinline__ void lane_decode_chunk(const GraphView& g, int32_t u, uint64_t pos, uint32_t cnt, F&& f) {
  LaneDec d;
  d.init(g, u, pos);
  for (uint32_t i = 0; i < cnt; ++i) {
    int32_t v, w;
    d.next(v, w);
    f(i, v, w);
  }
}

// Serial decode of a short (unchunked) neighbourhood by one lane; calls
// f(i, v, w) for i = 0..deg-1 (the interval neighbours of an interval-coded
// record first).
template <typename F>
__device__ __forceinline__ void lane_decode(const GraphView& g, int32_t u, uint32_t deg, F&& f) {
  uint64_t pos;
  (void)read_header(g, u, pos);
  lane_decode_chunk(g, u, pos, deg, f);
}

}  // namespace lp
