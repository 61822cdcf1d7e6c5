// Edge cut (Section I of the paper): total weight of the edges whose
// endpoints carry different labels.
#include "decode.h"
#include "graph.h"

namespace lp {

namespace {

constexpr uint32_t kErrFormat = 4;

// Edge cut, short neighbourhoods: one lane per vertex walks its neighbours
// serially; longer neighbourhoods are appended to a list for k_cut_long.
constexpr uint32_t kCutLane = 32;

__device__ __forceinline__ void block_add_u64(int64_t v, unsigned long long* acc) {
  __shared__ int64_t red[4];
  v = wave_reduce_add(v);
  if (lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t t = red[0] + red[1] + red[2] + red[3];
    if (t) atomicAdd(acc, (unsigned long long)t);
  }
}

template <bool COMP>
__global__ __launch_bounds__(256) void k_cut_short(GraphView g, const int32_t* C, const int32_t* deg,
                                                   unsigned long long* acc, int32_t* longl, uint32_t* nlong) {
  int64_t sum = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t d = (uint32_t)deg[u];
    const bool is_long = d > kCutLane;
    const uint64_t m = __ballot(is_long);
    if (m) {
      uint32_t base = 0;
      if (lane_id() == __ffsll((long long)m) - 1) base = atomicAdd(nlong, (uint32_t)__popcll(m));
      base = __shfl(base, __ffsll((long long)m) - 1, kWave);
      if (is_long) longl[base + __popcll(m & lanemask_lt())] = (int32_t)u;
    }
    if (d == 0 || is_long) continue;
    const int32_t cu = C[u];
    if constexpr (COMP) {
      lane_decode(g, (int32_t)u, d, [&](uint32_t, int32_t v, int32_t w) {
        if (C[v] != cu) sum += w;
      });
    } else {
      const uint64_t b = g.xadj[u];
      for (uint32_t k = 0; k < d; ++k)
        if (C[g.adjncy[b + k]] != cu) sum += g.adjwgt ? g.adjwgt[b + k] : 1;
    }
  }
  block_add_u64(sum, acc);
}

// Edge cut, long neighbourhoods: one wavefront per listed vertex.
template <bool COMP>
__global__ __launch_bounds__(256) void k_cut_long(GraphView g, const int32_t* C, const int32_t* deg,
                                                  const int32_t* longl, const uint32_t* nlong,
                                                  unsigned long long* acc, uint32_t* err) {
  __shared__ DecodeSmem<kWave> dsm[4];
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t cnt = *nlong;
  int64_t sum = 0;
  for (int64_t i = wid; i < cnt; i += nw) {
    const int32_t u = longl[i];
    const uint32_t d = (uint32_t)deg[u];
    const int32_t cu = C[u];
    auto body = [&](uint32_t, int32_t v, int32_t wt) {
      if (C[v] != cu) sum += wt;
    };
    if constexpr (COMP) {
      const Nbh h = nbh_locate(g, u, d);
      for (uint32_t ch = 0; ch < h.nchunks; ++ch) {
        uint64_t pos = nbh_chunk_pos(g, h, ch);
        const uint32_t first = ch * LP_CHUNK_LEN;
        const uint32_t cnt2 = (h.nchunks > 1) ? min((uint32_t)LP_CHUNK_LEN, d - first) : d;
        int32_t pv, pw;
        if (!group_decode<kWave>(g.bytes, pos, u, cnt2, g.weighted, true, pv, pw, dsm[w], body) && lane == 0)
          atomicOr(err, kErrFormat);
      }
    } else {
      const uint64_t b = g.xadj[u];
      for (uint32_t k = lane; k < d; k += kWave) body(k, g.adjncy[b + k], g.adjwgt ? g.adjwgt[b + k] : 1);
    }
  }
  block_add_u64(sum, acc);
}

}  // namespace

}  // namespace lp

using namespace lp;

extern "C" lp_status lp_edge_cut(const lp_graph* g, const int32_t* labels, int64_t* cut_out, void* stream) {
  clear_error();
  if (!g || !cut_out || (!labels && g->n > 0)) return LP_EINVAL;
  *cut_out = 0;
  if (g->n == 0) return LP_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  int32_t* deg = sc.alloc<int32_t>(g->n);
  int32_t* longl = sc.alloc<int32_t>(g->n);
  struct Acc {
    unsigned long long sum;
    uint32_t err, nlong;
  };
  Acc* acc = sc.alloc<Acc>(1);
  if (sc.failed) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(acc, 0, sizeof(Acc), s));
  LP_CHECK(compute_degrees(g, deg, s));
  const unsigned g1 = grid_for(g->n, 256, 8192);
  const unsigned g2 = 4096;
  if (g->compressed) {
    hipLaunchKernelGGL(k_cut_short<true>, dim3(g1), dim3(256), 0, s, g->view(), labels, deg, &acc->sum, longl,
                       &acc->nlong);
    hipLaunchKernelGGL(k_cut_long<true>, dim3(g2), dim3(256), 0, s, g->view(), labels, deg, longl, &acc->nlong,
                       &acc->sum, &acc->err);
  } else {
    hipLaunchKernelGGL(k_cut_short<false>, dim3(g1), dim3(256), 0, s, g->view(), labels, deg, &acc->sum, longl,
                       &acc->nlong);
    hipLaunchKernelGGL(k_cut_long<false>, dim3(g2), dim3(256), 0, s, g->view(), labels, deg, longl, &acc->nlong,
                       &acc->sum, &acc->err);
  }
  LP_CHECK_LAUNCH();
  Acc h;
  LP_CHECK_HIP(hipMemcpyAsync(&h, acc, sizeof(Acc), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  if (h.err) return LP_EINVAL;
  *cut_out = (int64_t)(h.sum / 2);
  return LP_OK;
}
