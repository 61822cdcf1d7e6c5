// Edge cut of a clustering (Section I: the partitioning objective): the total
// weight of the edges whose endpoints carry different labels. Every edge is
// visited by the same lane / tile / piece decoders as the rating kernels
// (with the graph's cached plan), each counting the weights of its edges that
// leave their vertex's cluster; the sum counts every cut edge twice.
#include "graph.h"

namespace lp {
lp_status visit_edges_cut(const lp_graph* g, const int32_t* labels, unsigned long long* cut, hipStream_t s);
}

using namespace lp;

extern "C" lp_status lp_edge_cut(const lp_graph* g, const int32_t* labels, int64_t* cut_out, void* stream) {
  clear_error();
  if (!g || !cut_out || (!labels && g->n > 0)) return LP_EINVAL;
  *cut_out = 0;
  if (g->n == 0) return LP_OK;
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  unsigned long long* acc = sc.alloc<unsigned long long>(1);
  if (!acc) return LP_ENOMEM;
  LP_CHECK_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long), s));
  LP_CHECK(visit_edges_cut(g, labels, acc, s));
  unsigned long long h = 0;
  LP_CHECK_HIP(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
  LP_CHECK_HIP(hipStreamSynchronize(s));
  *cut_out = (int64_t)(h / 2);
  return LP_OK;
}
