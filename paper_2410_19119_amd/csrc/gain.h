// Sparse gain table (Section V of the paper): the affinity of every vertex to
// every block adjacent to it, omega(u, V_b) = total weight of u's edges into
// block b, in O(m) memory. A vertex whose hash slice would not be smaller
// than k entries keeps a dense row of k affinities; every other vertex keeps
// a linear-probing hash slice of pow2(2 * deg) (block, affinity) entries,
// which can never fill with live blocks. Entries are int32 unless a weighted
// degree needs int64.
//
// Moves are applied in batches: every neighbour v of a moved vertex u loses
// omega(u, v) on u's old block and gains it on the new one (global atomics).
// Entries that drop to zero stay in place (selection skips them); a slice
// that runs out of free slots is rebuilt from the current blocks.
#pragma once

#include "graph.h"

namespace lp {

struct GainTable {
  const lp_graph* g = nullptr;
  int32_t k = 0;
  bool wide = false;          // int64 affinities
  uint64_t entries = 0;       // slots over all slices
  const int32_t* deg = nullptr;  // degrees (the handle's cached plan)
  uint64_t* off = nullptr;    // n + 1 slot offsets
  uint8_t* dense = nullptr;   // n: 1 = dense row of k affinities
  int32_t* key = nullptr;     // entries: block of a hash slot, -1 = empty
  void* val = nullptr;        // entries: affinities (int32 or int64)
  uint32_t* flag = nullptr;   // n: overflowed slice / duplicate check
  int32_t* list = nullptr;    // n: overflowed vertices
  uint32_t* cnt = nullptr;    // [0] overflowed vertices, [1] missing entries, [2] slices rebuilt so far,
                              // [3] work items
  int2* items = nullptr;      // work items of a fill (vertex, chunk) or an update (move, chunk)
  uint64_t nitems_cap = 0;
  uint64_t bytes = 0;
};

// What a selection step reads and writes: the LP round's snapshot, cap,
// tie-break seed and round, proposal outputs and the early-exit flag.
struct GtRound {
  const int32_t* C;
  const int64_t* W;
  const int32_t* vwgt;
  int64_t cap;
  uint64_t seed;
  uint32_t round;
  int32_t* ptgt;
  int64_t* pgain;
  const uint32_t* done;
};

// Allocates (library memory cache, stream-ordered on s) and fills the table
// for `blocks` (int32[n] in [0, k), checked by the caller).
lp_status gt_create(const lp_graph* g, const int32_t* blocks, int32_t k, hipStream_t s, GainTable* t);
void gt_release(GainTable* t, hipStream_t s);

// Best move of every listed vertex from its affinities (the rating of the LP
// rounds): lane_list holds vertices with short slices (one lane each),
// wave_list the others (one wavefront each).
lp_status gt_select(const GainTable& t, const GtRound& r, const int32_t* lane_list, int32_t nlane,
                    const int32_t* wave_list, int32_t nwave, hipStream_t s);

// Applies the moves {u, old block, new block, .} (u < 0: none) of the first
// *count entries; `blocks` already holds the new blocks (for rebuilds).
lp_status gt_update(const GainTable& t, const int4* moves, const uint32_t* count, int64_t max_moves,
                    const int32_t* blocks, hipStream_t s);

}  // namespace lp
