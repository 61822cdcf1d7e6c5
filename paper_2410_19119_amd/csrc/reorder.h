// Degree-ordered copy of a graph for the rating kernels (reorder.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lp.h"

struct lp_graph;

namespace lp {

struct Reorder {
  lp_graph* g = nullptr;    // the copy: vertex i is original vertex orig[i]
  int32_t* orig = nullptr;  // n: new -> original
  int32_t* pos = nullptr;   // n: original -> new
};

// Whether a handle can have a degree-ordered copy (a single graph whose edge
// count and key width fit the build's 32-bit counts and 64-bit keys).
bool reorder_applies(const lp_graph* g);

// The handle's copy, built on first use (synchronises s then).
lp_status get_reorder(const lp_graph* g, hipStream_t s, const Reorder** out);

// The handle's copy if an earlier call built it, else nullptr.
const Reorder* existing_reorder(const lp_graph* g);

}  // namespace lp
