// Definitions shared by host and device code of the library.
#pragma once

#include <stdint.h>

#include "lp.h"

namespace lp {

// Lane-per-vertex rating keeps up to this many neighbours in registers.
constexpr int kMaxLane = 16;

// Threads per workgroup of the hub kernels.
constexpr int kHubThreads = 256;

// Empty slot marker of LDS / global rating tables (labels are >= 0).
constexpr int32_t kEmpty = -1;

}  // namespace lp
