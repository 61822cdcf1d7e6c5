// Definitions shared by host and device code of the library.
#pragma once

#include <stdint.h>

#include "lp.h"

namespace lp {

// Degree buckets used by the rating kernels (result-invariant knobs).
constexpr int kMaxLane = 16;     // lane-per-vertex register capacity
constexpr int kMaxWave = 512;    // wave-per-vertex LDS table is 2 * kMaxWave entries
constexpr int kMaxBlock = 4096;  // block-per-vertex LDS table is 2 * kMaxBlock entries

// Threads per workgroup of the block-per-vertex and hub kernels.
constexpr int kBlockThreads = 512;
constexpr int kGroupThreads = 256;  // workgroup-per-vertex rating
constexpr int kHubThreads = 256;

// Empty slot marker of LDS / global rating tables (labels are >= 0).
constexpr int32_t kEmpty = -1;

}  // namespace lp
