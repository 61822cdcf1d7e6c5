// Host-side launchers of the device-wide primitives (prims.hip) and the
// scratch-memory helper used by every entry point.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "lp_common.h"

namespace lp {

// Reports a failed HIP call on stderr when LPGPU_DEBUG is set in the
// environment, then maps it to a status code.
lp_status hip_fail(hipError_t e, const char* what, const char* file, int line);

// Clears a pending error left by earlier runtime calls of the caller, so that
// launch checks only see this library's errors.
inline void clear_error() { (void)hipGetLastError(); }

// The library's device-memory cache (one per device). A block released on
// stream s is kept and handed out again: to work on s at once (stream order
// puts the new use after the old one), to another stream once the event
// recorded at the release has completed. Steady-state calls therefore make no
// HIP allocation and never wait for the allocator. cache_alloc returns
// nullptr when the device is out of memory even after the cache was emptied.
void* cache_alloc(size_t bytes, hipStream_t s);
void cache_free(void* p, hipStream_t s);
// Frees every cached block of every device (waits for each device first).
void cache_trim_all();
// The caller's allocator for all later cache_alloc calls (nullptr: the cache).
lp_status set_allocator(const lp_allocator* a);
// Bytes of the current device handed out and kept by the cache, and bytes
// handed out by the caller's allocator (all devices).
void memory_info(uint64_t* live, uint64_t* cached, uint64_t* external);

// Stream-ordered scratch allocations from the cache, released (on the same
// stream) when the object goes out of scope. A failed allocation sets
// `failed`.
class Scratch {
 public:
  explicit Scratch(hipStream_t s) : stream_(s) {}
  ~Scratch() {
    for (void* p : ptrs_) cache_free(p, stream_);
  }
  template <typename T>
  T* alloc(size_t count) {
    const size_t bytes = (count ? count : 1) * sizeof(T);
    void* p = cache_alloc(bytes, stream_);
    if (!p) {
      (void)hip_fail(hipErrorOutOfMemory, "cache_alloc", __FILE__, __LINE__);
      failed = true;
      return nullptr;
    }
    ptrs_.push_back(p);
    return static_cast<T*>(p);
  }
  hipStream_t stream() const { return stream_; }
  bool failed = false;

 private:
  hipStream_t stream_;
  std::vector<void*> ptrs_;
};

// Exclusive prefix sum of in[0..n) into out[0..n); *total_dev (if not null)
// receives the sum of all n inputs. out may alias in.
lp_status scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total_dev,
                             Scratch& sc);
lp_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev,
                             Scratch& sc);

// Segmented inclusive prefix sum: out[i] = sum of val[j] for j in the run of
// equal seg[] values that ends at i (runs are maximal stretches of equal
// consecutive seg values). count is read from *count_dev (<= max_n).
lp_status seg_scan_incl_i64(const uint32_t* seg, const int64_t* val, int64_t* out,
                            const uint32_t* count_dev, int64_t max_n, Scratch& sc);

// Stable LSD radix sort of (key, val) pairs on key bits [0, bits). The
// number of valid pairs is *count_dev (<= max_n). Sorts in place using the
// two buffer pairs; returns the buffers that hold the result in *keys_out,
// *vals_out.
lp_status radix_sort_pairs(uint64_t* keys_a, uint32_t* vals_a, uint64_t* keys_b, uint32_t* vals_b,
                           const uint32_t* count_dev, int64_t max_n, int bits, uint64_t** keys_out,
                           uint32_t** vals_out, Scratch& sc);

#define last_error() ::lp::hip_fail(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

inline unsigned grid_for(int64_t items, int per_block, unsigned cap = 1u << 20) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (int64_t)cap) b = cap;
  return (unsigned)b;
}

#define LP_CHECK_HIP(call)                                            \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) {                                           \
      (void)hipGetLastError();                                        \
      return ::lp::hip_fail(e_, #call, __FILE__, __LINE__);           \
    }                                                                 \
  } while (0)

#define LP_CHECK(st)                  \
  do {                                \
    lp_status s_ = (st);              \
    if (s_ != LP_OK) return s_;       \
  } while (0)

#define LP_CHECK_LAUNCH() LP_CHECK(last_error())

}  // namespace lp
