// handover.hpp -- a 64-bit value handed from one block to another through
// the workspace without a fence: two 64-bit words {tag:32, half:32}, each
// written and read with one relaxed agent-scope atomic.  The tag names the
// call's generation (1 + gen mod (2^32 - 1), so a zeroed workspace never
// matches; generations advance with next_gen, so consecutive calls never
// share a tag), and a reader takes the value once both words carry the tag
// of its own call, so a half from an earlier call is never mixed in.
#pragma once
#include "common.hpp"

namespace desc {
namespace handover {

__device__ __forceinline__ uint64_t tag_of(uint32_t gen) {
  return (uint64_t)(1u + gen % 0xFFFFFFFFu) << 32;
}

__device__ __forceinline__ void publish(uint64_t* w, uint64_t tag, uint64_t v) {
  store_status(&w[0], tag | (v & 0xFFFFFFFFull));
  store_status(&w[1], tag | (v >> 32));
}

// Waits until both words carry `tag` and returns the value in `v`; false
// (v unchanged) when `max_polls` polls found it not ready (none with
// max_polls = 0), which only an inconsistent workspace or a debug wait limit
// can cause.
__device__ __forceinline__ bool poll(const uint64_t* w, uint64_t tag, uint64_t& v,
                                     uint32_t max_polls) {
  for (uint32_t polls = 0;; ++polls) {
    if (polls == max_polls) return false;
    const uint64_t lo = load_status(&w[0]), hi = load_status(&w[1]);
    if ((lo & ~0xFFFFFFFFull) == tag && (hi & ~0xFFFFFFFFull) == tag) {
      v = (hi << 32) | (lo & 0xFFFFFFFFull);
      return true;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Zeroes both words: for a word with one reader, once that reader has it.
__device__ __forceinline__ void clear(uint64_t* w) {
  store_status(&w[0], 0);
  store_status(&w[1], 0);
}

}  // namespace handover
}  // namespace desc
