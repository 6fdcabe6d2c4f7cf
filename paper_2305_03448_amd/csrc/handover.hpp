// handover.hpp -- a 64-bit value handed from one block to another through
// the workspace without a fence: two 64-bit words {tag:32, half:32}, each
// written and read with one relaxed agent-scope atomic.  The tag names the
// call's generation (1 + gen mod (2^32 - 1), so a zeroed workspace never
// matches), and a reader takes the value once both words carry the tag of
// its own call, so a half from an earlier call is never mixed in.
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
// (v unchanged) when the poll limit is reached, which only an inconsistent
// workspace can cause.
__device__ __forceinline__ bool poll(const uint64_t* w, uint64_t tag, uint64_t& v) {
  uint64_t lo = load_status(&w[0]), hi = load_status(&w[1]);
  for (uint32_t polls = 0; (lo & ~0xFFFFFFFFull) != tag || (hi & ~0xFFFFFFFFull) != tag;
       ++polls) {
    if (polls == kSpinLimit) return false;
    __builtin_amdgcn_s_sleep(2);
    lo = load_status(&w[0]);
    hi = load_status(&w[1]);
  }
  v = (hi << 32) | (lo & 0xFFFFFFFFull);
  return true;
}

}  // namespace handover
}  // namespace desc
