// common.hpp -- shared types of the HIP kernels and the host dispatch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "view.hpp"

namespace desc {

// 4 x 32-bit vectors for 16-byte global accesses.  Alignment 4: the hardware
// accepts dword-aligned dwordx4 accesses, which the segmented kernels need for
// segments that start anywhere.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4u __attribute__((ext_vector_type(4))) __attribute__((aligned(4)));

constexpr int kWave = 64;

// Agent-scope relaxed atomics on 64-bit status words.  The value travels
// inside the word, so no release/acquire fence (and no L2 write-back) is
// needed to publish it across XCDs.
__device__ __forceinline__ uint64_t load_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t fetch_add_u32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A buffer resource over `bytes` bytes from `base` (raw, 32-bit elements):
// a buffer load at a byte offset >= bytes returns zero without touching
// memory.  The GEMM tiles address their stages through such ranges, with
// the offsets given by the BufferWindow view over each range.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  constexpr int kRawDword3 = 0x00020000;   // gfx9 word 3: 32-bit data format, no swizzle
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, kRawDword3);
}

// Wait until every global memory access this wave issued has completed
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their maxima).  After it a
// device-scope atomic store is visible to every agent-scope reader.
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Workspace header shared by the single-launch kernels that keep state
// between calls (see the workspace contract in desc.h): a generation number
// that tags every status word written in one call.  The block that finishes
// the call advances it, once every other block of the call has read it, so
// the next call on the same workspace needs no clearing pass.  No counter is
// shared between blocks: same-address device-scope atomics serialise in the
// memory-side atomic unit (tens of ns each), which would cap the tile rate.
//
// Stale words.  A tag repeats after a period of generations, so a word left
// behind by an earlier call could carry the current tag.  Every kernel keeps
// the state area in a form where that cannot happen: when a call ends, each
// word after the header is zero or carries that call's tag.  The kernels
// with one reader per word (the reductions' block slots) clear a word once
// they have read it; the look-back scans write every word of their region
// [0, used) and the block that advances the generation clears the words of
// the previous call's region beyond it ([used, hw), hw the previous call's
// extent, kept here).  So the next call sees only its predecessor's tag or
// zero, and consecutive generations never share a tag (next_gen skips the
// value whose tag would repeat).
struct WsHeader {
  uint32_t gen;
  uint32_t error;        // byte 4: device status word (DESC_DEV_* codes), sticky until queried
  uint64_t hw;           // words after the header that the last call left tagged
  uint32_t wait_limit;   // 0: kSpinLimit polls per wait; else at most wait_limit - 1
  uint32_t pad[11];
};

// Device status codes written into WsHeader::error (see desc.h).
constexpr uint32_t kDevWaitLimit = 1;   // a bounded wait gave up: the output is wrong
constexpr uint32_t kDevPlanes = 2;      // grouped BF16X3 planes did not fit: nothing computed

// Upper bound on the polls of one wait for another block.  A wait that
// exceeds it can only come from a workspace that was not zeroed before its
// first use, or from overlapping calls on one workspace; the kernel then
// records the error and finishes instead of spinning forever.
constexpr uint32_t kSpinLimit = 1u << 20;

// The generation after `g`.  0xFFFFFFFF is skipped: the 32-bit tags are
// 1 + g mod (2^32 - 1), under which it would repeat the tag of 0.
__device__ __forceinline__ uint32_t next_gen(uint32_t g) {
  return g >= 0xFFFFFFFEu ? 0u : g + 1u;
}

// Most polls of one wait under this workspace's limit.
__device__ __forceinline__ uint32_t max_polls(uint32_t wait_limit) {
  return wait_limit == 0 ? kSpinLimit : wait_limit - 1u;
}

// What a block of a stateful kernel reads from the header at its start.
struct CallState {
  uint32_t gen;
  uint32_t polls;   // max_polls of the workspace
};
__device__ __forceinline__ CallState read_call_state(const WsHeader* hdr) {
  return CallState{__hip_atomic_load(&hdr->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                   max_polls(__hip_atomic_load(&hdr->wait_limit, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT))};
}
__device__ __forceinline__ void set_error(WsHeader* hdr, uint32_t code) {
  __hip_atomic_store(&hdr->error, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Clears words [from, to) of a state area with one block of kThreads
// threads (to <= from clears nothing).
template <int kThreads>
__device__ __forceinline__ void clear_words(uint64_t* words, uint64_t from, uint64_t to,
                                            uint32_t thread) {
  auto w = array(words, (idx_t)to);
  for (idx_t i = (idx_t)from + thread; i < (idx_t)to; i += kThreads)
    __hip_atomic_store(&w[i], (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
static_assert(sizeof(WsHeader) == 64, "header is one 64-byte line");

}  // namespace desc
