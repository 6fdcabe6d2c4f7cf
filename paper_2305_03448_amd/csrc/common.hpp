// common.hpp -- shared types of the HIP kernels and the host dispatch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
struct WsHeader {
  uint32_t gen;
  uint32_t error;     // set non-zero when a call found the workspace inconsistent
  uint32_t pad[14];
};

// Upper bound on the polls of one wait for another block.  A wait that
// exceeds it can only come from a workspace that was not zeroed before its
// first use; the kernel then records the error and finishes instead of
// spinning forever.
constexpr uint32_t kSpinLimit = 1u << 20;
static_assert(sizeof(WsHeader) == 64, "header is one 64-byte line");

}  // namespace desc
