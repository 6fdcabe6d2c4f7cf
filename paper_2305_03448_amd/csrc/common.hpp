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

// Workspace header shared by the single-launch kernels that keep state
// between calls (see the workspace contract in desc.h): a generation number
// that tags every status word written in one call, a dynamic work counter
// and a count of finished blocks.  The block that finishes last resets the
// counters and advances the generation, so the next call on the same
// workspace needs no clearing pass.
struct WsHeader {
  uint32_t gen;
  uint32_t next;
  uint32_t done;
  uint32_t error;     // set non-zero when a call found the workspace inconsistent
  uint32_t pad[12];
};

// Upper bound on the polls of one look-back wait.  A wait that exceeds it can
// only come from a workspace that was not zeroed before its first use; the
// kernel then records the error and finishes instead of spinning forever.
constexpr uint32_t kSpinLimit = 1u << 20;
static_assert(sizeof(WsHeader) == 64, "header is one 64-byte line");

}  // namespace desc
