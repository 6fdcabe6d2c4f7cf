// wave.hpp -- wave64 primitives for the steps below a block.
//
// The paper schedules grid -> blocks -> threads; on CDNA a block's threads
// run as 64-lane waves in lockstep, so the steps inside one wave need no
// barrier.  Prefix sums across the lanes of a wave use DPP row shifts
// (row_shr 1/2/4/8 inside each 16-lane row) and the row broadcasts of lane 15
// and lane 31 to carry between rows -- six instructions for 64 lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace desc {
namespace wave {

// DPP controls (GFX9 encoding).
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

// Inclusive prefix sum of a 32-bit value over the 64 lanes, wrapping mod 2^32.
__device__ __forceinline__ uint32_t inclusive_add_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr1, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr2, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr4, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr8, 0xf, 0xf, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowBcast15, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowBcast31, 0xc, 0xf, false);
  return v;
}

__device__ __forceinline__ uint32_t lane_read_u32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Sum of a 64-bit value over the 64 lanes (result valid in every lane).
__device__ __forceinline__ int64_t sum_i64(int64_t v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

// Sum of a 32-bit value over the 64 lanes, wrapping (valid in every lane).
__device__ __forceinline__ uint32_t sum_u32(uint32_t v) {
  return lane_read_u32(inclusive_add_u32(v), 63);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// A value the caller knows to be equal in every lane (read back from LDS,
// say), moved to a scalar register so that what is derived from it -- loads
// of a descriptor, addresses -- stays scalar as well.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

}  // namespace wave
}  // namespace desc
