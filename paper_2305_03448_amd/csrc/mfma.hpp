// mfma.hpp -- the CDNA matrix-core fragments the GEMM kernels are built on.
//
// All three instructions used here work on a 32 x 32 output tile held by one
// wave, 16 FP32 accumulators per lane:
//
//   v_mfma_f32_32x32x2_f32      A: 1 float per lane,  B: 1 float per lane
//   v_mfma_f32_32x32x16_bf16    A: 8 bf16 per lane,   B: 8 bf16 per lane
//   v_mfma_f32_32x32x64_f8f6f4  A: 32 fp8 per lane,   B: 32 fp8 per lane
//
// Operand rows / columns: lane l supplies row (l % 32) of A and column
// (l % 32) of B.  The reduction index k that a (lane, register slot) pair
// carries is the same for A and B, so a kernel may assign k to the pairs in
// any one-to-one way, as long as it loads A and B the same way: the sum over
// k is unchanged.  Every kernel here gives lane l the k values
// [half * S, half * S + S) of the instruction's K, half = l / 32 and S the
// per-lane count.
//
// Accumulator layout (all three): register r of lane l holds
//   row = 8 * (r / 4) + 4 * (l / 32) + (r % 4),   column = l % 32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace desc {
namespace mfma {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x16 f32_32x32x2(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
// 16 x 16 x 4: lane l supplies row (A) or column (B) l % 16 at k slot l / 16;
// accumulator register r of lane l is row 4 (l / 16) + r, column l % 16.
__device__ __forceinline__ f32x4 f32_16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 bf16_32x32x16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// fp8 e4m3 (OCP) for both operands: format code 0 for A and for B.  With
// zero scale operands the compiler emits the unscaled instruction.
__device__ __forceinline__ f32x16 fp8_32x32x64(i32x8 a, i32x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// Row of the 32 x 32 tile held by accumulator register r of lane l.
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r / 4) + 4 * (lane / 32) + (r % 4); }
__device__ __forceinline__ int acc_col(int lane) { return lane % 32; }

}  // namespace mfma
}  // namespace desc
