// launch.hpp -- internal launchers between the C-ABI entry points and the
// kernels.  Arguments are already validated; each returns the HIP error of
// its launch(es).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace desc {
namespace launch {

// reduce.hip
constexpr int kReduceMaxBlocks = 2048;
size_t reduce_i32_workspace(int64_t n);
hipError_t reduce_i32(const int32_t* in, int64_t n, int64_t* out, void* ws, hipStream_t s);

// scan.hip
size_t scan_i32_workspace(int64_t n);
hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s);

// transpose.hip
int64_t transpose_max_rows();
hipError_t transpose_32(const uint32_t* in, uint32_t* out, int64_t batch, int64_t rows,
                        int64_t cols, hipStream_t s);

// gemm_f32.hip
hipError_t gemm_f32(const float* A, int64_t lda, const float* B, int64_t ldb, float* C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s);

// copy.hip
hipError_t copy_32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);

}  // namespace launch
}  // namespace desc
