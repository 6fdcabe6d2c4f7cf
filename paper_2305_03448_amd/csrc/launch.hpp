// launch.hpp -- internal launchers between the C-ABI entry points and the
// kernels.  Arguments are already validated; each returns the HIP error of
// its launch(es).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/desc.h"

namespace desc {
namespace launch {

// Blocks of `kernel` (of `threads` threads) that fit the device at once: its
// occupancy per CU times the CUs, per device, computed on first use
// (`fallback_per_cu` if the occupancy query fails).
template <class K>
int resident_grid(K kernel, int (&cache)[64], int fallback_per_cu, int threads) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cache[dev] == 0) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess ||
        per < 1)
      per = fallback_per_cu;
    cache[dev] = cus * per;
  }
  return cache[dev];
}

// reduce.hip
constexpr int kReduceMaxBlocks = 2048;
size_t reduce_i32_workspace(int64_t n);
hipError_t reduce_i32(const int32_t* in, int64_t n, int64_t* out, void* ws, hipStream_t s);

// reduce_ops.hip
int64_t reduce_op_grid(int64_t n);
size_t reduce_op_workspace(int64_t n);
hipError_t minmax_i32(const int32_t* in, int64_t n, int32_t* out, void* ws, hipStream_t s);
hipError_t sum_f32(const float* in, int64_t n, double* out, void* ws, hipStream_t s);

// scan.hip
size_t scan_i32_workspace(int64_t n);
hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s,
                    bool exclusive = false);

// scan_f32.hip
size_t scan_f32_workspace(int64_t n);
hipError_t scan_f32(const float* in, float* out, int64_t n, void* ws, hipStream_t s);

// transpose.hip
int64_t transpose_max_rows();
hipError_t transpose_32(const uint32_t* in, uint32_t* out, int64_t batch, int64_t rows,
                        int64_t cols, hipStream_t s);
int64_t transpose_elem_max_rows(int64_t elem_bytes);
hipError_t transpose_elem(const void* in, void* out, int64_t elem_bytes, int64_t batch,
                          int64_t rows, int64_t cols, hipStream_t s);

// gemm_f32.hip
hipError_t gemm_f32(const float* A, int64_t lda, const float* B, int64_t ldb, float* C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s);

// gemm_lowp.hip
size_t gemm_lowp_workspace(int mode, int64_t M, int64_t N, int64_t K);
hipError_t gemm_bf16x3(const float* A, int64_t lda, const float* B, int64_t ldb, float* C,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws, hipStream_t s);
hipError_t gemm_fp8(const float* A, int64_t lda, const float* B, int64_t ldb, float* C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws, hipStream_t s);
hipError_t split_bf16_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint16_t* hi,
                           uint16_t* lo, int64_t ldh, hipStream_t s);
hipError_t split_bf16_cols(const float* B, int64_t K, int64_t N, int64_t ldb, uint16_t* hi_t,
                           uint16_t* lo_t, int64_t ldh, hipStream_t s);
hipError_t quant_e4m3_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint8_t* q,
                           int64_t ldq, float* scale, hipStream_t s);
size_t quant_e4m3_cols_workspace(int64_t K, int64_t N);
hipError_t quant_e4m3_cols(const float* B, int64_t K, int64_t N, int64_t ldb, uint8_t* qt,
                           int64_t ldq, float* scale, void* ws, hipStream_t s);

// segmented.hip
size_t segmented_workspace(int64_t n, int64_t S, bool scan);
int64_t segmented_max_grid(int64_t n, int64_t S);
// persistent: allow the reduce's one-launch form (up to 8192 segments); the
// batched form passes false, since its offsets share the workspace.
hipError_t reduce_segmented_i32(const int32_t* in, int64_t n, const int64_t* offsets, int64_t S,
                                int64_t* out, void* ws, hipStream_t s, bool persistent = true);
hipError_t scan_segmented_i32(const int32_t* in, int32_t* out, int64_t n, const int64_t* offsets,
                              int64_t S, void* ws, hipStream_t s);

// grouped.hip
size_t gemm_grouped_workspace(int64_t G);
size_t gemm_grouped_bf16x3_head(int64_t G);
// head + the planes of the problems the current configuration stages
// through planes; SIZE_MAX for a refused shape
size_t gemm_grouped_bf16x3_workspace(const desc_gemm_problem* host, int64_t G);
hipError_t gemm_grouped_bf16x3(const desc_gemm_problem* problems, int64_t G, void* ws,
                               size_t ws_bytes, hipStream_t s);
hipError_t gemm_grouped_f32(const desc_gemm_problem* problems, int64_t G, void* ws,
                            hipStream_t s);

// batched.hip
size_t batched_offsets_bytes(int64_t B);
size_t batched_workspace(int64_t B, int64_t L, bool scan);   // segmented ws, then the offsets
size_t strided_problems_bytes(int64_t G);
hipError_t reduce_batched_i32(const int32_t* in, int64_t B, int64_t L, int64_t* out, void* ws,
                              hipStream_t s);
hipError_t scan_batched_i32(const int32_t* in, int32_t* out, int64_t B, int64_t L, void* ws,
                            hipStream_t s);
hipError_t gemm_strided_batched(int mode, int64_t G, int64_t M, int64_t N, int64_t K,
                                const float* A, int64_t lda, int64_t sa, const float* Bm,
                                int64_t ldb, int64_t sb, float* C, int64_t ldc, int64_t sc,
                                void* ws, size_t ws_bytes, hipStream_t s);
// grouped.hip: the BF16X3 workspace for G problems of one shape
size_t gemm_grouped_bf16x3_workspace_uniform(const desc_gemm_problem& p, int64_t G);

// copy.hip
hipError_t copy_32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);
hipError_t reverse_32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s);

// noalloc.hip
int64_t scan_noalloc_max_n();
hipError_t noalloc_scratch(hipStream_t s, void** out, size_t* bytes);

// status.hip
hipError_t workspace_status(void* ws, int32_t* out, hipStream_t s);
hipError_t workspace_set_wait_limit(void* ws, uint32_t encoded, hipStream_t s);

// variants.hip
hipError_t reduce_blocks_i32(const int32_t* in, int64_t n, int64_t E, int64_t* out,
                             hipStream_t s);
size_t scan_two_pass_workspace(int64_t n);
hipError_t scan_two_pass_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                             hipStream_t s);

}  // namespace launch
}  // namespace desc
