// api.hip -- the C-ABI entry points: argument checks, then the launchers.
//
// Checks run in a fixed order (null -> size -> host pointer -> alias ->
// workspace) and return before anything is launched.  Nothing here reads
// device memory, allocates or synchronises, so every entry point may be
// captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <atomic>

#include "../../include/desc.h"
#include "launch.hpp"
#include "tuning.hpp"

#include <stdio.h>
#include <string.h>

namespace {

thread_local int g_last_hip_error = 0;
std::atomic<desc_pointer_classifier> g_classifier{nullptr};

// 0 = GPU memory, 1 = host memory, -1 = unknown to HIP.
int classify(const void* p) {
  if (desc_pointer_classifier fn = g_classifier.load(std::memory_order_acquire)) return fn(p);
  hipPointerAttribute_t attr;
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();   // an unknown pointer leaves an error behind
    return -1;
  }
  switch (attr.type) {
    case hipMemoryTypeDevice:
    case hipMemoryTypeManaged:
      return 0;
    case hipMemoryTypeHost:
      return 1;
    default:
      return -1;
  }
}

desc_status hip_status(hipError_t e) {
  if (e == hipSuccess) return DESC_OK;
  g_last_hip_error = (int)e;
  return DESC_ERR_HIP;
}

bool mul_overflows(int64_t a, int64_t b) {
  if (a == 0 || b == 0) return false;
  return a > INT64_MAX / b;
}

// Byte extent of `count` elements of `size` bytes, or -1 on overflow.
int64_t bytes_of(int64_t count, int64_t size) {
  if (count < 0 || mul_overflows(count, size)) return -1;
  return count * size;
}

struct Range {
  const void* p;
  int64_t bytes;
};

bool overlap(Range a, Range b) {
  if (a.bytes <= 0 || b.bytes <= 0) return false;
  const uintptr_t a0 = (uintptr_t)a.p, b0 = (uintptr_t)b.p;
  return a0 < b0 + (uintptr_t)b.bytes && b0 < a0 + (uintptr_t)a.bytes;
}

desc_status check_device(std::initializer_list<const void*> ptrs) {
  for (const void* p : ptrs)
    if (p != nullptr && classify(p) != 0) return DESC_ERR_HOST_POINTER;
  return DESC_OK;
}

bool misaligned(const void* p, size_t a) { return ((uintptr_t)p % a) != 0; }

#define DESC_TRY(expr)                  \
  do {                                  \
    const desc_status _s = (expr);      \
    if (_s != DESC_OK) return _s;       \
  } while (0)

}  // namespace

extern "C" {

const char* desc_status_string(desc_status s) {
  switch (s) {
    case DESC_OK: return "DESC_OK";
    case DESC_ERR_NULL: return "DESC_ERR_NULL: a required pointer is NULL";
    case DESC_ERR_SIZE: return "DESC_ERR_SIZE: negative size or byte count overflow";
    case DESC_ERR_HOST_POINTER: return "DESC_ERR_HOST_POINTER: pointer is not GPU memory";
    case DESC_ERR_ALIAS: return "DESC_ERR_ALIAS: an output overlaps an input";
    case DESC_ERR_WORKSPACE: return "DESC_ERR_WORKSPACE: workspace too small";
    case DESC_ERR_UNSUPPORTED: return "DESC_ERR_UNSUPPORTED: mode or shape not provided";
    case DESC_ERR_HIP: return "DESC_ERR_HIP: a HIP call failed";
    case DESC_ERR_ALIGNMENT: return "DESC_ERR_ALIGNMENT: pointer not aligned to its element";
    case DESC_ERR_LIMIT:
      return "DESC_ERR_LIMIT: size above the fixed scratch of an allocation-free entry point";
  }
  return "unknown desc_status";
}

int desc_last_hip_error(void) { return g_last_hip_error; }

int desc_version(void) { return 100; }

void desc_set_pointer_classifier(desc_pointer_classifier fn) {
  g_classifier.store(fn, std::memory_order_release);
}

// ----------------------------------------------------------------- device status
desc_status desc_workspace_status(void* ws, size_t ws_bytes, int32_t* status, void* stream) {
  if (ws == nullptr || status == nullptr) return DESC_ERR_NULL;
  DESC_TRY(check_device({ws, status}));
  if (misaligned(ws, 8) || misaligned(status, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({status, 4}, {ws, (int64_t)ws_bytes})) return DESC_ERR_ALIAS;
  if (ws_bytes < 64) return DESC_ERR_WORKSPACE;
  return hip_status(desc::launch::workspace_status(ws, status, (hipStream_t)stream));
}

desc_status desc_workspace_set_wait_limit(void* ws, size_t ws_bytes, int64_t max_polls,
                                          void* stream) {
  if (ws == nullptr) return DESC_ERR_NULL;
  if (max_polls > (int64_t)0xFFFFFFFEu) return DESC_ERR_SIZE;
  DESC_TRY(check_device({ws}));
  if (misaligned(ws, 8)) return DESC_ERR_ALIGNMENT;
  if (ws_bytes < 64) return DESC_ERR_WORKSPACE;
  const uint32_t encoded = max_polls < 0 ? 0u : (uint32_t)max_polls + 1u;
  return hip_status(desc::launch::workspace_set_wait_limit(ws, encoded, (hipStream_t)stream));
}

// ----------------------------------------------------------------- reduce
size_t desc_reduce_i32_workspace(int64_t n) { return desc::launch::reduce_i32_workspace(n); }

desc_status desc_reduce_i32(const int32_t* in, int64_t n, int64_t* out, void* ws,
                            size_t ws_bytes, void* stream) {
  if (out == nullptr || ws == nullptr || (in == nullptr && n > 0)) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  DESC_TRY(check_device({n > 0 ? (const void*)in : nullptr, out, ws}));
  if (misaligned(in, 4) || misaligned(out, 8) || misaligned(ws, 8)) return DESC_ERR_ALIGNMENT;
  const int64_t wsb = (int64_t)desc_reduce_i32_workspace(n);
  if (overlap({out, 8}, {in, nb}) || overlap({ws, (int64_t)ws_bytes}, {in, nb}) ||
      overlap({ws, (int64_t)ws_bytes}, {out, 8}))
    return DESC_ERR_ALIAS;
  if ((int64_t)ws_bytes < wsb) return DESC_ERR_WORKSPACE;
  return hip_status(desc::launch::reduce_i32(in, n, out, ws, (hipStream_t)stream));
}

// ----------------------------------------------------------------- min/max, float sum
size_t desc_reduce_op_workspace(int64_t n) { return desc::launch::reduce_op_workspace(n); }

namespace {
// The checks shared by the two reductions: `in` holds n 4-byte elements,
// `out` out_bytes bytes aligned to out_align.
desc_status reduce_op_checked(const void* in, int64_t n, void* out, int64_t out_bytes,
                              int64_t out_align, void* ws, size_t ws_bytes) {
  if (out == nullptr || ws == nullptr || (in == nullptr && n > 0)) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  DESC_TRY(check_device({n > 0 ? in : nullptr, out, ws}));
  if (misaligned(in, 4) || misaligned(out, out_align) || misaligned(ws, 8))
    return DESC_ERR_ALIGNMENT;
  if (overlap({out, out_bytes}, {in, nb}) || overlap({ws, (int64_t)ws_bytes}, {in, nb}) ||
      overlap({ws, (int64_t)ws_bytes}, {out, out_bytes}))
    return DESC_ERR_ALIAS;
  if (ws_bytes < desc_reduce_op_workspace(n)) return DESC_ERR_WORKSPACE;
  return DESC_OK;
}
}  // namespace

desc_status desc_reduce_minmax_i32(const int32_t* in, int64_t n, int32_t* out, void* ws,
                                   size_t ws_bytes, void* stream) {
  DESC_TRY(reduce_op_checked(in, n, out, 8, 4, ws, ws_bytes));
  return hip_status(desc::launch::minmax_i32(in, n, out, ws, (hipStream_t)stream));
}

desc_status desc_reduce_sum_f32(const float* in, int64_t n, double* out, void* ws,
                                size_t ws_bytes, void* stream) {
  DESC_TRY(reduce_op_checked(in, n, out, 8, 8, ws, ws_bytes));
  return hip_status(desc::launch::sum_f32(in, n, out, ws, (hipStream_t)stream));
}

// ----------------------------------------------------------------- scan
size_t desc_scan_i32_workspace(int64_t n) {
  return desc::launch::scan_i32_workspace(n < 0 ? 0 : n);
}

namespace {
desc_status scan_checked(const int32_t* in, int32_t* out, int64_t n, void* ws, size_t ws_bytes,
                         void* stream, bool exclusive) {
  if (ws == nullptr || ((in == nullptr || out == nullptr) && n > 0)) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  if (n == 0) return DESC_OK;
  DESC_TRY(check_device({in, out, ws}));
  if (misaligned(in, 4) || misaligned(out, 4) || misaligned(ws, 8)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb}) || overlap({ws, (int64_t)ws_bytes}, {in, nb}) ||
      overlap({ws, (int64_t)ws_bytes}, {out, nb}))
    return DESC_ERR_ALIAS;
  if (ws_bytes < desc_scan_i32_workspace(n)) return DESC_ERR_WORKSPACE;
  return hip_status(desc::launch::scan_i32(in, out, n, ws, (hipStream_t)stream, exclusive));
}
}  // namespace

desc_status desc_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                          size_t ws_bytes, void* stream) {
  return scan_checked(in, out, n, ws, ws_bytes, stream, false);
}

desc_status desc_scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                                    size_t ws_bytes, void* stream) {
  return scan_checked(in, out, n, ws, ws_bytes, stream, true);
}

desc_status desc_scan_i32_noalloc(const int32_t* in, int32_t* out, int64_t n, void* stream) {
  if ((in == nullptr || out == nullptr) && n > 0) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  if (n == 0) return DESC_OK;
  DESC_TRY(check_device({in, out}));
  if (misaligned(in, 4) || misaligned(out, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb})) return DESC_ERR_ALIAS;
  if (n > desc::launch::scan_noalloc_max_n()) return DESC_ERR_LIMIT;
  void* scratch = nullptr;
  size_t bytes = 0;
  DESC_TRY(hip_status(desc::launch::noalloc_scratch((hipStream_t)stream, &scratch, &bytes)));
  if (bytes < desc_scan_i32_workspace(n)) return DESC_ERR_LIMIT;
  return hip_status(desc::launch::scan_i32(in, out, n, scratch, (hipStream_t)stream, false));
}

// ----------------------------------------------------------------- fixed-order float scan
size_t desc_scan_f32_workspace(int64_t n) { return desc::launch::scan_f32_workspace(n); }

desc_status desc_scan_f32(const float* in, float* out, int64_t n, void* ws, size_t ws_bytes,
                          void* stream) {
  if (ws == nullptr || ((in == nullptr || out == nullptr) && n > 0)) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  if (n == 0) return DESC_OK;
  DESC_TRY(check_device({in, out, ws}));
  if (misaligned(in, 4) || misaligned(out, 4) || misaligned(ws, 8)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb}) || overlap({ws, (int64_t)ws_bytes}, {in, nb}) ||
      overlap({ws, (int64_t)ws_bytes}, {out, nb}))
    return DESC_ERR_ALIAS;
  if (ws_bytes < desc_scan_f32_workspace(n)) return DESC_ERR_WORKSPACE;
  return hip_status(desc::launch::scan_f32(in, out, n, ws, (hipStream_t)stream));
}

// ----------------------------------------------------------------- the paper's forms
desc_status desc_reduce_blocks_i32(const int32_t* in, int64_t n, int64_t E, int64_t* out,
                                   void* stream) {
  if ((in == nullptr || out == nullptr) && n > 0) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0 || E <= 0 || E % 1024 != 0) return DESC_ERR_SIZE;
  if (n == 0) return DESC_OK;
  const int64_t blocks = (n + E - 1) / E;
  if (blocks > INT32_MAX) return DESC_ERR_SIZE;
  const int64_t ob = blocks * 8;
  DESC_TRY(check_device({in, out}));
  if (misaligned(in, 4) || misaligned(out, 8)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, ob}, {in, nb})) return DESC_ERR_ALIAS;
  return hip_status(desc::launch::reduce_blocks_i32(in, n, E, out, (hipStream_t)stream));
}

size_t desc_scan_two_pass_i32_workspace(int64_t n) {
  return desc::launch::scan_two_pass_workspace(n < 0 ? 0 : n);
}

desc_status desc_scan_two_pass_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (ws == nullptr || ((in == nullptr || out == nullptr) && n > 0)) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  if (n == 0) return DESC_OK;
  DESC_TRY(check_device({in, out, ws}));
  if (misaligned(in, 4) || misaligned(out, 4) || misaligned(ws, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb}) || overlap({ws, (int64_t)ws_bytes}, {in, nb}) ||
      overlap({ws, (int64_t)ws_bytes}, {out, nb}))
    return DESC_ERR_ALIAS;
  if (ws_bytes < desc_scan_two_pass_i32_workspace(n)) return DESC_ERR_WORKSPACE;
  return hip_status(desc::launch::scan_two_pass_i32(in, out, n, ws, (hipStream_t)stream));
}

// ----------------------------------------------------------------- transpose
desc_status desc_transpose_batched_f32(const float* in, float* out, int64_t batch,
                                       int64_t rows, int64_t cols, void* stream) {
  if (batch < 0 || rows < 0 || cols < 0) return DESC_ERR_SIZE;
  const int64_t per = bytes_of(rows, cols);
  const int64_t cnt = per < 0 ? -1 : bytes_of(per, batch);
  const int64_t nb = cnt < 0 ? -1 : bytes_of(cnt, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  if (nb > 0 && (in == nullptr || out == nullptr)) return DESC_ERR_NULL;
  if (nb == 0) return DESC_OK;
  if (rows > desc::launch::transpose_max_rows() || batch > 65535 || cols > INT32_MAX)
    return DESC_ERR_UNSUPPORTED;
  DESC_TRY(check_device({in, out}));
  if (misaligned(in, 4) || misaligned(out, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb})) return DESC_ERR_ALIAS;
  return hip_status(desc::launch::transpose_32((const uint32_t*)in, (uint32_t*)out, batch, rows,
                                               cols, (hipStream_t)stream));
}

desc_status desc_transpose_f32(const float* in, float* out, int64_t rows, int64_t cols,
                               void* stream) {
  return desc_transpose_batched_f32(in, out, 1, rows, cols, stream);
}

desc_status desc_transpose_batched(const void* in, void* out, int64_t elem_bytes, int64_t batch,
                                   int64_t rows, int64_t cols, void* stream) {
  if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8)
    return DESC_ERR_UNSUPPORTED;
  if (elem_bytes == 4)
    return desc_transpose_batched_f32((const float*)in, (float*)out, batch, rows, cols, stream);
  if (batch < 0 || rows < 0 || cols < 0) return DESC_ERR_SIZE;
  const int64_t per = bytes_of(rows, cols);
  const int64_t cnt = per < 0 ? -1 : bytes_of(per, batch);
  const int64_t nb = cnt < 0 ? -1 : bytes_of(cnt, elem_bytes);
  if (nb < 0) return DESC_ERR_SIZE;
  if (nb > 0 && (in == nullptr || out == nullptr)) return DESC_ERR_NULL;
  if (nb == 0) return DESC_OK;
  if (rows > desc::launch::transpose_elem_max_rows(elem_bytes) || batch > 65535 ||
      cols > INT32_MAX)
    return DESC_ERR_UNSUPPORTED;
  DESC_TRY(check_device({in, out}));
  if (misaligned(in, (size_t)elem_bytes) || misaligned(out, (size_t)elem_bytes))
    return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb})) return DESC_ERR_ALIAS;
  return hip_status(
      desc::launch::transpose_elem(in, out, elem_bytes, batch, rows, cols, (hipStream_t)stream));
}

// ----------------------------------------------------------------- GEMM
size_t desc_gemm_workspace(desc_gemm_mode mode, int64_t M, int64_t N, int64_t K) {
  if (M < 0 || N < 0 || K < 0) return 0;
  switch (mode) {
    case DESC_GEMM_BF16X3: return desc::launch::gemm_lowp_workspace(1, M, N, K);
    case DESC_GEMM_FP8_ROWCOL: return desc::launch::gemm_lowp_workspace(2, M, N, K);
    default: return 0;
  }
}

namespace {

// Byte extent of a row-major rows x cols matrix with row stride ld (in
// elements of `es` bytes); -1 on overflow.
int64_t matrix_bytes(int64_t rows, int64_t cols, int64_t ld, int64_t es) {
  if (rows == 0 || cols == 0) return 0;
  const int64_t last = bytes_of(rows - 1, ld);
  if (last < 0 || last > INT64_MAX - cols) return -1;
  return bytes_of(last + cols, es);
}

}  // namespace

desc_status desc_gemm(desc_gemm_mode mode, int64_t M, int64_t N, int64_t K, const float* A,
                      int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc, void* ws,
                      size_t ws_bytes, void* stream) {
  if (M < 0 || N < 0 || K < 0) return DESC_ERR_SIZE;
  if (mode != DESC_GEMM_F32 && mode != DESC_GEMM_BF16X3 && mode != DESC_GEMM_FP8_ROWCOL)
    return DESC_ERR_UNSUPPORTED;
  if (M == 0 || N == 0) return DESC_OK;
  const size_t need = desc_gemm_workspace(mode, M, N, K);
  if (C == nullptr || (K > 0 && (A == nullptr || B == nullptr)) || (need > 0 && ws == nullptr))
    return DESC_ERR_NULL;
  // row-major with leading dimensions at least the row lengths
  if (ldc < N || (K > 0 && (lda < K || ldb < N))) return DESC_ERR_SIZE;
  const int64_t a_b = matrix_bytes(M, K, lda, 4), b_b = matrix_bytes(K, N, ldb, 4);
  const int64_t c_b = matrix_bytes(M, N, ldc, 4);
  if (a_b < 0 || b_b < 0 || c_b < 0 || M > ((int64_t)1 << 31) || N > ((int64_t)1 << 31))
    return DESC_ERR_SIZE;
  DESC_TRY(check_device({K > 0 ? (const void*)A : nullptr, K > 0 ? (const void*)B : nullptr, C,
                         need > 0 ? ws : nullptr}));
  if (misaligned(A, 4) || misaligned(B, 4) || misaligned(C, 4) || misaligned(ws, 256))
    return DESC_ERR_ALIGNMENT;
  if (overlap({C, c_b}, {A, a_b}) || overlap({C, c_b}, {B, b_b})) return DESC_ERR_ALIAS;
  if (need > 0 && (overlap({ws, (int64_t)ws_bytes}, {A, a_b}) ||
                   overlap({ws, (int64_t)ws_bytes}, {B, b_b}) ||
                   overlap({ws, (int64_t)ws_bytes}, {C, c_b})))
    return DESC_ERR_ALIAS;
  if (ws_bytes < need) return DESC_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (K == 0 || mode == DESC_GEMM_F32)
    return hip_status(desc::launch::gemm_f32(A, lda, B, ldb, C, ldc, M, N, K, s));
  if (mode == DESC_GEMM_BF16X3)
    return hip_status(desc::launch::gemm_bf16x3(A, lda, B, ldb, C, ldc, M, N, K, ws, s));
  return hip_status(desc::launch::gemm_fp8(A, lda, B, ldb, C, ldc, M, N, K, ws, s));
}

// ----------------------------------------------------------------- operand preparation
desc_status desc_split_bf16_rows(const float* A, int64_t M, int64_t K, int64_t lda,
                                 uint16_t* hi, uint16_t* lo, int64_t ldh, void* stream) {
  if (M < 0 || K < 0) return DESC_ERR_SIZE;
  if (M == 0 || K == 0) return DESC_OK;
  if (A == nullptr || hi == nullptr || lo == nullptr) return DESC_ERR_NULL;
  if (lda < K || ldh < K) return DESC_ERR_SIZE;
  const int64_t a_b = matrix_bytes(M, K, lda, 4), h_b = matrix_bytes(M, K, ldh, 2);
  if (a_b < 0 || h_b < 0) return DESC_ERR_SIZE;
  DESC_TRY(check_device({A, hi, lo}));
  if (misaligned(A, 4) || misaligned(hi, 2) || misaligned(lo, 2)) return DESC_ERR_ALIGNMENT;
  if (overlap({hi, h_b}, {A, a_b}) || overlap({lo, h_b}, {A, a_b}) || overlap({hi, h_b}, {lo, h_b}))
    return DESC_ERR_ALIAS;
  return hip_status(
      desc::launch::split_bf16_rows(A, M, K, lda, hi, lo, ldh, (hipStream_t)stream));
}

desc_status desc_split_bf16_cols(const float* B, int64_t K, int64_t N, int64_t ldb,
                                 uint16_t* hi_t, uint16_t* lo_t, int64_t ldh, void* stream) {
  if (K < 0 || N < 0) return DESC_ERR_SIZE;
  if (K == 0 || N == 0) return DESC_OK;
  if (B == nullptr || hi_t == nullptr || lo_t == nullptr) return DESC_ERR_NULL;
  if (ldb < N || ldh < K || K > (int64_t)65535 * 64 * 64 || N > (int64_t)65535 * 64)
    return DESC_ERR_SIZE;
  const int64_t b_b = matrix_bytes(K, N, ldb, 4), h_b = matrix_bytes(N, K, ldh, 2);
  if (b_b < 0 || h_b < 0) return DESC_ERR_SIZE;
  DESC_TRY(check_device({B, hi_t, lo_t}));
  if (misaligned(B, 4) || misaligned(hi_t, 2) || misaligned(lo_t, 2)) return DESC_ERR_ALIGNMENT;
  if (overlap({hi_t, h_b}, {B, b_b}) || overlap({lo_t, h_b}, {B, b_b}) ||
      overlap({hi_t, h_b}, {lo_t, h_b}))
    return DESC_ERR_ALIAS;
  return hip_status(
      desc::launch::split_bf16_cols(B, K, N, ldb, hi_t, lo_t, ldh, (hipStream_t)stream));
}

desc_status desc_quant_e4m3_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint8_t* q,
                                 int64_t ldq, float* scale, void* stream) {
  if (M < 0 || K < 0) return DESC_ERR_SIZE;
  if (M == 0) return DESC_OK;
  if (scale == nullptr || (K > 0 && (A == nullptr || q == nullptr))) return DESC_ERR_NULL;
  if (M > INT32_MAX || (K > 0 && (lda < K || ldq < K))) return DESC_ERR_SIZE;
  const int64_t a_b = matrix_bytes(M, K, lda, 4), q_b = matrix_bytes(M, K, ldq, 1);
  if (a_b < 0 || q_b < 0) return DESC_ERR_SIZE;
  DESC_TRY(check_device({K > 0 ? (const void*)A : nullptr, K > 0 ? (const void*)q : nullptr,
                         scale}));
  if (misaligned(A, 4) || misaligned(scale, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({q, q_b}, {A, a_b}) || overlap({scale, M * 4}, {A, a_b}) ||
      overlap({scale, M * 4}, {q, q_b}))
    return DESC_ERR_ALIAS;
  return hip_status(
      desc::launch::quant_e4m3_rows(A, M, K, lda, q, ldq, scale, (hipStream_t)stream));
}

size_t desc_quant_e4m3_cols_workspace(int64_t K, int64_t N) {
  if (K < 0 || N < 0) return 0;
  return desc::launch::quant_e4m3_cols_workspace(K, N);
}

desc_status desc_quant_e4m3_cols(const float* B, int64_t K, int64_t N, int64_t ldb,
                                 uint8_t* q_t, int64_t ldq, float* scale, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (K < 0 || N < 0) return DESC_ERR_SIZE;
  if (N == 0) return DESC_OK;
  if (scale == nullptr || ws == nullptr || (K > 0 && (B == nullptr || q_t == nullptr)))
    return DESC_ERR_NULL;
  if ((K > 0 && (ldb < N || ldq < K)) || K > (int64_t)65535 * 64 * 64 ||
      N > (int64_t)65535 * 64)
    return DESC_ERR_SIZE;
  const int64_t b_b = matrix_bytes(K, N, ldb, 4), q_b = matrix_bytes(N, K, ldq, 1);
  if (b_b < 0 || q_b < 0) return DESC_ERR_SIZE;
  DESC_TRY(check_device({K > 0 ? (const void*)B : nullptr, K > 0 ? (const void*)q_t : nullptr,
                         scale, ws}));
  if (misaligned(B, 4) || misaligned(scale, 4) || misaligned(ws, 4)) return DESC_ERR_ALIGNMENT;
  const int64_t wsb = (int64_t)ws_bytes;
  if (overlap({q_t, q_b}, {B, b_b}) || overlap({scale, N * 4}, {B, b_b}) ||
      overlap({scale, N * 4}, {q_t, q_b}) || overlap({ws, wsb}, {B, b_b}) ||
      overlap({ws, wsb}, {q_t, q_b}) || overlap({ws, wsb}, {scale, N * 4}))
    return DESC_ERR_ALIAS;
  if (ws_bytes < desc_quant_e4m3_cols_workspace(K, N)) return DESC_ERR_WORKSPACE;
  return hip_status(
      desc::launch::quant_e4m3_cols(B, K, N, ldb, q_t, ldq, scale, ws, (hipStream_t)stream));
}

// ----------------------------------------------------------------- grouped GEMM
size_t desc_gemm_grouped_workspace(int64_t G) {
  return G < 0 ? 0 : desc::launch::gemm_grouped_workspace(G);
}

size_t desc_gemm_grouped_workspace_for(desc_gemm_mode mode, int64_t G,
                                       const desc_gemm_problem* problems_host) {
  if (G < 0 || G > INT32_MAX) return 0;
  if (mode == DESC_GEMM_F32) return desc::launch::gemm_grouped_workspace(G);
  if (mode != DESC_GEMM_BF16X3) return 0;
  if (G > 0 && problems_host == nullptr) return 0;
  const size_t total = desc::launch::gemm_grouped_bf16x3_workspace(problems_host, G);
  return total == SIZE_MAX ? 0 : total;   // refused shape or overflow
}

desc_status desc_gemm_grouped(desc_gemm_mode mode, int64_t G, const desc_gemm_problem* problems,
                              void* ws, size_t ws_bytes, void* stream) {
  if (G < 0) return DESC_ERR_SIZE;
  if (mode != DESC_GEMM_F32 && mode != DESC_GEMM_BF16X3) return DESC_ERR_UNSUPPORTED;
  if (G == 0) return DESC_OK;
  if (problems == nullptr || ws == nullptr) return DESC_ERR_NULL;
  const int64_t pb = bytes_of(G, (int64_t)sizeof(desc_gemm_problem));
  if (pb < 0 || G > INT32_MAX) return DESC_ERR_SIZE;
  DESC_TRY(check_device({problems, ws}));
  const size_t align = mode == DESC_GEMM_F32 ? 64 : 256;
  if (misaligned(problems, 8) || misaligned(ws, align)) return DESC_ERR_ALIGNMENT;
  if (overlap({ws, (int64_t)ws_bytes}, {problems, pb})) return DESC_ERR_ALIAS;
  if (mode == DESC_GEMM_F32) {
    if (ws_bytes < desc_gemm_grouped_workspace(G)) return DESC_ERR_WORKSPACE;
    return hip_status(desc::launch::gemm_grouped_f32(problems, G, ws, (hipStream_t)stream));
  }
  if (ws_bytes < desc::launch::gemm_grouped_bf16x3_head(G)) return DESC_ERR_WORKSPACE;
  return hip_status(
      desc::launch::gemm_grouped_bf16x3(problems, G, ws, ws_bytes, (hipStream_t)stream));
}

// ----------------------------------------------------------------- strided batched GEMM
namespace {
// Bytes from the first element of batch 0 to the end of the last row of
// batch G - 1 (rows x cols at leading dimension ld, batches `stride` apart).
int64_t batch_span_bytes(int64_t G, int64_t stride, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t one = matrix_bytes(rows, cols, ld, 4);
  if (one <= 0 || G <= 1) return one;
  const int64_t step = bytes_of(G - 1, stride);
  if (step < 0 || step > INT64_MAX / 4) return -1;
  if (step * 4 > INT64_MAX - one) return -1;
  return step * 4 + one;
}
}  // namespace

size_t desc_gemm_strided_batched_workspace(desc_gemm_mode mode, int64_t G, int64_t M, int64_t N,
                                           int64_t K, int64_t lda, int64_t ldb) {
  if (G < 0 || G > INT32_MAX || M < 0 || N < 0 || K < 0) return 0;
  // the grouped workspace first (rounded up to 256 bytes), then the descriptors
  const size_t descs = desc::launch::strided_problems_bytes(G);
  size_t rest = 0;
  if (mode == DESC_GEMM_F32) {
    rest = desc::launch::gemm_grouped_workspace(G);
  } else {
    if (mode != DESC_GEMM_BF16X3) return 0;
    const desc_gemm_problem p{M, N, K, lda, ldb, N, nullptr, nullptr, nullptr};
    rest = desc::launch::gemm_grouped_bf16x3_workspace_uniform(p, G);
  }
  if (rest >= SIZE_MAX - 511 - descs) return 0;
  return ((rest + 255) & ~(size_t)255) + descs;
}

desc_status desc_gemm_strided_batched(desc_gemm_mode mode, int64_t G, int64_t M, int64_t N,
                                      int64_t K, const float* A, int64_t lda, int64_t stride_a,
                                      const float* B, int64_t ldb, int64_t stride_b, float* C,
                                      int64_t ldc, int64_t stride_c, void* ws, size_t ws_bytes,
                                      void* stream) {
  if (G < 0 || M < 0 || N < 0 || K < 0 || stride_a < 0 || stride_b < 0 || stride_c < 0)
    return DESC_ERR_SIZE;
  if (mode != DESC_GEMM_F32 && mode != DESC_GEMM_BF16X3) return DESC_ERR_UNSUPPORTED;
  if (G == 0 || M == 0 || N == 0) return DESC_OK;
  if (C == nullptr || ws == nullptr || (K > 0 && (A == nullptr || B == nullptr)))
    return DESC_ERR_NULL;
  if (G > INT32_MAX || ldc < N || (K > 0 && (lda < K || ldb < N))) return DESC_ERR_SIZE;
  const int64_t a_b = K > 0 ? batch_span_bytes(G, stride_a, M, K, lda) : 0;
  const int64_t b_b = K > 0 ? batch_span_bytes(G, stride_b, K, N, ldb) : 0;
  const int64_t c_b = batch_span_bytes(G, stride_c, M, N, ldc);
  if (a_b < 0 || b_b < 0 || c_b < 0) return DESC_ERR_SIZE;
  DESC_TRY(check_device({K > 0 ? (const void*)A : nullptr, K > 0 ? (const void*)B : nullptr, C,
                         ws}));
  if (misaligned(A, 4) || misaligned(B, 4) || misaligned(C, 4) || misaligned(ws, 256))
    return DESC_ERR_ALIGNMENT;
  // outputs must not overlap the operands, one another, or the workspace
  if (overlap({C, c_b}, {A, a_b}) || overlap({C, c_b}, {B, b_b}) ||
      (G > 1 && stride_c < (M - 1) * ldc + N))
    return DESC_ERR_ALIAS;
  const int64_t wsb = (int64_t)ws_bytes;
  if (overlap({ws, wsb}, {A, a_b}) || overlap({ws, wsb}, {B, b_b}) || overlap({ws, wsb}, {C, c_b}))
    return DESC_ERR_ALIAS;
  const size_t need = desc_gemm_strided_batched_workspace(mode, G, M, N, K, lda, ldb);
  if (need == 0) return DESC_ERR_SIZE;
  if (ws_bytes < need) return DESC_ERR_WORKSPACE;
  return hip_status(desc::launch::gemm_strided_batched(mode, G, M, N, K, A, lda, stride_a, B,
                                                       ldb, stride_b, C, ldc, stride_c, ws,
                                                       ws_bytes, (hipStream_t)stream));
}

// ----------------------------------------------------------------- uniform batched reduce/scan
size_t desc_reduce_batched_i32_workspace(int64_t batch, int64_t len) {
  if (batch < 0 || len < 0 || (len > 0 && batch > INT64_MAX / len)) return 0;
  return desc::launch::batched_workspace(batch, len, false);
}

size_t desc_scan_batched_i32_workspace(int64_t batch, int64_t len) {
  if (batch < 0 || len < 0 || (len > 0 && batch > INT64_MAX / len)) return 0;
  return desc::launch::batched_workspace(batch, len, true);
}

namespace {
desc_status check_batched(const int32_t* in, const void* out, int64_t out_bytes, int64_t n,
                          int64_t batch, void* ws, size_t ws_bytes, size_t need) {
  if (ws == nullptr || out == nullptr || (n > 0 && in == nullptr)) return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0 || out_bytes < 0 || batch > INT32_MAX ||
      desc::launch::segmented_max_grid(n, batch) > INT32_MAX)
    return DESC_ERR_SIZE;
  DESC_TRY(check_device({n > 0 ? (const void*)in : nullptr, out, ws}));
  if (misaligned(in, 4) || misaligned(out, 4) || misaligned(ws, 8)) return DESC_ERR_ALIGNMENT;
  const int64_t wsb = (int64_t)ws_bytes;
  if (overlap({out, out_bytes}, {in, nb}) || overlap({ws, wsb}, {in, nb}) ||
      overlap({ws, wsb}, {out, out_bytes}))
    return DESC_ERR_ALIAS;
  if (ws_bytes < need) return DESC_ERR_WORKSPACE;
  return DESC_OK;
}
}  // namespace

desc_status desc_reduce_batched_i32(const int32_t* in, int64_t batch, int64_t len, int64_t* out,
                                    void* ws, size_t ws_bytes, void* stream) {
  if (batch < 0 || len < 0 || (len > 0 && batch > INT64_MAX / len)) return DESC_ERR_SIZE;
  if (batch == 0) return DESC_OK;
  const int64_t ob = bytes_of(batch, 8);
  DESC_TRY(check_batched(in, out, ob, batch * len, batch, ws, ws_bytes,
                         desc_reduce_batched_i32_workspace(batch, len)));
  if (misaligned(out, 8)) return DESC_ERR_ALIGNMENT;
  return hip_status(
      desc::launch::reduce_batched_i32(in, batch, len, out, ws, (hipStream_t)stream));
}

desc_status desc_scan_batched_i32(const int32_t* in, int32_t* out, int64_t batch, int64_t len,
                                  void* ws, size_t ws_bytes, void* stream) {
  if (batch < 0 || len < 0 || (len > 0 && batch > INT64_MAX / len)) return DESC_ERR_SIZE;
  if (batch == 0 || len == 0) return DESC_OK;
  DESC_TRY(check_batched(in, out, bytes_of(batch * len, 4), batch * len, batch, ws, ws_bytes,
                         desc_scan_batched_i32_workspace(batch, len)));
  return hip_status(
      desc::launch::scan_batched_i32(in, out, batch, len, ws, (hipStream_t)stream));
}

// ----------------------------------------------------------------- segmented
size_t desc_reduce_segmented_i32_workspace(int64_t n, int64_t num_segments) {
  if (n < 0 || num_segments < 0) return 0;
  return desc::launch::segmented_workspace(n, num_segments, false);
}

size_t desc_scan_segmented_i32_workspace(int64_t n, int64_t num_segments) {
  if (n < 0 || num_segments < 0) return 0;
  return desc::launch::segmented_workspace(n, num_segments, true);
}

namespace {

desc_status check_segmented(const int32_t* in, const void* out, int64_t out_bytes, int64_t n,
                            const int64_t* offsets, int64_t S, void* ws, size_t ws_bytes,
                            size_t need) {
  if (offsets == nullptr || ws == nullptr || (n > 0 && in == nullptr) ||
      (out == nullptr && out_bytes > 0))
    return DESC_ERR_NULL;
  const int64_t nb = bytes_of(n, 4), ob = bytes_of(S + 1, 8);
  if (nb < 0 || ob < 0 || out_bytes < 0 || desc::launch::segmented_max_grid(n, S) > INT32_MAX)
    return DESC_ERR_SIZE;
  DESC_TRY(check_device({n > 0 ? (const void*)in : nullptr, offsets, out, ws}));
  if (misaligned(in, 4) || misaligned(offsets, 8) || misaligned(out, 4) || misaligned(ws, 8))
    return DESC_ERR_ALIGNMENT;
  const int64_t wsb = (int64_t)ws_bytes;
  if (overlap({out, out_bytes}, {in, nb}) || overlap({out, out_bytes}, {offsets, ob}) ||
      overlap({ws, wsb}, {in, nb}) || overlap({ws, wsb}, {offsets, ob}) ||
      overlap({ws, wsb}, {out, out_bytes}))
    return DESC_ERR_ALIAS;
  if (ws_bytes < need) return DESC_ERR_WORKSPACE;
  return DESC_OK;
}

}  // namespace

desc_status desc_reduce_segmented_i32(const int32_t* in, int64_t n, const int64_t* offsets,
                                      int64_t num_segments, int64_t* out, void* ws,
                                      size_t ws_bytes, void* stream) {
  if (n < 0 || num_segments < 0) return DESC_ERR_SIZE;
  if (num_segments == 0) return DESC_OK;
  const int64_t ob = bytes_of(num_segments, 8);
  DESC_TRY(check_segmented(in, out, ob, n, offsets, num_segments, ws, ws_bytes,
                           desc_reduce_segmented_i32_workspace(n, num_segments)));
  if (misaligned(out, 8)) return DESC_ERR_ALIGNMENT;
  return hip_status(desc::launch::reduce_segmented_i32(in, n, offsets, num_segments, out, ws,
                                                       (hipStream_t)stream));
}

desc_status desc_scan_segmented_i32(const int32_t* in, int32_t* out, int64_t n,
                                    const int64_t* offsets, int64_t num_segments, void* ws,
                                    size_t ws_bytes, void* stream) {
  if (n < 0 || num_segments < 0) return DESC_ERR_SIZE;
  if (num_segments == 0 || n == 0) return DESC_OK;
  DESC_TRY(check_segmented(in, out, bytes_of(n, 4), n, offsets, num_segments, ws, ws_bytes,
                           desc_scan_segmented_i32_workspace(n, num_segments)));
  return hip_status(desc::launch::scan_segmented_i32(in, out, n, offsets, num_segments, ws,
                                                     (hipStream_t)stream));
}

// ----------------------------------------------------------------- copy
desc_status desc_copy_32(const void* in, void* out, int64_t n, void* stream) {
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  if (nb > 0 && (in == nullptr || out == nullptr)) return DESC_ERR_NULL;
  if (nb == 0) return DESC_OK;
  DESC_TRY(check_device({in, out}));
  if (misaligned(in, 4) || misaligned(out, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb})) return DESC_ERR_ALIAS;
  return hip_status(
      desc::launch::copy_32((const uint32_t*)in, (uint32_t*)out, n, (hipStream_t)stream));
}

desc_status desc_reverse_u32(const void* in, void* out, int64_t n, void* stream) {
  const int64_t nb = bytes_of(n, 4);
  if (nb < 0) return DESC_ERR_SIZE;
  if (nb > 0 && (in == nullptr || out == nullptr)) return DESC_ERR_NULL;
  if (nb == 0) return DESC_OK;
  DESC_TRY(check_device({in, out}));
  if (misaligned(in, 4) || misaligned(out, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({out, nb}, {in, nb})) return DESC_ERR_ALIAS;
  return hip_status(
      desc::launch::reverse_32((const uint32_t*)in, (uint32_t*)out, n, (hipStream_t)stream));
}

// ----------------------------------------------------------------- configurations
int desc_config_count(desc_op op) { return desc::tune::config_count((int)op); }

const char* desc_config_name(desc_op op, int cfg) { return desc::tune::config_name((int)op, cfg); }

const char* desc_op_name(desc_op op) { return desc::tune::op_name((int)op); }

int desc_size_class(desc_op op, int64_t size) { return desc::tune::size_class((int)op, size); }

desc_status desc_config_set(desc_op op, int size_class, int cfg) {
  return desc::tune::set((int)op, size_class, cfg) ? DESC_OK : DESC_ERR_UNSUPPORTED;
}

int desc_config_get(desc_op op, int size_class) {
  if ((int)op < 0 || (int)op >= desc::tune::kNumOps || size_class < 0 ||
      size_class >= desc::tune::kClasses)
    return -1;
  return desc::tune::get((int)op, size_class);
}

desc_status desc_config_load(const char* path) {
  if (path == nullptr) return DESC_ERR_NULL;
  FILE* f = fopen(path, "r");
  if (f == nullptr) return DESC_ERR_UNSUPPORTED;
  char line[256];
  desc_status st = DESC_OK;
  while (fgets(line, sizeof line, f)) {
    char op[64], cfg[64];
    int cls = -1;
    if (line[0] == '#' || sscanf(line, "%63s %d %63s", op, &cls, cfg) != 3) continue;
    int o = -1, c = -1;
    for (int i = 0; i < desc::tune::kNumOps; ++i)
      if (desc::tune::op_name(i) && strcmp(desc::tune::op_name(i), op) == 0) o = i;
    for (int j = 0; o >= 0 && j < desc::tune::config_count(o); ++j)
      if (strcmp(desc::tune::config_name(o, j), cfg) == 0) c = j;
    if (o < 0 || c < 0 || !desc::tune::set(o, cls, c)) st = DESC_ERR_UNSUPPORTED;
  }
  fclose(f);
  return st;
}

}  // extern "C"
