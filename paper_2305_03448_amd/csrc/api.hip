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
  }
  return "unknown desc_status";
}

int desc_last_hip_error(void) { return g_last_hip_error; }

int desc_version(void) { return 100; }

void desc_set_pointer_classifier(desc_pointer_classifier fn) {
  g_classifier.store(fn, std::memory_order_release);
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

// ----------------------------------------------------------------- scan
size_t desc_scan_i32_workspace(int64_t n) {
  return desc::launch::scan_i32_workspace(n < 0 ? 0 : n);
}

desc_status desc_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                          size_t ws_bytes, void* stream) {
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
  return hip_status(desc::launch::scan_i32(in, out, n, ws, (hipStream_t)stream));
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

// ----------------------------------------------------------------- GEMM
size_t desc_gemm_workspace(desc_gemm_mode mode, int64_t M, int64_t N, int64_t K) {
  if (M < 0 || N < 0 || K < 0) return 0;
  switch (mode) {
    case DESC_GEMM_F32: return 0;
    default: return 0;
  }
}

desc_status desc_gemm(desc_gemm_mode mode, int64_t M, int64_t N, int64_t K, const float* A,
                      int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc, void* ws,
                      size_t ws_bytes, void* stream) {
  if (M < 0 || N < 0 || K < 0) return DESC_ERR_SIZE;
  if (mode != DESC_GEMM_F32) return DESC_ERR_UNSUPPORTED;
  if (M == 0 || N == 0) return DESC_OK;
  if (C == nullptr || (K > 0 && (A == nullptr || B == nullptr))) return DESC_ERR_NULL;
  // row-major with leading dimensions at least the row lengths
  if (ldc < N || (K > 0 && (lda < K || ldb < N))) return DESC_ERR_SIZE;
  const int64_t a_el = K > 0 ? bytes_of(M - 1, lda) : 0, b_el = K > 0 ? bytes_of(K - 1, ldb) : 0;
  const int64_t c_el = bytes_of(M - 1, ldc);
  if (a_el < 0 || b_el < 0 || c_el < 0) return DESC_ERR_SIZE;
  const int64_t a_b = K > 0 ? bytes_of(a_el + K, 4) : 0, b_b = K > 0 ? bytes_of(b_el + N, 4) : 0;
  const int64_t c_b = bytes_of(c_el + N, 4);
  if (a_b < 0 || b_b < 0 || c_b < 0 || M * N > ((int64_t)1 << 46)) return DESC_ERR_SIZE;
  DESC_TRY(check_device({K > 0 ? (const void*)A : nullptr, K > 0 ? (const void*)B : nullptr, C,
                         ws_bytes ? ws : nullptr}));
  if (misaligned(A, 4) || misaligned(B, 4) || misaligned(C, 4)) return DESC_ERR_ALIGNMENT;
  if (overlap({C, c_b}, {A, a_b}) || overlap({C, c_b}, {B, b_b})) return DESC_ERR_ALIAS;
  const size_t need = desc_gemm_workspace(mode, M, N, K);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) return DESC_ERR_WORKSPACE;
  return hip_status(
      desc::launch::gemm_f32(A, lda, B, ldb, C, ldc, M, N, K, (hipStream_t)stream));
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
