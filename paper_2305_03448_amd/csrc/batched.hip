// batched.hip -- uniform batched forms on top of the segmented and grouped
// kernels: B rows of L int32 reduced or scanned row by row, and G GEMMs of
// one shape at fixed strides.
//
// A uniform batch is a segmented (or grouped) problem whose description is
// implicit.  A one-pass kernel writes that description into the back of
// the workspace -- offsets s * L for s <= B, or G problem descriptors at
// the given strides -- and the segmented or grouped kernels run on it
// unchanged, with their own workspace at the front (so its header, and the
// device status word in it, sits where it does for the direct calls), and
// results and guarantees are theirs.  The description costs
// 8 (B + 1) or 72 G bytes of writes, and a kernel rather than a host copy
// keeps the call capture-safe and free of host-to-device traffic.
#include "common.hpp"
#include "launch.hpp"
#include "view.hpp"

namespace desc {
namespace {

constexpr int kFillBlock = 256;

__global__ __launch_bounds__(kFillBlock) void uniform_offsets_kernel(int64_t* __restrict__ off,
                                                                     int64_t B, int64_t L) {
  auto o = array(off, B + 1);
  const idx_t s = (idx_t)block_x().index() * kFillBlock + thread_x<kFillBlock>().index();
  if (s <= B) o[s] = s * L;
}

__global__ __launch_bounds__(kFillBlock) void strided_problems_kernel(
    desc_gemm_problem* __restrict__ p, int64_t G, int64_t M, int64_t N, int64_t K,
    const float* A, int64_t lda, int64_t sa, const float* Bm, int64_t ldb, int64_t sb, float* C,
    int64_t ldc, int64_t sc) {
  auto probs = array(p, G);
  const idx_t g = (idx_t)block_x().index() * kFillBlock + thread_x<kFillBlock>().index();
  if (g < G) probs[g] = desc_gemm_problem{M, N, K, lda, ldb, ldc, A + g * sa, Bm + g * sb, C + g * sc};
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

namespace launch {

size_t batched_offsets_bytes(int64_t B) { return round256(8 * (size_t)(B + 1)); }
size_t strided_problems_bytes(int64_t G) { return round256(sizeof(desc_gemm_problem) * (size_t)G); }

size_t batched_workspace(int64_t B, int64_t L, bool scan) {
  return round256(segmented_workspace(B * L, B, scan)) + batched_offsets_bytes(B);
}

static hipError_t batched_offsets(int64_t B, int64_t L, bool scan, void* ws, int64_t** off,
                                  hipStream_t s) {
  *off = (int64_t*)((char*)ws + round256(segmented_workspace(B * L, B, scan)));
  hipLaunchKernelGGL(uniform_offsets_kernel, dim3((unsigned)((B + kFillBlock) / kFillBlock)),
                     dim3(kFillBlock), 0, s, *off, B, L);
  return hipGetLastError();
}

hipError_t reduce_batched_i32(const int32_t* in, int64_t B, int64_t L, int64_t* out, void* ws,
                              hipStream_t s) {
  int64_t* off = nullptr;
  const hipError_t e = batched_offsets(B, L, false, ws, &off, s);
  if (e != hipSuccess) return e;
  return reduce_segmented_i32(in, B * L, off, B, out, ws, s, false);
}

hipError_t scan_batched_i32(const int32_t* in, int32_t* out, int64_t B, int64_t L, void* ws,
                            hipStream_t s) {
  int64_t* off = nullptr;
  const hipError_t e = batched_offsets(B, L, true, ws, &off, s);
  if (e != hipSuccess) return e;
  return scan_segmented_i32(in, out, B * L, off, B, ws, s);
}

hipError_t gemm_strided_batched(int mode, int64_t G, int64_t M, int64_t N, int64_t K,
                                const float* A, int64_t lda, int64_t sa, const float* Bm,
                                int64_t ldb, int64_t sb, float* C, int64_t ldc, int64_t sc,
                                void* ws, size_t ws_bytes, hipStream_t s) {
  // The descriptors take the last 256-byte-aligned strided_problems_bytes(G)
  // of the workspace; the grouped kernels get everything before them.
  const size_t rest_bytes = (ws_bytes - strided_problems_bytes(G)) & ~(size_t)255;
  desc_gemm_problem* p = (desc_gemm_problem*)((char*)ws + rest_bytes);
  hipLaunchKernelGGL(strided_problems_kernel, dim3((unsigned)((G + kFillBlock - 1) / kFillBlock)),
                     dim3(kFillBlock), 0, s, p, G, M, N, K, A, lda, sa, Bm, ldb, sb, C, ldc, sc);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == DESC_GEMM_F32) return gemm_grouped_f32(p, G, ws, s);
  return gemm_grouped_bf16x3(p, G, ws, rest_bytes, s);
}

}  // namespace launch
}  // namespace desc
