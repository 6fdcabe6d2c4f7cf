// gemm_f32.hip -- C = A * B in FP32 on the matrix cores (the "matrix
// multiplication" benchmark of Sec. 5; precision and layout read as FP32,
// row-major, C overwritten).
//
// A is M x K (row stride lda), B is K x N (row stride ldb), C is M x N (row
// stride ldc), all row-major FP32.  Block tiles are BM x BN with a K step of
// BK; the four waves of a block form a 2 x 2 grid, each owning a
// (BM/2) x (BN/2) tile of 32 x 32 v_mfma_f32_32x32x2_f32 fragments.
//
// Per K step, the block copies the A tile into LDS k-major ([BK][BM]) and
// the B tile as it is ([BK][BN]), so that the 64 lanes of a wave read a
// fragment from consecutive LDS words.  The LDS tiles are double buffered:
// the global loads of step t+1 are issued before the matrix ops of step t
// and written to the other buffer after them, one barrier per step.  Edge
// tiles (and unaligned operands) load element by element with zero fill
// and store under guards, so any M, N, K and leading dimensions work.
//
// The tile routine is shared with the grouped GEMM (grouped.hip).
#include "gemm_f32.hpp"
#include "launch.hpp"
#include "tuning.hpp"

namespace desc {
namespace {

template <class C, bool kVec>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ B, int64_t ldb,
                                                       float* __restrict__ Cm, int64_t ldc,
                                                       int64_t M, int64_t N, int64_t K) {
  __shared__ float lds[gemm_f32::lds_floats<C>()];
  const GemmProblemF32 p{A, lda, B, ldb, Cm, ldc, M, N, K};
  const idx_t tiles_n = (N + C::bn - 1) / C::bn;
  const idx_t t = gemm_f32::xcd_tile(block_x(), (M + C::bm - 1) / C::bm, tiles_n);
  gemm_f32::tile<C, kVec>(p, t / tiles_n, t % tiles_n, lds);
}

template <class C, bool kVec>
__global__ __launch_bounds__(C::threads) __attribute__((amdgpu_waves_per_eu(C::depth)))
void gemm_f32w_kernel(
    const float* __restrict__ A, int64_t lda, const float* __restrict__ B, int64_t ldb,
    float* __restrict__ Cm, int64_t ldc, int64_t M, int64_t N, int64_t K) {
  __shared__ __attribute__((aligned(16))) float lds[C::lds_floats];
  const GemmProblemF32 p{A, lda, B, ldb, Cm, ldc, M, N, K};
  const idx_t tiles_n = (N + C::bn - 1) / C::bn;
  const idx_t t = gemm_f32::xcd_tile(block_x(), (M + C::bm - 1) / C::bm, tiles_n);
  const idx_t tm = t / tiles_n, tn = t % tiles_n;
  if (kVec && gemm_f32::interior_tile<C>(p, tm, tn))
    gemm_f32::tile_rowmajor<C, true, true>(p, tm, tn, lds);
  else
    gemm_f32::tile_rowmajor<C, kVec>(p, tm, tn, lds);
}

template <class C>
hipError_t launch_gemm_w(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                         int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s) {
  const int64_t tiles = ((M + C::bm - 1) / C::bm) * ((N + C::bn - 1) / C::bn);
  // the clamped group loads need K and N in whole groups of four (K, N >= 4)
  if (gemm_f32::vec_ok(A, lda, B, ldb) && K % 4 == 0 && N % 4 == 0 && K > 0)
    hipLaunchKernelGGL((gemm_f32w_kernel<C, true>), dim3((unsigned)tiles), dim3(C::threads), 0,
                       s, A, lda, B, ldb, Cm, ldc, M, N, K);
  else
    hipLaunchKernelGGL((gemm_f32w_kernel<C, false>), dim3((unsigned)tiles), dim3(C::threads), 0,
                       s, A, lda, B, ldb, Cm, ldc, M, N, K);
  return hipGetLastError();
}

template <class C>
hipError_t launch_gemm(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s) {
  const int64_t tiles = ((M + C::bm - 1) / C::bm) * ((N + C::bn - 1) / C::bn);
  const bool vec = gemm_f32::vec_ok(A, lda, B, ldb);
  if (vec)
    hipLaunchKernelGGL((gemm_f32_kernel<C, true>), dim3((unsigned)tiles), dim3(256), 0, s, A, lda,
                       B, ldb, Cm, ldc, M, N, K);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<C, false>), dim3((unsigned)tiles), dim3(256), 0, s, A,
                       lda, B, ldb, Cm, ldc, M, N, K);
  return hipGetLastError();
}

// "_rm": the row-major-A tile form; "_w8": eight waves (2 x 4).
constexpr const char* kNames[] = {"m128n128k16", "m256n128k16", "m128n128k32", "m64n64k16",
                                  "m256n256k16_rm_w8_d2", "m256n128k16_rm", "m256n128k16_rm_d2",
                                  "m128n128k16_rm", "m128n128k16_rm_d2", "m128n128k16_rm_d2_x16",
                                  "m256n128k16_rm_d2_x16"};
constexpr int kDefaults[tune::kClasses] = {3, 0, 0, 0};
const bool kRegistered =
    (tune::register_op(tune::kGemmF32, "gemm_f32", 11, kNames, kDefaults), true);

}  // namespace

namespace launch {

hipError_t gemm_f32(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  (void)kRegistered;
  switch (tune::get(tune::kGemmF32, tune::size_class(tune::kGemmF32, M * N * (K ? K : 1)))) {
    case 1: return launch_gemm<GemmCfgF32<256, 128, 16>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 2: return launch_gemm<GemmCfgF32<128, 128, 32>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 3: return launch_gemm<GemmCfgF32<64, 64, 16>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 4:
      return launch_gemm_w<gemm_f32::GemmCfgF32W<256, 256, 16, 2, 4, 2>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 5:
      return launch_gemm_w<gemm_f32::GemmCfgF32W<256, 128, 16, 2, 2>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 6:
      return launch_gemm_w<gemm_f32::GemmCfgF32W<256, 128, 16, 2, 2, 2>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 7:
      return launch_gemm_w<gemm_f32::GemmCfgF32W<128, 128, 16, 2, 2>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 8:
      return launch_gemm_w<gemm_f32::GemmCfgF32W<128, 128, 16, 2, 2, 2>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 9:
      return launch_gemm_w<gemm_f32::GemmCfgF32W<128, 128, 16, 2, 2, 2, true>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    case 10:
      return launch_gemm_w<gemm_f32::GemmCfgF32W<256, 128, 16, 2, 2, 2, true>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
    default: return launch_gemm<GemmCfgF32<128, 128, 16>>(A, lda, B, ldb, Cm, ldc, M, N, K, s);
  }
}

}  // namespace launch
}  // namespace desc
