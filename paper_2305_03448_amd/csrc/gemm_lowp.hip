// gemm_lowp.hip -- the precision forms of C = A * B: three-product split
// bfloat16 with FP32 accumulation, and e4m3 with per-row / per-column
// absmax scaling.  Both prepare their operands in the workspace and then run
// the NT matrix-core tile of gemm_nt.hpp.
//
// BF16x3.  a = hi + lo with hi = bf16(a), lo = bf16(a - hi) (a - hi is exact
// in FP32), likewise for b; C ~ Ah*Bh + Ah*Bl + Al*Bh (the Al*Bl term is
// below FP32 resolution).  Pre-pass: A -> Ah, Al as [Mp][Kp] bf16 (an
// element-wise pass), B -> Bh^T, Bl^T as [Np][Kp] bf16 (an LDS-tiled
// transpose, split on the way).
//
// FP8.  alpha_i = max_k |a_ik|; q_ik = e4m3(a_ik * (448 / alpha_i)) with one
// FP32 division and one FP32 multiply; s_i = alpha_i / 448 (an all-zero row
// uses 448/alpha = 1 and s = 0).  Columns of B likewise with beta_j.  Then
// C_ij = s_i * t_j * sum_k q_ik q_kj, the sum on the matrix cores in FP32.
// Pre-pass: one block per row of A (absmax, then encode); column absmax of
// B as partial maxima over K slices; an LDS-tiled transpose of B that
// encodes with the column scales and writes q^T as [Np][Kp].
//
// Padding: Mp, Np are multiples of 256 and Kp a multiple of 128 elements;
// the pre-pass writes zeros there, so the GEMM main loop has no guards.
#include "common.hpp"
#include "gemm_nt.hpp"
#include "launch.hpp"
#include "lowp.hpp"
#include "tuning.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

constexpr int kBlock = 256;
constexpr int64_t kPadMN = 256, kPadK = 128;

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ split
// Rows of A (M x K, stride lda) -> hi, lo (rows_out x k_out, stride ldh);
// positions beyond M or K are written as zero.  Thread = 4 consecutive k.
__global__ __launch_bounds__(kBlock) void split_rows_kernel(const float* __restrict__ A,
                                                            int64_t M, int64_t K, int64_t lda,
                                                            uint16_t* __restrict__ hi,
                                                            uint16_t* __restrict__ lo,
                                                            int64_t rows_out, int64_t k_out,
                                                            int64_t ldh) {
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  auto a = matrix(A, M, lda);
  auto h = matrix(hi, rows_out, ldh);
  auto l = matrix(lo, rows_out, ldh);
  const int64_t groups = (k_out + 3) / 4;
  const int64_t total = rows_out * groups;
  for (idx_t g = block.index() * kBlock + thread.index(); g < total;
       g += block.count() * kBlock) {
    const idx_t r = g / groups, c = 4 * (g % groups);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (c + j >= k_out) break;
      const float v = (r < M && c + j < K) ? a.at(r, c + j) : 0.f;
      const lowp::Split s = lowp::split_bf16(v);
      h.at(r, c + j) = s.hi;
      l.at(r, c + j) = s.lo;
    }
  }
}

// Columns of B (K x N, stride ldb) -> hi^T, lo^T (n_out x k_out, stride ldh).
// 64 x 64 tiles of B through LDS; grid (k tiles, n tiles).
__global__ __launch_bounds__(kBlock) void split_cols_t_kernel(const float* __restrict__ B,
                                                              int64_t K, int64_t N, int64_t ldb,
                                                              uint16_t* __restrict__ hi,
                                                              uint16_t* __restrict__ lo,
                                                              int64_t n_out, int64_t k_out,
                                                              int64_t ldh) {
  __shared__ float lds[64 * 65];
  auto kt = block_x();
  auto nt = block_y();
  auto thread = thread_x<kBlock>();
  auto tile = matrix(lds, 64, 65);
  auto b = matrix(B, K, ldb);
  auto h = matrix(hi, n_out, ldh);
  auto l = matrix(lo, n_out, ldh);
  const idx_t k0 = kt.index() * 64, n0 = nt.index() * 64;
  for (idx_t e = thread.index(); e < 64 * 64; e += kBlock) {   // read along n
    const idx_t r = e / 64, c = e % 64;
    tile.at(r, c) = (k0 + r < K && n0 + c < N) ? b.at(k0 + r, n0 + c) : 0.f;
  }
  sync(thread);
  for (idx_t e = thread.index(); e < 64 * 64; e += kBlock) {   // write along k
    const idx_t c = e / 64, r = e % 64;
    if (n0 + c < n_out && k0 + r < k_out) {
      const lowp::Split s = lowp::split_bf16(tile.at(r, c));
      h.at(n0 + c, k0 + r) = s.hi;
      l.at(n0 + c, k0 + r) = s.lo;
    }
  }
}

// ------------------------------------------------------------------ e4m3
__device__ __forceinline__ float block_max(float v, float* red) {
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v = fmaxf(v, __shfl_xor(v, s, 64));
  if (lane_of_wave().index() == 0) red[wv.index()] = v;
  sync(thread);
  float m = red[0];
#pragma unroll
  for (int w = 1; w < kBlock / kWave; ++w) m = fmaxf(m, red[w]);
  return m;
}

// One block per output row: absmax over the row, then encode.
// q is rows_out x k_out (stride ldq); rows >= M and columns >= K get zero.
__global__ __launch_bounds__(kBlock) void quant_rows_kernel(const float* __restrict__ A,
                                                            int64_t M, int64_t K, int64_t lda,
                                                            uint8_t* __restrict__ q,
                                                            int64_t k_out, int64_t ldq,
                                                            float* __restrict__ scale) {
  __shared__ float red[kBlock / kWave];
  auto row = block_x();
  auto thread = thread_x<kBlock>();
  const idx_t r = row.index();
  auto a = matrix(A, M, lda);
  auto qr = matrix(q, row.count(), ldq).idx(r);
  float amax = 0.f;
  if (r < M)
    for (idx_t k = thread.index(); k < K; k += kBlock) amax = fmaxf(amax, fabsf(a.at(r, k)));
  amax = block_max(amax, red);
  const float inv = amax > 0.f ? 448.0f / amax : 1.0f;
  for (idx_t k = thread.index(); k < k_out; k += kBlock)
    qr[k] = (r < M && k < K) ? lowp::e4m3_rne_sat(a.at(r, k) * inv) : (uint8_t)0;
  if (thread.index() == 0) array(scale, row.count())[r] = amax / 448.0f;
}

// Partial column maxima of |B| over K slices: part[s][n] for slice s of
// `rows_per` rows; grid (column blocks of 256, slices).
__global__ __launch_bounds__(kBlock) void colmax_partial_kernel(const float* __restrict__ B,
                                                                int64_t K, int64_t N,
                                                                int64_t ldb, int64_t rows_per,
                                                                float* __restrict__ part,
                                                                int64_t ldp) {
  auto cb = block_x();
  auto sl = block_y();
  auto thread = thread_x<kBlock>();
  auto b = matrix(B, K, ldb);
  const idx_t n = cb.index() * kBlock + thread.index();
  const idx_t k0 = sl.index() * rows_per;
  const idx_t k1 = k0 + rows_per < K ? k0 + rows_per : K;
  float m = 0.f;
  if (n < N)
    for (idx_t k = k0; k < k1; ++k) m = fmaxf(m, fabsf(b.at(k, n)));
  if (n < ldp) matrix(part, sl.count(), ldp).at(sl.index(), n) = m;
}

// Encode 64 x 64 tiles of B with their column scales and write them
// transposed: qt is n_out x k_out (stride ldq).  The first k tile of each
// column block also writes the column scales.
__global__ __launch_bounds__(kBlock) void quant_cols_t_kernel(const float* __restrict__ B,
                                                              int64_t K, int64_t N, int64_t ldb,
                                                              const float* __restrict__ part,
                                                              int64_t nslices, int64_t ldp,
                                                              uint8_t* __restrict__ qt,
                                                              int64_t n_out, int64_t k_out,
                                                              int64_t ldq,
                                                              float* __restrict__ scale) {
  __shared__ uint8_t codes[64 * 68];
  __shared__ float inv_s[64];
  auto kt = block_x();
  auto nt = block_y();
  auto thread = thread_x<kBlock>();
  auto tile = matrix(codes, 64, 68);
  auto b = matrix(B, K, ldb);
  auto pm = matrix(part, nslices, ldp);
  auto out = matrix(qt, n_out, ldq);
  const idx_t k0 = kt.index() * 64, n0 = nt.index() * 64;
  if (thread.index() < 64) {
    const idx_t n = n0 + thread.index();
    float m = 0.f;
    if (n < N)
      for (idx_t s = 0; s < nslices; ++s) m = fmaxf(m, pm.at(s, n));
    inv_s[thread.index()] = m > 0.f ? 448.0f / m : 1.0f;
    if (kt.index() == 0 && n < n_out) array(scale, n_out)[n] = m / 448.0f;
  }
  sync(thread);
  for (idx_t e = thread.index(); e < 64 * 64; e += kBlock) {   // read along n
    const idx_t r = e / 64, c = e % 64;
    tile.at(r, c) = (k0 + r < K && n0 + c < N)
                        ? lowp::e4m3_rne_sat(b.at(k0 + r, n0 + c) * inv_s[c])
                        : (uint8_t)0;
  }
  sync(thread);
  for (idx_t e = thread.index(); e < 64 * 64; e += kBlock) {   // write along k
    const idx_t c = e / 64, r = e % 64;
    if (n0 + c < n_out && k0 + r < k_out) out.at(n0 + c, k0 + r) = tile.at(r, c);
  }
}

int64_t colmax_slices(int64_t K, int64_t N) {
  const int64_t cblocks = (N + kBlock - 1) / kBlock;
  int64_t s = 1024 / (cblocks > 0 ? cblocks : 1);
  const int64_t kmax = (K + 63) / 64;
  if (s > kmax) s = kmax;
  return s < 1 ? 1 : s;
}

// ------------------------------------------------------------------ GEMM launch
template <class C>
__global__ __launch_bounds__(256) void gemm_nt_kernel(NtOperands p, int64_t tiles_m,
                                                      int64_t tiles_n) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[C::lds_bytes];
  const idx_t t = gemm_f32::xcd_tile(block_x(), tiles_m, tiles_n);
  gemm_nt::tile<C>(p, t / tiles_n, t % tiles_n, lds);
}

template <class C>
hipError_t launch_nt(const NtOperands& p, int64_t Mp, int64_t Np, hipStream_t s) {
  const int64_t tm = Mp / C::bm, tn = Np / C::bn;
  hipLaunchKernelGGL((gemm_nt_kernel<C>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, p, tm, tn);
  return hipGetLastError();
}

struct LowpLayout {
  int64_t Mp, Np, Kp;
  size_t a_plane, b_plane;       // bytes of one operand plane
  size_t off[8];                 // byte offsets of the workspace parts
  size_t total;
};

// bf16x3: Ah, Al, Bh^T, Bl^T.  fp8: qA, qB^T, sA, sB, column partials.
LowpLayout layout(int mode, int64_t M, int64_t N, int64_t K) {
  LowpLayout L{};
  L.Mp = round_up(M > 0 ? M : 1, kPadMN);
  L.Np = round_up(N > 0 ? N : 1, kPadMN);
  L.Kp = round_up(K > 0 ? K : 1, kPadK);
  const size_t es = mode == 1 ? 2 : 1;
  L.a_plane = align256((size_t)L.Mp * L.Kp * es);
  L.b_plane = align256((size_t)L.Np * L.Kp * es);
  size_t o = 0;
  if (mode == 1) {
    L.off[0] = o; o += L.a_plane;
    L.off[1] = o; o += L.a_plane;
    L.off[2] = o; o += L.b_plane;
    L.off[3] = o; o += L.b_plane;
  } else {
    L.off[0] = o; o += L.a_plane;
    L.off[2] = o; o += L.b_plane;
    L.off[4] = o; o += align256((size_t)L.Mp * 4);
    L.off[5] = o; o += align256((size_t)L.Np * 4);
    L.off[6] = o; o += align256((size_t)colmax_slices(K, N) * L.Np * 4);
  }
  L.total = o;
  return L;
}

unsigned grid_for(int64_t items) {
  int64_t g = (items + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  return (unsigned)(g < 1 ? 1 : g);
}

constexpr const char* kNamesBf16[] = {"m128n128k32", "m256n128k32", "m128n256k32",
                                      "m256n256k32_d1"};
constexpr const char* kNamesFp8[] = {"m128n128k128", "m128n128k64", "m256n128k128",
                                     "m128n256k128", "m256n128k64"};
constexpr int kDefaults[tune::kClasses] = {0, 0, 0, 0};
const bool kRegistered =
    (tune::register_op(tune::kGemmBf16x3, "gemm_bf16x3", 4, kNamesBf16, kDefaults),
     tune::register_op(tune::kGemmFp8, "gemm_fp8", 5, kNamesFp8, kDefaults), true);

}  // namespace

namespace launch {

size_t gemm_lowp_workspace(int mode, int64_t M, int64_t N, int64_t K) {
  return layout(mode, M, N, K).total;
}

hipError_t split_bf16_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint16_t* hi,
                           uint16_t* lo, int64_t ldh, hipStream_t s) {
  hipLaunchKernelGGL(split_rows_kernel, dim3(grid_for(M * ((K + 3) / 4))), dim3(kBlock), 0, s, A,
                     M, K, lda, hi, lo, M, K, ldh);
  return hipGetLastError();
}

hipError_t split_bf16_cols(const float* B, int64_t K, int64_t N, int64_t ldb, uint16_t* hi_t,
                           uint16_t* lo_t, int64_t ldh, hipStream_t s) {
  const dim3 grid((unsigned)((K + 63) / 64), (unsigned)((N + 63) / 64));
  hipLaunchKernelGGL(split_cols_t_kernel, grid, dim3(kBlock), 0, s, B, K, N, ldb, hi_t, lo_t, N,
                     K, ldh);
  return hipGetLastError();
}

hipError_t quant_e4m3_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint8_t* q,
                           int64_t ldq, float* scale, hipStream_t s) {
  hipLaunchKernelGGL(quant_rows_kernel, dim3((unsigned)M), dim3(kBlock), 0, s, A, M, K, lda, q, K,
                     ldq, scale);
  return hipGetLastError();
}

size_t quant_e4m3_cols_workspace(int64_t K, int64_t N) {
  return (size_t)colmax_slices(K, N) * (size_t)(N > 0 ? N : 1) * 4;
}

hipError_t quant_e4m3_cols(const float* B, int64_t K, int64_t N, int64_t ldb, uint8_t* qt,
                           int64_t ldq, float* scale, void* ws, hipStream_t s) {
  const int64_t S = colmax_slices(K, N), rows_per = (K + S - 1) / S;
  float* part = (float*)ws;
  hipLaunchKernelGGL(colmax_partial_kernel, dim3((unsigned)((N + kBlock - 1) / kBlock), (unsigned)S),
                     dim3(kBlock), 0, s, B, K, N, ldb, rows_per, part, N);
  hipLaunchKernelGGL(quant_cols_t_kernel, dim3((unsigned)((K + 63) / 64), (unsigned)((N + 63) / 64)),
                     dim3(kBlock), 0, s, B, K, N, ldb, part, S, N, qt, N, K, ldq, scale);
  return hipGetLastError();
}

hipError_t gemm_bf16x3(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws, hipStream_t s) {
  (void)kRegistered;
  const LowpLayout L = layout(1, M, N, K);
  uint8_t* w = (uint8_t*)ws;
  uint16_t *ah = (uint16_t*)(w + L.off[0]), *al = (uint16_t*)(w + L.off[1]);
  uint16_t *bh = (uint16_t*)(w + L.off[2]), *bl = (uint16_t*)(w + L.off[3]);
  hipLaunchKernelGGL(split_rows_kernel, dim3(grid_for(L.Mp * (L.Kp / 4))), dim3(kBlock), 0, s, A,
                     M, K, lda, ah, al, L.Mp, L.Kp, L.Kp);
  hipLaunchKernelGGL(split_cols_t_kernel, dim3((unsigned)(L.Kp / 64), (unsigned)(L.Np / 64)),
                     dim3(kBlock), 0, s, B, K, N, ldb, bh, bl, L.Np, L.Kp, L.Kp);
  NtOperands p{{(const uint8_t*)ah, (const uint8_t*)al},
               {(const uint8_t*)bh, (const uint8_t*)bl},
               L.Kp * 2, Cm, ldc, M, N, nullptr, nullptr};
  switch (tune::get(tune::kGemmBf16x3, tune::size_class(tune::kGemmBf16x3, M * N * K))) {
    case 1: return launch_nt<NtCfg<256, 128, 64, Bf16x3Mode>>(p, L.Mp, L.Np, s);
    case 2: return launch_nt<NtCfg<128, 256, 64, Bf16x3Mode>>(p, L.Mp, L.Np, s);
    case 3: return launch_nt<NtCfg<256, 256, 64, Bf16x3Mode, 1>>(p, L.Mp, L.Np, s);
    default: return launch_nt<NtCfg<128, 128, 64, Bf16x3Mode>>(p, L.Mp, L.Np, s);
  }
}

hipError_t gemm_fp8(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws, hipStream_t s) {
  (void)kRegistered;
  const LowpLayout L = layout(2, M, N, K);
  uint8_t* w = (uint8_t*)ws;
  uint8_t *qa = w + L.off[0], *qb = w + L.off[2];
  float *sa = (float*)(w + L.off[4]), *sb = (float*)(w + L.off[5]), *part = (float*)(w + L.off[6]);
  hipLaunchKernelGGL(quant_rows_kernel, dim3((unsigned)L.Mp), dim3(kBlock), 0, s, A, M, K, lda, qa,
                     L.Kp, L.Kp, sa);
  const int64_t S = colmax_slices(K, N), rows_per = (K + S - 1) / S;
  hipLaunchKernelGGL(colmax_partial_kernel, dim3((unsigned)(L.Np / kBlock + (L.Np % kBlock != 0)),
                                                 (unsigned)S),
                     dim3(kBlock), 0, s, B, K, N, ldb, rows_per, part, L.Np);
  hipLaunchKernelGGL(quant_cols_t_kernel, dim3((unsigned)(L.Kp / 64), (unsigned)(L.Np / 64)),
                     dim3(kBlock), 0, s, B, K, N, ldb, part, S, L.Np, qb, L.Np, L.Kp, L.Kp, sb);
  NtOperands p{{qa, nullptr}, {qb, nullptr}, L.Kp, Cm, ldc, M, N, sa, sb};
  switch (tune::get(tune::kGemmFp8, tune::size_class(tune::kGemmFp8, M * N * K))) {
    case 1: return launch_nt<NtCfg<128, 128, 64, Fp8Mode>>(p, L.Mp, L.Np, s);
    case 2: return launch_nt<NtCfg<256, 128, 128, Fp8Mode>>(p, L.Mp, L.Np, s);
    case 3: return launch_nt<NtCfg<128, 256, 128, Fp8Mode>>(p, L.Mp, L.Np, s);
    case 4: return launch_nt<NtCfg<256, 128, 64, Fp8Mode>>(p, L.Mp, L.Np, s);
    default: return launch_nt<NtCfg<128, 128, 128, Fp8Mode>>(p, L.Mp, L.Np, s);
  }
}

}  // namespace launch
}  // namespace desc
