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
// Pre-pass, two launches: one block per row of A (absmax, then encode)
// beside the column absmax of B as partial maxima over K slices; then an
// LDS-tiled transpose of B that encodes with the column scales and writes
// q^T as [Np][Kp].
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
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef uint8_t u8x4 __attribute__((ext_vector_type(4)));

// Rows of A (M x K, stride lda) -> hi, lo (rows_out x k_out, stride ldh);
// positions beyond M or K are written as zero.  Thread = 4 consecutive k:
// one 16-byte load and two 8-byte stores when the group is whole and
// aligned (vec_in: A and lda allow float4; vec_out: hi, lo and ldh allow
// 8-byte stores), element by element otherwise.
__global__ __launch_bounds__(kBlock) void split_rows_kernel(const float* __restrict__ A,
                                                            int64_t M, int64_t K, int64_t lda,
                                                            uint16_t* __restrict__ hi,
                                                            uint16_t* __restrict__ lo,
                                                            int64_t rows_out, int64_t k_out,
                                                            int64_t ldh, bool vec_in,
                                                            bool vec_out) {
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
    f32x4 v;
    if (vec_in && r < M && c + 4 <= K) {
      v = *(const f32x4*)&a.at(r, c);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (r < M && c + j < K) ? a.at(r, c + j) : 0.f;
    }
    const lowp::Split4 sp = lowp::split_bf16x4(v[0], v[1], v[2], v[3]);
    const u16x4 vh = sp.hi, vl = sp.lo;
    if (vec_out && c + 4 <= k_out) {
      *(u16x4*)&h.at(r, c) = vh;
      *(u16x4*)&l.at(r, c) = vl;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (c + j < k_out) {
          h.at(r, c + j) = vh[j];
          l.at(r, c + j) = vl[j];
        }
    }
  }
}

// Columns of B (K x N, stride ldb) -> hi^T, lo^T (n_out x k_out, stride ldh).
// 64 x 64 tiles of B through LDS; grid (k tiles, n tiles).  Reads run along
// n (thread = 4 columns of one row), writes along k (thread = 4 consecutive
// k of one output row, two 8-byte stores).
__global__ __launch_bounds__(kBlock) void split_cols_t_kernel(const float* __restrict__ B,
                                                              int64_t K, int64_t N, int64_t ldb,
                                                              uint16_t* __restrict__ hi,
                                                              uint16_t* __restrict__ lo,
                                                              int64_t n_out, int64_t k_out,
                                                              int64_t ldh, bool vec_in,
                                                              bool vec_out) {
  __shared__ float lds[64 * 65];
  auto kt = block_x();
  auto nt = block_y();
  auto thread = thread_x<kBlock>();
  auto tile = matrix(lds, 64, 65);
  auto b = matrix(B, K, ldb);
  auto h = matrix(hi, n_out, ldh);
  auto l = matrix(lo, n_out, ldh);
  const idx_t k0 = kt.index() * 64, n0 = nt.index() * 64;
  const int tx = (int)thread.index() % 16, ty = (int)thread.index() / 16;
#pragma unroll
  for (int i = 0; i < 4; ++i) {                 // rows ty + 16 i, columns 4 tx ..
    const idx_t r = ty + 16 * i, c = 4 * tx;
    f32x4 v;
    if (vec_in && k0 + r < K && n0 + c + 4 <= N) {
      v = *(const f32x4*)&b.at(k0 + r, n0 + c);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[j] = (k0 + r < K && n0 + c + j < N) ? b.at(k0 + r, n0 + c + j) : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) tile.at(r, c + j) = v[j];
  }
  sync(thread);
#pragma unroll
  for (int i = 0; i < 4; ++i) {                 // output rows (columns of B) ty + 16 i
    const idx_t c = ty + 16 * i, r = 4 * tx;
    if (n0 + c >= n_out) continue;
    const lowp::Split4 sp = lowp::split_bf16x4(tile.at(r, c), tile.at(r + 1, c),
                                               tile.at(r + 2, c), tile.at(r + 3, c));
    const u16x4 vh = sp.hi, vl = sp.lo;
    if (vec_out && k0 + r + 4 <= k_out) {
      *(u16x4*)&h.at(n0 + c, k0 + r) = vh;
      *(u16x4*)&l.at(n0 + c, k0 + r) = vl;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k0 + r + j < k_out) {
          h.at(n0 + c, k0 + r + j) = vh[j];
          l.at(n0 + c, k0 + r + j) = vl[j];
        }
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

// One block per output row: absmax over the row, then encode, 4 consecutive
// k per thread (16-byte loads and 4-byte stores when whole and aligned).
// Rows of up to kRowCache * 1024 elements stay in registers between the two
// phases, so the row is read once; longer rows are read again to encode.
// q is rows_out x k_out (stride ldq); rows >= M and columns >= K get zero.
constexpr int kRowCache = 8;   // float4 per thread

// Row r of rows_out (the block's row; the caller's grid may hold other work).
__device__ __forceinline__ void quant_row(const float* __restrict__ A, int64_t M, int64_t K,
                                          int64_t lda, uint8_t* __restrict__ q, int64_t rows_out,
                                          int64_t k_out, int64_t ldq, float* __restrict__ scale,
                                          bool vec_in, bool vec_out, idx_t r) {
  __shared__ float red[kBlock / kWave];
  auto thread = thread_x<kBlock>();
  auto a = matrix(A, M, lda);
  auto qr = matrix(q, rows_out, ldq).idx(r);
  auto load4 = [&](idx_t c) {
    f32x4 v;
    if (vec_in && r < M && c + 4 <= K) {
      v = *(const f32x4*)&a.at(r, c);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (r < M && c + j < K) ? a.at(r, c + j) : 0.f;
    }
    return v;
  };
  auto encode = [&](idx_t c, const f32x4& v, float inv) {
    // positions past the row (padding) get code 0
    uint32_t keep = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) keep |= (r < M && c + j < K) ? (0xffu << (8 * j)) : 0u;
    const uint32_t w = lowp::e4m3x4(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv) & keep;
    const u8x4 e = __builtin_bit_cast(u8x4, w);
    if (vec_out && c + 4 <= k_out) {
      *(u8x4*)&qr[c] = e;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (c + j < k_out) qr[c + j] = e[j];
    }
  };
  const bool cached = k_out <= 4 * kBlock * kRowCache && K <= k_out;
  float amax = 0.f;
  f32x4 cache[kRowCache];
  if (cached && vec_in && r < M && K % 4 == 0) {
    // Branch-free: every load reads a valid address (column 0 past the end
    // of the row) and the value is dropped by a select, so the loads are all
    // in flight together instead of one conditional load after another.
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < kRowCache; ++i) {
      const idx_t c = 4 * (thread.index() + kBlock * i);
      const f32x4 v = *(const f32x4*)&a.at(r, c < K ? c : 0);
      cache[i] = c < K ? v : zero;
    }
#pragma unroll
    for (int i = 0; i < kRowCache; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) amax = fmaxf(amax, fabsf(cache[i][j]));
  } else if (cached) {
#pragma unroll
    for (int i = 0; i < kRowCache; ++i) {
      const idx_t c = 4 * (thread.index() + kBlock * i);
      cache[i] = c < K ? load4(c) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 4; ++j) amax = fmaxf(amax, fabsf(cache[i][j]));
    }
  } else {
    for (idx_t c = 4 * thread.index(); c < K; c += 4 * kBlock) {
      const f32x4 v = load4(c);
#pragma unroll
      for (int j = 0; j < 4; ++j) amax = fmaxf(amax, fabsf(v[j]));
    }
  }
  amax = block_max(amax, red);
  const float inv = amax > 0.f ? 448.0f / amax : 1.0f;
  if (cached) {
#pragma unroll
    for (int i = 0; i < kRowCache; ++i) {
      const idx_t c = 4 * (thread.index() + kBlock * i);
      if (c < k_out) encode(c, cache[i], inv);
    }
  } else {
    for (idx_t c = 4 * thread.index(); c < k_out; c += 4 * kBlock) encode(c, load4(c), inv);
  }
  if (thread.index() == 0) array(scale, rows_out)[r] = amax / 448.0f;
}

__global__ __launch_bounds__(kBlock) void quant_rows_kernel(const float* __restrict__ A,
                                                            int64_t M, int64_t K, int64_t lda,
                                                            uint8_t* __restrict__ q,
                                                            int64_t k_out, int64_t ldq,
                                                            float* __restrict__ scale,
                                                            bool vec_in, bool vec_out) {
  auto row = block_x();
  quant_row(A, M, K, lda, q, row.count(), k_out, ldq, scale, vec_in, vec_out, row.index());
}

// Partial column maxima of |B| over K slices: part[s][n] for slice s of
// `rows_per` rows; grid (column blocks of 1024, slices).  Thread = 4
// consecutive columns, read as one 16-byte vector per row when aligned;
// eight rows are loaded before they are combined.
// Column block cb (kBlock * 4 columns) of slice sl (of nslices).
__device__ __forceinline__ void colmax_part(const float* __restrict__ B, int64_t K, int64_t N,
                                            int64_t ldb, int64_t rows_per,
                                            float* __restrict__ part, int64_t ldp, bool vec_in,
                                            idx_t cb, idx_t sl, idx_t nslices) {
  auto thread = thread_x<kBlock>();
  auto b = matrix(B, K, ldb);
  const idx_t n = (cb * kBlock + thread.index()) * 4;
  const idx_t k0 = sl * rows_per;
  const idx_t k1 = k0 + rows_per < K ? k0 + rows_per : K;
  f32x4 m = {0.f, 0.f, 0.f, 0.f};
  if (vec_in && n + 4 <= N) {
#pragma unroll 8
    for (idx_t k = k0; k < k1; ++k) {
      const f32x4 v = *(const f32x4*)&b.at(k, n);
#pragma unroll
      for (int j = 0; j < 4; ++j) m[j] = fmaxf(m[j], fabsf(v[j]));
    }
  } else {
    for (idx_t k = k0; k < k1; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (n + j < N) m[j] = fmaxf(m[j], fabsf(b.at(k, n + j)));
  }
  auto pr = matrix(part, nslices, ldp).idx(sl);
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (n + j < ldp) pr[n + j] = m[j];
}

__global__ __launch_bounds__(kBlock) void colmax_partial_kernel(const float* __restrict__ B,
                                                                int64_t K, int64_t N,
                                                                int64_t ldb, int64_t rows_per,
                                                                float* __restrict__ part,
                                                                int64_t ldp, bool vec_in) {
  auto sl = block_y();
  colmax_part(B, K, N, ldb, rows_per, part, ldp, vec_in, block_x().index(), sl.index(),
              sl.count());
}

// The FP8 GEMM's first pass in one launch: the column-maximum partials of B
// (the first cblocks * nslices blocks, the longer ones, so they start first)
// and the row quantisation of A (one block per padded row), which do not
// depend on each other.
__global__ __launch_bounds__(kBlock) void fp8_prepass_kernel(
    const float* __restrict__ A, int64_t M, int64_t K, int64_t lda, uint8_t* __restrict__ qa,
    int64_t rows_out, int64_t k_out, int64_t ldqa, float* __restrict__ sa, bool a_vec_in,
    const float* __restrict__ B, int64_t N, int64_t ldb, int64_t rows_per,
    float* __restrict__ part, int64_t ldp, bool b_vec_in, int64_t cblocks, int64_t nslices) {
  const idx_t blk = block_x().index(), col_blocks = cblocks * nslices;
  if (blk < col_blocks)
    colmax_part(B, K, N, ldb, rows_per, part, ldp, b_vec_in, blk % cblocks, blk / cblocks,
                nslices);
  else
    quant_row(A, M, K, lda, qa, rows_out, k_out, ldqa, sa, a_vec_in, true, blk - col_blocks);
}

// Encode tiles of kKT k x 64 columns of B with their column scales and
// write them transposed: qt is n_out x k_out (stride ldq), so a tile's
// output rows are kKT bytes: whole 128-byte lines at kKT = 128.  A block
// takes one k tile of one column block; the first block of each column
// block also writes the column scales.  The tile's loads are issued before
// the column maxima are gathered from the slice partials, so the two sets
// of loads are in flight together.  Reads run along n (thread = 4 columns
// of one row), writes along k (thread = 4 consecutive k, one 4-byte store).
template <int kKT>
__global__ __launch_bounds__(kBlock) void quant_cols_t_kernel(const float* __restrict__ B,
                                                              int64_t K, int64_t N, int64_t ldb,
                                                              const float* __restrict__ part,
                                                              int64_t nslices, int64_t ldp,
                                                              uint8_t* __restrict__ qt,
                                                              int64_t n_out, int64_t k_out,
                                                              int64_t ldq,
                                                              float* __restrict__ scale,
                                                              bool vec_in, bool vec_out) {
  static_assert(kKT % 16 == 0 && kKT / 4 <= kBlock && kBlock % (kKT / 4) == 0, "tile shape");
  constexpr int kRows = kKT / 16;               // rows of the tile per thread
  constexpr int kLanesPerRow = kKT / 4;         // threads per output row
  constexpr int kOutRows = kBlock / kLanesPerRow;
  __shared__ uint8_t codes[kKT * 68];
  __shared__ float inv_s[64];
  __shared__ float pmax[4][64];
  auto kt = block_x();
  auto nt = block_y();
  auto thread = thread_x<kBlock>();
  auto tile = matrix(codes, kKT, 68);
  auto b = matrix(B, K, ldb);
  auto pm = matrix(part, nslices, ldp);
  auto out = matrix(qt, n_out, ldq);
  const idx_t n0 = nt.index() * 64, k0 = kt.index() * kKT;
  const int tx = (int)thread.index() % 16, ty = (int)thread.index() / 16;
  f32x4 v[kRows];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {             // rows ty + 16 i, columns 4 tx ..
    const idx_t r = ty + 16 * i, c = 4 * tx;
    if (vec_in && k0 + r < K && n0 + c + 4 <= N) {
      v[i] = *(const f32x4*)&b.at(k0 + r, n0 + c);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        v[i][j] = (k0 + r < K && n0 + c + j < N) ? b.at(k0 + r, n0 + c + j) : 0.f;
    }
  }
  {
    // column maxima of the 64 columns from the slice partials: thread
    // (g, c) takes slices g, g + 4, ... of column c (loads coalesced along
    // the columns, independent, so they are in flight together)
    const int c = (int)thread.index() % 64, g = (int)thread.index() / 64;
    const idx_t n = n0 + c;
    float m = 0.f;
    if (n < N)
#pragma unroll 8
      for (idx_t sl = g; sl < nslices; sl += 4) m = fmaxf(m, pm.at(sl, n));
    pmax[g][c] = m;
  }
  sync(thread);
  if (thread.index() < 64) {
    const int c = (int)thread.index();
    const idx_t n = n0 + c;
    const float m = fmaxf(fmaxf(pmax[0][c], pmax[1][c]), fmaxf(pmax[2][c], pmax[3][c]));
    inv_s[c] = m > 0.f ? 448.0f / m : 1.0f;
    if (kt.index() == 0 && n < n_out) array(scale, n_out)[n] = m / 448.0f;
  }
  sync(thread);
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const idx_t r = ty + 16 * i, c = 4 * tx;
    uint32_t keep = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) keep |= (k0 + r < K && n0 + c + j < N) ? (0xffu << (8 * j)) : 0u;
    const uint32_t w = lowp::e4m3x4(v[i][0] * inv_s[c], v[i][1] * inv_s[c + 1],
                                    v[i][2] * inv_s[c + 2], v[i][3] * inv_s[c + 3]) & keep;
    *(u8x4*)&tile.at(r, c) = __builtin_bit_cast(u8x4, w);
  }
  sync(thread);
  const int ox = (int)thread.index() % kLanesPerRow, oy = (int)thread.index() / kLanesPerRow;
#pragma unroll
  for (int i = 0; i < 64 / kOutRows; ++i) {     // output rows oy + kOutRows i, k = 4 ox ..
    const idx_t c = oy + kOutRows * i, r = 4 * ox;
    if (n0 + c >= n_out) continue;
    u8x4 e;
#pragma unroll
    for (int j = 0; j < 4; ++j) e[j] = tile.at(r + j, c);
    if (vec_out && k0 + r + 4 <= k_out) {
      *(u8x4*)&out.at(n0 + c, k0 + r) = e;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k0 + r + j < k_out) out.at(n0 + c, k0 + r + j) = e[j];
    }
  }
}
// The encode's k tile: 64 up to 8192 tiles of 64 x 64, 128 beyond (whole
// 128-byte output lines; measured at 8192^2: 75 against 90 us; at 4096^2 the
// 64-k tiles keep twice the blocks in flight: 18.5 against 20.7 us).
template <class F>
hipError_t launch_cols_t(int64_t K, int64_t N, hipStream_t s, F&& args) {
  const int64_t t64 = ((K + 63) / 64) * ((N + 63) / 64);
  if (t64 > 8192) {
    args([&](auto... a) {
      hipLaunchKernelGGL(quant_cols_t_kernel<128>,
                         dim3((unsigned)((K + 127) / 128), (unsigned)((N + 63) / 64)),
                         dim3(kBlock), 0, s, a...);
    });
  } else {
    args([&](auto... a) {
      hipLaunchKernelGGL(quant_cols_t_kernel<64>,
                         dim3((unsigned)((K + 63) / 64), (unsigned)((N + 63) / 64)),
                         dim3(kBlock), 0, s, a...);
    });
  }
  return hipGetLastError();
}

int64_t colmax_slices(int64_t K, int64_t N) {
  const int64_t cblocks = (N + 4 * kBlock - 1) / (4 * kBlock);
  int64_t s = 256 / (cblocks > 0 ? cblocks : 1);
  const int64_t kmax = (K + 63) / 64;
  if (s > kmax) s = kmax;
  return s < 1 ? 1 : s;
}

// ------------------------------------------------------------------ GEMM launch
template <class C, bool kBuf>
__global__ __launch_bounds__(C::threads) void gemm_nt_kernel(NtOperands p, int64_t tiles_m,
                                                             int64_t tiles_n) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[C::lds_bytes];
  const idx_t t = gemm_f32::xcd_tile(block_x(), tiles_m, tiles_n);
  gemm_nt::tile<C, kBuf>(p, t / tiles_n, t % tiles_n, lds);
}

// Split-BF16 tiles straight from the FP32 operands (no pre-pass).
template <class C, bool kVec>
__global__ __launch_bounds__(C::threads) void gemm_split_kernel(gemm_nt::F32Operands f,
                                                                float* __restrict__ Cm,
                                                                int64_t ldc, int64_t tiles_m,
                                                                int64_t tiles_n) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[C::lds_bytes];
  const idx_t t = gemm_f32::xcd_tile(block_x(), tiles_m, tiles_n);
  gemm_nt::tile_split<C, kVec>(f, Cm, ldc, t / tiles_n, t % tiles_n, lds);
}

template <class C>
hipError_t launch_split(const gemm_nt::F32Operands& f, float* Cm, int64_t ldc, hipStream_t s) {
  const int64_t tm = (f.M + C::bm - 1) / C::bm, tn = (f.N + C::bn - 1) / C::bn;
  if (gemm_f32::vec_ok(f.A, f.lda, f.A, f.lda) && f.K % 4 == 0)
    hipLaunchKernelGGL((gemm_split_kernel<C, true>), dim3((unsigned)(tm * tn)), dim3(C::threads),
                       0, s, f, Cm, ldc, tm, tn);
  else
    hipLaunchKernelGGL((gemm_split_kernel<C, false>), dim3((unsigned)(tm * tn)),
                       dim3(C::threads), 0, s, f, Cm, ldc, tm, tn);
  return hipGetLastError();
}

// The buffer-range loads need a tile's rows of a plane to span less than
// 2^31 bytes (K up to about 8M FP8 or 4M BF16 values at 256-row tiles).
template <class C>
hipError_t launch_nt(const NtOperands& p, int64_t Mp, int64_t Np, hipStream_t s) {
  const int64_t tm = Mp / C::bm, tn = Np / C::bn;
  const int64_t rows = C::bm > C::bn ? C::bm : C::bn;
  if (rows * p.row_bytes < (int64_t(1) << 31))
    hipLaunchKernelGGL((gemm_nt_kernel<C, true>), dim3((unsigned)(tm * tn)), dim3(C::threads), 0,
                       s, p, tm, tn);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<C, false>), dim3((unsigned)(tm * tn)), dim3(C::threads), 0,
                       s, p, tm, tn);
  return hipGetLastError();
}

struct LowpLayout {
  int64_t Mp, Np, Kp;
  size_t a_plane, b_plane;       // bytes of one operand plane
  size_t off[8];                 // byte offsets of the workspace parts
  size_t total;
};

// bf16x3: Ah, Al, Bh^T, Bl^T.  fp8: qA, qB^T, sA, sB, column partials.
LowpLayout lowp_layout(int mode, int64_t M, int64_t N, int64_t K) {
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

// "_w8": eight waves (2 x 4) share the tile instead of four (2 x 2);
// "_fused": the operands split while they are staged (no pre-pass);
// "_p": fragment reads one group of matrix ops ahead (NtCfg kPipe).
constexpr const char* kNamesBf16[] = {"m128n128k32", "m256n128k32", "m128n256k32",
                                      "m256n256k32_d1", "m256n256k32_w8d1",
                                      "m128n128k32_fused", "m256n256k32_w8d1_fused"};
constexpr const char* kNamesFp8[] = {"m128n128k128", "m128n128k64", "m256n128k128",
                                     "m128n256k128", "m256n128k64", "m256n256k64_w8d1",
                                     "m256n256k128_w8d1", "m256n256k128_w8d1_p", "m128n128k128_p"};
constexpr int kDefaults[tune::kClasses] = {0, 0, 0, 0};
const bool kRegistered =
    (tune::register_op(tune::kGemmBf16x3, "gemm_bf16x3", 7, kNamesBf16, kDefaults),
     tune::register_op(tune::kGemmFp8, "gemm_fp8", 9, kNamesFp8, kDefaults), true);

}  // namespace

namespace launch {

size_t gemm_lowp_workspace(int mode, int64_t M, int64_t N, int64_t K) {
  return lowp_layout(mode, M, N, K).total;
}

bool f4_ok(const void* p, int64_t ld) { return ((uintptr_t)p % 16) == 0 && ld % 4 == 0; }
bool w_ok(const void* p, int64_t ld, int64_t es) {   // 4 elements of es bytes per store
  return ((uintptr_t)p % (4 * es)) == 0 && ld % 4 == 0;
}

hipError_t split_bf16_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint16_t* hi,
                           uint16_t* lo, int64_t ldh, hipStream_t s) {
  hipLaunchKernelGGL(split_rows_kernel, dim3(grid_for(M * ((K + 3) / 4))), dim3(kBlock), 0, s, A,
                     M, K, lda, hi, lo, M, K, ldh, f4_ok(A, lda),
                     w_ok(hi, ldh, 2) && w_ok(lo, ldh, 2));
  return hipGetLastError();
}

hipError_t split_bf16_cols(const float* B, int64_t K, int64_t N, int64_t ldb, uint16_t* hi_t,
                           uint16_t* lo_t, int64_t ldh, hipStream_t s) {
  const dim3 grid((unsigned)((K + 63) / 64), (unsigned)((N + 63) / 64));
  hipLaunchKernelGGL(split_cols_t_kernel, grid, dim3(kBlock), 0, s, B, K, N, ldb, hi_t, lo_t, N,
                     K, ldh, f4_ok(B, ldb), w_ok(hi_t, ldh, 2) && w_ok(lo_t, ldh, 2));
  return hipGetLastError();
}

hipError_t quant_e4m3_rows(const float* A, int64_t M, int64_t K, int64_t lda, uint8_t* q,
                           int64_t ldq, float* scale, hipStream_t s) {
  hipLaunchKernelGGL(quant_rows_kernel, dim3((unsigned)M), dim3(kBlock), 0, s, A, M, K, lda, q, K,
                     ldq, scale, f4_ok(A, lda), w_ok(q, ldq, 1));
  return hipGetLastError();
}

size_t quant_e4m3_cols_workspace(int64_t K, int64_t N) {
  return (size_t)colmax_slices(K, N) * (size_t)(N > 0 ? N : 1) * 4;
}

hipError_t quant_e4m3_cols(const float* B, int64_t K, int64_t N, int64_t ldb, uint8_t* qt,
                           int64_t ldq, float* scale, void* ws, hipStream_t s) {
  const int64_t S = colmax_slices(K, N), rows_per = (K + S - 1) / S;
  float* part = (float*)ws;
  hipLaunchKernelGGL(colmax_partial_kernel,
                     dim3((unsigned)((N + 4 * kBlock - 1) / (4 * kBlock)), (unsigned)S),
                     dim3(kBlock), 0, s, B, K, N, ldb, rows_per, part, N, f4_ok(B, ldb));
  const bool vin = f4_ok(B, ldb), vout = w_ok(qt, ldq, 1);
  launch_cols_t(K, N, s, [&](auto&& go) {
    go(B, K, N, ldb, (const float*)part, S, N, qt, N, K, ldq, scale, vin, vout);
  });
  return hipGetLastError();
}

hipError_t gemm_bf16x3(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws, hipStream_t s) {
  (void)kRegistered;
  const int cfg = tune::get(tune::kGemmBf16x3, tune::size_class(tune::kGemmBf16x3, M * N * K));
  if (cfg >= 5 && K > 0 && lda <= gemm_nt::kSplitMaxLd && ldb <= gemm_nt::kSplitMaxLd) {
    const gemm_nt::F32Operands f{A, lda, B, ldb, M, N, K};
    if (cfg == 6) return launch_split<NtCfg<256, 256, 64, Bf16x3Mode, 1, 2, 4>>(f, Cm, ldc, s);
    return launch_split<NtCfg<128, 128, 64, Bf16x3Mode>>(f, Cm, ldc, s);
  }
  // the pre-pass form (also the fused configurations' path for K = 0 and
  // strides past the split source's limit)
  const LowpLayout L = lowp_layout(1, M, N, K);
  uint8_t* w = (uint8_t*)ws;
  uint16_t *ah = (uint16_t*)(w + L.off[0]), *al = (uint16_t*)(w + L.off[1]);
  uint16_t *bh = (uint16_t*)(w + L.off[2]), *bl = (uint16_t*)(w + L.off[3]);
  hipLaunchKernelGGL(split_rows_kernel, dim3(grid_for(L.Mp * (L.Kp / 4))), dim3(kBlock), 0, s, A,
                     M, K, lda, ah, al, L.Mp, L.Kp, L.Kp, f4_ok(A, lda), true);
  hipLaunchKernelGGL(split_cols_t_kernel, dim3((unsigned)(L.Kp / 64), (unsigned)(L.Np / 64)),
                     dim3(kBlock), 0, s, B, K, N, ldb, bh, bl, L.Np, L.Kp, L.Kp, f4_ok(B, ldb), true);
  NtOperands p{{(const uint8_t*)ah, (const uint8_t*)al},
               {(const uint8_t*)bh, (const uint8_t*)bl},
               L.Kp * 2, Cm, ldc, M, N, nullptr, nullptr};
  switch (cfg) {
    case 1: return launch_nt<NtCfg<256, 128, 64, Bf16x3Mode>>(p, L.Mp, L.Np, s);
    case 2: return launch_nt<NtCfg<128, 256, 64, Bf16x3Mode>>(p, L.Mp, L.Np, s);
    case 3: return launch_nt<NtCfg<256, 256, 64, Bf16x3Mode, 1>>(p, L.Mp, L.Np, s);
    case 4:
    case 6: return launch_nt<NtCfg<256, 256, 64, Bf16x3Mode, 1, 2, 4>>(p, L.Mp, L.Np, s);
    default: return launch_nt<NtCfg<128, 128, 64, Bf16x3Mode>>(p, L.Mp, L.Np, s);
  }
}

hipError_t gemm_fp8(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws, hipStream_t s) {
  (void)kRegistered;
  const LowpLayout L = lowp_layout(2, M, N, K);
  uint8_t* w = (uint8_t*)ws;
  uint8_t *qa = w + L.off[0], *qb = w + L.off[2];
  float *sa = (float*)(w + L.off[4]), *sb = (float*)(w + L.off[5]), *part = (float*)(w + L.off[6]);
  const int64_t S = colmax_slices(K, N), rows_per = (K + S - 1) / S;
  const int64_t cblocks = (L.Np + 4 * kBlock - 1) / (4 * kBlock);
  hipLaunchKernelGGL(fp8_prepass_kernel, dim3((unsigned)(cblocks * S + L.Mp)), dim3(kBlock), 0, s,
                     A, M, K, lda, qa, L.Mp, L.Kp, L.Kp, sa, f4_ok(A, lda), B, N, ldb, rows_per,
                     part, L.Np, f4_ok(B, ldb), cblocks, S);
  const bool vin = f4_ok(B, ldb);
  launch_cols_t(L.Kp, L.Np, s, [&](auto&& go) {
    go(B, K, N, ldb, (const float*)part, S, L.Np, qb, L.Np, L.Kp, L.Kp, sb, vin, true);
  });
  NtOperands p{{qa, nullptr}, {qb, nullptr}, L.Kp, Cm, ldc, M, N, sa, sb};
  switch (tune::get(tune::kGemmFp8, tune::size_class(tune::kGemmFp8, M * N * K))) {
    case 1: return launch_nt<NtCfg<128, 128, 64, Fp8Mode>>(p, L.Mp, L.Np, s);
    case 2: return launch_nt<NtCfg<256, 128, 128, Fp8Mode>>(p, L.Mp, L.Np, s);
    case 3: return launch_nt<NtCfg<128, 256, 128, Fp8Mode>>(p, L.Mp, L.Np, s);
    case 4: return launch_nt<NtCfg<256, 128, 64, Fp8Mode>>(p, L.Mp, L.Np, s);
    case 5: return launch_nt<NtCfg<256, 256, 64, Fp8Mode, 1, 2, 4>>(p, L.Mp, L.Np, s);
    case 6: return launch_nt<NtCfg<256, 256, 128, Fp8Mode, 1, 2, 4>>(p, L.Mp, L.Np, s);
    case 7: return launch_nt<NtCfg<256, 256, 128, Fp8Mode, 1, 2, 4, true>>(p, L.Mp, L.Np, s);
    case 8: return launch_nt<NtCfg<128, 128, 128, Fp8Mode, 2, 2, 2, true>>(p, L.Mp, L.Np, s);
    default: return launch_nt<NtCfg<128, 128, 128, Fp8Mode>>(p, L.Mp, L.Np, s);
  }
}

}  // namespace launch
}  // namespace desc
