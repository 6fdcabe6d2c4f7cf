// gemm_f32.hpp -- the FP32 matrix-core tile routine shared by the plain and
// the grouped GEMM.  See gemm_f32.hip for the scheme.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "layouts.hpp"
#include "mfma.hpp"
#include "view.hpp"

namespace desc {

struct GemmProblemF32 {
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  float* C;
  int64_t ldc;
  int64_t M, N, K;
};

// Block tile BM x BN, K step BK; 256 threads as a 2 x 2 grid of waves.
template <int kBM, int kBN, int kBK>
struct GemmCfgF32 {
  static constexpr int bm = kBM, bn = kBN, bk = kBK;
  static constexpr int wtm = kBM / 2, wtn = kBN / 2;     // wave tile
  static constexpr int fm = wtm / 32, fn = wtn / 32;     // 32 x 32 fragments per wave
  static constexpr int pa = kBM + 4, pb = kBN + 4;       // LDS pitches (words)
  static constexpr int a_vec = kBM * kBK / 4 / 256;      // float4 per thread per step
  static constexpr int b_vec = kBK * kBN / 4 / 256;
  static_assert(fm >= 1 && fn >= 1 && a_vec >= 1 && b_vec >= 1, "tile too small");
  static_assert(kBK % 4 == 0 && kBN % 4 == 0, "16-byte rows");
};

namespace gemm_f32 {

template <class C>
constexpr int lds_floats() { return 2 * C::bk * C::pa + 2 * C::bk * C::pb; }

__host__ __device__ inline bool vec_ok(const float* A, int64_t lda, const float* B, int64_t ldb) {
  return ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && lda % 4 == 0 && ldb % 4 == 0;
}

// Tile order.  Blocks are dispatched round-robin over the 8 XCDs, each with
// its own L2; the linear block id is first mapped so that each XCD receives a
// contiguous run of tile ids, and tile ids are then laid out in groups of 8
// tile rows (column-major inside a group), so the blocks running together on
// one XCD cover a compact patch of C and share their A rows and B columns.
__device__ __forceinline__ idx_t xcd_tile(const Block& b, idx_t tiles_m, idx_t tiles_n) {
  const idx_t T = tiles_m * tiles_n;
  idx_t u = b.index();
  if (T % 8 == 0) u = (u % 8) * (T / 8) + u / 8;
  constexpr idx_t kGroup = 8;
  const idx_t per_group = kGroup * tiles_n;
  const idx_t g = u / per_group;
  const idx_t first_m = g * kGroup;
  const idx_t gsize = tiles_m - first_m < kGroup ? tiles_m - first_m : kGroup;
  const idx_t r = u - g * per_group;
  return (first_m + r % gsize) * tiles_n + r / gsize;
}

// One BM x BN tile of C = A * B.  `lds` holds lds_floats<C>() floats.
template <class C, bool kVec>
__device__ __forceinline__ void tile(const GemmProblemF32& p, idx_t tm, idx_t tn, float* lds) {
  constexpr int BM = C::bm, BN = C::bn, BK = C::bk;
  auto thread = thread_x<256>();
  auto wv = wave_of_block<256>();
  const int lane = (int)lane_of_wave().index();
  const int half = lane / 32, col32 = lane % 32;
  const int wm = (int)wv.index() / 2, wn = (int)wv.index() % 2;
  const idx_t m0 = tm * BM, n0 = tn * BN;

  auto a_lds = matrices(lds, 2, BK, C::pa);                          // [buf][k][m]
  auto b_lds = matrices(lds + 2 * BK * C::pa, 2, BK, C::pb);         // [buf][k][n]
  auto a_g = matrix(p.A, p.M, p.lda);
  auto b_g = matrix(p.B, p.K, p.ldb);

  f32x4 ra[C::a_vec], rb[C::b_vec];

  // A tile rows m0.., columns k0..: float4 q = t + 256 i -> (row q / (BK/4), group q % (BK/4))
  auto load = [&](idx_t k0) {
    const bool a_full = kVec && m0 + BM <= p.M && k0 + BK <= p.K;
    const bool b_full = kVec && n0 + BN <= p.N && k0 + BK <= p.K;
#pragma unroll
    for (int i = 0; i < C::a_vec; ++i) {
      const int q = (int)thread.index() + 256 * i;
      const idx_t r = m0 + q / (BK / 4), c = k0 + 4 * (q % (BK / 4));
      if (a_full) {
        ra[i] = *(const f32x4*)&a_g.at(r, c);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) ra[i][j] = (r < p.M && c + j < p.K) ? a_g.at(r, c + j) : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < C::b_vec; ++i) {
      const int q = (int)thread.index() + 256 * i;
      const idx_t r = k0 + q / (BN / 4), c = n0 + 4 * (q % (BN / 4));
      if (b_full) {
        rb[i] = *(const f32x4*)&b_g.at(r, c);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) rb[i][j] = (r < p.K && c + j < p.N) ? b_g.at(r, c + j) : 0.f;
      }
    }
  };
  auto store = [&](int buf) {
    auto as = a_lds.idx(buf);
    auto bs = b_lds.idx(buf);
#pragma unroll
    for (int i = 0; i < C::a_vec; ++i) {
      const int q = (int)thread.index() + 256 * i;
      const int r = q / (BK / 4), c = 4 * (q % (BK / 4));
#pragma unroll
      for (int j = 0; j < 4; ++j) as.at(c + j, r) = ra[i][j];
    }
#pragma unroll
    for (int i = 0; i < C::b_vec; ++i) {
      const int q = (int)thread.index() + 256 * i;
      const int r = q / (BN / 4), c = 4 * (q % (BN / 4));
      *(f32x4*)&bs.at(r, c) = rb[i];
    }
  };

  mfma::f32x16 acc[C::fm][C::fn];
#pragma unroll
  for (int i = 0; i < C::fm; ++i)
#pragma unroll
    for (int j = 0; j < C::fn; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const idx_t nk = (p.K + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  sync(thread);
  for (idx_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) load((kt + 1) * BK);
    auto as = a_lds.idx(buf);
    auto bs = b_lds.idx(buf);
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk) {
      const int k = 2 * kk + half;
      float a[C::fm], b[C::fn];
#pragma unroll
      for (int i = 0; i < C::fm; ++i) a[i] = as.at(k, wm * C::wtm + i * 32 + col32);
#pragma unroll
      for (int j = 0; j < C::fn; ++j) b[j] = bs.at(k, wn * C::wtn + j * 32 + col32);
#pragma unroll
      for (int i = 0; i < C::fm; ++i)
#pragma unroll
        for (int j = 0; j < C::fn; ++j) acc[i][j] = mfma::f32_32x32x2(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) store(buf ^ 1);
    sync(thread);
  }

  auto c_g = matrix(p.C, p.M, p.ldc);
  if (m0 + BM <= p.M && n0 + BN <= p.N) {       // whole tile inside C: no guards
#pragma unroll
    for (int i = 0; i < C::fm; ++i)
#pragma unroll
      for (int j = 0; j < C::fn; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          c_g.at(m0 + wm * C::wtm + i * 32 + mfma::acc_row(r, lane),
                 n0 + wn * C::wtn + j * 32 + col32) = acc[i][j][r];
  } else {
#pragma unroll
    for (int i = 0; i < C::fm; ++i)
#pragma unroll
      for (int j = 0; j < C::fn; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const idx_t row = m0 + wm * C::wtm + i * 32 + mfma::acc_row(r, lane);
          const idx_t col = n0 + wn * C::wtn + j * 32 + col32;
          if (row < p.M && col < p.N) c_g.at(row, col) = acc[i][j][r];
        }
  }
}

// Second form of the tile, for the plain GEMM: kWM x kWN waves, and A kept
// in LDS as it is in memory, [m][k] with pitch BK + 4, so that it is written
// with 16-byte stores and read with 16-byte loads.  The reduction index is
// assigned to the matrix instruction's two k slots by halves of the stage:
// lanes 0-31 carry k = kk and lanes 32-63 k = BK/2 + kk at step kk, so a
// lane's A values for a stage are contiguous (the same assignment for A and
// B keeps the product exact).  B stays [k][n] with pitch BN + 4.
//
// k16: 16 x 16 x 4 instructions instead of 32 x 32 x 2 (the stage's four k
// quarters on the instruction's four k slots).  Same work per stage and the
// same LDS traffic; the smaller instruction sustains a higher rate on this
// part (measured: 139 against 125 TFLOP/s in a loop of independent
// instructions on every CU).
template <int kBM, int kBN, int kBK, int kWM, int kWN, int kDepth = 1, bool kK16 = false>
struct GemmCfgF32W {
  static constexpr int bm = kBM, bn = kBN, bk = kBK, threads = 64 * kWM * kWN, depth = kDepth;
  static constexpr int wm = kWM, wn = kWN;
  static constexpr bool k16 = kK16;
  static constexpr int frag = kK16 ? 16 : 32;             // fragment edge
  static constexpr int wtm = kBM / kWM, wtn = kBN / kWN;
  static constexpr int fm = wtm / frag, fn = wtn / frag;
  using acc_t = typename std::conditional<kK16, f32x4, mfma::f32x16>::type;
  static constexpr int acc_regs = kK16 ? 4 : 16;
  static constexpr int pa = kBK + 4, pb = kBN + 4;        // LDS pitches (words)
  static constexpr int a_vec = kBM * kBK / 4 / threads;    // float4 per thread per stage
  static constexpr int b_vec = kBK * kBN / 4 / threads;
  static constexpr int lds_floats = 2 * kBM * pa + 2 * kBK * pb;
  static_assert(fm >= 1 && fn >= 1 && a_vec >= 1 && b_vec >= 1, "tile too small");
  static_assert(a_vec * threads * 4 == kBM * kBK && b_vec * threads * 4 == kBK * kBN,
                "stage divides evenly among the threads");
  static_assert(kBK % 8 == 0 && kBN % 4 == 0, "whole 16-byte groups per half stage");
  static_assert(!kK16 || kBK == 16, "16 x 16 x 4 form: a lane's quarter is one 16-byte read");
};

// An interior tile of the row-major form: the whole tile inside C, K a
// multiple of BK, and each operand's span of the tile below 2^31 bytes
// (A's BM rows, B's BN columns over all K), operands 16-byte aligned with
// leading dimensions that are multiples of 4.  Then every stage's loads are
// whole 16-byte groups inside the operands.
template <class C>
__device__ __forceinline__ bool interior_tile(const GemmProblemF32& p, idx_t tm, idx_t tn) {
  constexpr int64_t kSpan = int64_t(1) << 29;   // elements: 2^31 bytes
  return (tm + 1) * C::bm <= p.M && (tn + 1) * C::bn <= p.N && p.K > 0 && p.K % C::bk == 0 &&
         (C::bm - 1) * p.lda + p.K < kSpan && (p.K - 1) * p.ldb + C::bn < kSpan &&
         vec_ok(p.A, p.lda, p.B, p.ldb);
}

// kInterior (interior_tile holds): each lane's positions inside a stage are
// the same in every stage, so its loads are fixed byte offsets in one buffer
// range over the tile's rows of A (or columns of B) for the whole K loop,
// and a stage moves only the scalar offset -- no address arithmetic and no
// bounds handling per load.
template <class C, bool kVec, bool kInterior = false>
__device__ __forceinline__ void tile_rowmajor(const GemmProblemF32& p, idx_t tm, idx_t tn,
                                              float* lds) {
  constexpr int BM = C::bm, BN = C::bn, BK = C::bk, T = C::threads, HK = BK / 2;
  auto thread = thread_x<T>();
  auto wv = wave_of_block<T>();
  const int lane = (int)lane_of_wave().index();
  const int half = lane / 32, col32 = lane % 32;
  const int wm = (int)wv.index() / C::wn, wn = (int)wv.index() % C::wn;
  const idx_t m0 = tm * BM, n0 = tn * BN;

  auto a_lds = matrices(lds, 2, BM, C::pa);                          // [buf][m][k]
  auto b_lds = matrices(lds + 2 * BM * C::pa, 2, BK, C::pb);         // [buf][k][n]
  auto a_g = matrix(p.A, p.M, p.lda);
  auto b_g = matrix(p.B, p.K, p.ldb);

  // Register staging sets: stage j travels through set j % depth.
  struct Regs {
    f32x4 a[C::a_vec], b[C::b_vec];
  };
  Regs R0, R1;
  // kVec (16-byte aligned rows, K and N multiples of 4): every group of four
  // is wholly inside or wholly outside the operand, so it is loaded from a
  // clamped position and zeroed when outside -- no branch per load, which
  // would keep a second set of registers live.  Otherwise single guarded
  // loads.
  // the interior form's ranges and each lane's offsets in them
  const BufferWindow<4> win_a{(uint32_t)p.lda, BM, (int32_t)p.K};
  const BufferWindow<4> win_b{(uint32_t)p.ldb, (int32_t)p.K, BN};
  __amdgpu_buffer_rsrc_t rs_a, rs_b;
  uint32_t off_a[C::a_vec], off_b[C::b_vec];
  if constexpr (kInterior) {
    rs_a = buffer_rsrc(&a_g.at(m0, 0), win_a.bytes());
    rs_b = buffer_rsrc(&b_g.at(0, n0), win_b.bytes());
#pragma unroll
    for (int i = 0; i < C::a_vec; ++i) {
      const int q = (int)thread.index() + T * i;
      off_a[i] = win_a.offset(q / (BK / 4), 4 * (q % (BK / 4)));
    }
#pragma unroll
    for (int i = 0; i < C::b_vec; ++i) {
      const int q = (int)thread.index() + T * i;
      off_b[i] = win_b.offset(q / (BN / 4), 4 * (q % (BN / 4)));
    }
  }
  auto load = [&](idx_t kt, Regs& R) {
    const idx_t k0 = kt * BK;
    if constexpr (kInterior) {
      // stage kt: k0 columns into A's range, k0 rows into B's
      const int sa = (int)win_a.col_valid((int32_t)k0), sb = (int)win_b.row((int32_t)k0);
#pragma unroll
      for (int i = 0; i < C::a_vec; ++i)
        R.a[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs_a, (int)off_a[i],
                                                                                  sa, 0));
#pragma unroll
      for (int i = 0; i < C::b_vec; ++i)
        R.b[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs_b, (int)off_b[i],
                                                                                  sb, 0));
      return;
    }
#pragma unroll
    for (int i = 0; i < C::a_vec; ++i) {
      const int q = (int)thread.index() + T * i;
      const idx_t r = m0 + q / (BK / 4), c = k0 + 4 * (q % (BK / 4));
      if constexpr (kVec) {
        const bool in = r < p.M && c < p.K;
        const f32x4 v = *(const f32x4*)&a_g.at(r < p.M ? r : p.M - 1, c < p.K ? c : p.K - 4);
#pragma unroll
        for (int j = 0; j < 4; ++j) R.a[i][j] = in ? v[j] : 0.f;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) R.a[i][j] = (r < p.M && c + j < p.K) ? a_g.at(r, c + j) : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < C::b_vec; ++i) {
      const int q = (int)thread.index() + T * i;
      const idx_t r = k0 + q / (BN / 4), c = n0 + 4 * (q % (BN / 4));
      if constexpr (kVec) {
        const bool in = r < p.K && c < p.N;
        const f32x4 v = *(const f32x4*)&b_g.at(r < p.K ? r : p.K - 1, c < p.N ? c : p.N - 4);
#pragma unroll
        for (int j = 0; j < 4; ++j) R.b[i][j] = in ? v[j] : 0.f;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) R.b[i][j] = (r < p.K && c + j < p.N) ? b_g.at(r, c + j) : 0.f;
      }
    }
  };
  auto store = [&](const Regs& R, int buf) {
    auto as = a_lds.idx(buf);
    auto bs = b_lds.idx(buf);
#pragma unroll
    for (int i = 0; i < C::a_vec; ++i) {
      const int q = (int)thread.index() + T * i;
      *(f32x4*)&as.at(layout::gemm_store_row<BK>(q), layout::gemm_store_word<BK>(q)) = R.a[i];
    }
#pragma unroll
    for (int i = 0; i < C::b_vec; ++i) {
      const int q = (int)thread.index() + T * i;
      *(f32x4*)&bs.at(layout::gemm_store_row<BN>(q), layout::gemm_store_word<BN>(q)) = R.b[i];
    }
  };

  typename C::acc_t acc[C::fm][C::fn];
#pragma unroll
  for (int i = 0; i < C::fm; ++i)
#pragma unroll
    for (int j = 0; j < C::fn; ++j)
#pragma unroll
      for (int r = 0; r < C::acc_regs; ++r) acc[i][j][r] = 0.f;

  // matrix ops of the stage in LDS buffer `buf`
  auto compute = [&](int buf) {
    auto as = a_lds.idx(buf);
    auto bs = b_lds.idx(buf);
    if constexpr (C::k16) {
      const int quarter = lane / 16, c16 = lane % 16;
      f32x4 a[C::fm];
#pragma unroll
      for (int i = 0; i < C::fm; ++i)
        a[i] = *(const f32x4*)&as.at(layout::gemm16_a_frag_row<C::wtm>(wm, i, c16),
                                      layout::gemm16_frag_k<BK>(quarter));
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        float b[C::fn];
#pragma unroll
        for (int j = 0; j < C::fn; ++j)
          b[j] = bs.at(layout::gemm16_frag_k<BK>(quarter) + kk,
                       layout::gemm16_b_frag_word<C::wtn>(wn, j, c16));
#pragma unroll
        for (int i = 0; i < C::fm; ++i)
#pragma unroll
          for (int j = 0; j < C::fn; ++j) acc[i][j] = mfma::f32_16x16x4(a[i][kk], b[j], acc[i][j]);
      }
    } else {
#pragma unroll
    for (int k4 = 0; k4 < HK; k4 += 4) {
      // this lane's four k values of the step group: k = half * HK + k4 + 0..3
      f32x4 a[C::fm];
#pragma unroll
      for (int i = 0; i < C::fm; ++i)
        a[i] = *(const f32x4*)&as.at(layout::gemm_a_frag_row<C::wtm>(wm, i, col32),
                                      layout::gemm_frag_k<BK>(half, k4));
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        float b[C::fn];
#pragma unroll
        for (int j = 0; j < C::fn; ++j)
          b[j] = bs.at(layout::gemm_frag_k<BK>(half, k4) + kk,
                       layout::gemm_b_frag_word<C::wtn>(wn, j, col32));
#pragma unroll
        for (int i = 0; i < C::fm; ++i)
#pragma unroll
          for (int j = 0; j < C::fn; ++j) acc[i][j] = mfma::f32_32x32x2(a[i][kk], b[j], acc[i][j]);
      }
    }
    }
  };

  const idx_t nk = (p.K + BK - 1) / BK;
  if constexpr (C::depth == 1) {
    // stage kt+1's loads are issued before stage kt's matrix ops
    if (nk > 0) {
      load(0, R0);
      store(R0, 0);
    }
    sync(thread);
    for (idx_t kt = 0; kt < nk; ++kt) {
      const int buf = (int)(kt & 1);
      if (kt + 1 < nk) load(kt + 1, R0);
      compute(buf);
      if (kt + 1 < nk) store(R0, buf ^ 1);
      sync(thread);
    }
  } else {
    // two stages ahead: iteration kt issues stage kt+2's loads, computes
    // stage kt and writes stage kt+1 (loaded one iteration earlier); pairs
    // of iterations name their register sets statically
    if (nk > 0) {
      load(0, R0);
      store(R0, 0);
    }
    if (nk > 1) load(1, R1);
    sync(thread);
    idx_t kt = 0;
    for (; kt + 3 < nk; kt += 2) {
      load(kt + 2, R0);
      compute(0);
      store(R1, 1);
      sync(thread);
      load(kt + 3, R1);
      compute(1);
      store(R0, 0);
      sync(thread);
    }
    // at most three stages left, kt even
    if (kt < nk) {
      if (kt + 2 < nk) load(kt + 2, R0);
      compute(0);
      if (kt + 1 < nk) store(R1, 1);
      sync(thread);
    }
    if (kt + 1 < nk) {
      compute(1);
      if (kt + 2 < nk) store(R0, 0);
      sync(thread);
    }
    if (kt + 2 < nk) {
      compute(0);
      sync(thread);
    }
  }

  // The wave's 32 x 32 fragments of C: register r of the lane holds row
  // mfma::acc_row(r, lane) = 8 (r / 4) + 4 half + r % 4 and column col32 of
  // its fragment (the row written out in 64-bit arithmetic, so the compiler
  // folds the constant parts into the store offsets).
  auto c_g = matrix(p.C, p.M, p.ldc);
  // row and column of accumulator register r of fragment (i, j)
  auto acc_row = [&](int i, int r) -> idx_t {
    if constexpr (C::k16) return m0 + wm * C::wtm + i * 16 + 4 * (lane / 16) + r;
    else return m0 + wm * C::wtm + i * 32 + 8 * (r / 4) + 4 * half + r % 4;
  };
  auto acc_col = [&](int j) -> idx_t {
    if constexpr (C::k16) return n0 + wn * C::wtn + j * 16 + lane % 16;
    else return n0 + wn * C::wtn + j * 32 + col32;
  };
  if (m0 + BM <= p.M && n0 + BN <= p.N) {
#pragma unroll
    for (int i = 0; i < C::fm; ++i)
#pragma unroll
      for (int j = 0; j < C::fn; ++j)
#pragma unroll
        for (int r = 0; r < C::acc_regs; ++r) c_g.at(acc_row(i, r), acc_col(j)) = acc[i][j][r];
  } else {
#pragma unroll
    for (int i = 0; i < C::fm; ++i)
#pragma unroll
      for (int j = 0; j < C::fn; ++j)
#pragma unroll
        for (int r = 0; r < C::acc_regs; ++r) {
          const idx_t row = acc_row(i, r), col = acc_col(j);
          if (row < p.M && col < p.N) c_g.at(row, col) = acc[i][j][r];
        }
  }
}

}  // namespace gemm_f32
}  // namespace desc
