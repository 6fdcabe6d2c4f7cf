// gemm_nt.hpp -- matrix-core tile routine for the low-precision GEMM modes.
//
// Both operands arrive K-contiguous ("NT"): A as [Mp][Kp] and B transposed as
// [Np][Kp], padded with zeros to whole tiles by the operand pre-pass, so the
// main loop needs no guards.  Rows are byte strings here: a stage copies BKB
// bytes of K per row of each operand plane into LDS as 16-byte chunks,
// double buffered, one barrier per stage.  The LDS rows are unpadded and the
// chunk index is XOR-swizzled with the row (xor_swizzle), so both the
// coalesced staging writes (consecutive lanes along a row) and the fragment
// reads (one chunk of 16 consecutive rows) hit distinct banks.
//
// Modes:
//   Bf16x3 -- planes {hi, lo}; per 16-wide K step three 32x32x16 bf16
//             products lo*hi, hi*lo, hi*hi accumulate into one FP32 tile.
//   Fp8    -- one plane of e4m3 codes; one 32x32x64 fp8 product per 64-wide
//             K step; the epilogue multiplies by the row scale of A and the
//             column scale of B.
#pragma once
#include "common.hpp"
#include "gemm_f32.hpp"
#include "lowp.hpp"
#include "mfma.hpp"
#include "layouts.hpp"
#include "view.hpp"

namespace desc {

struct NtOperands {
  const uint8_t* a[2];    // A planes, [Mp][row_bytes]
  const uint8_t* b[2];    // B^T planes, [Np][row_bytes]
  int64_t row_bytes;      // Kp * element size
  float* C;
  int64_t ldc;
  int64_t M, N;           // valid part of C
  const float* sa;        // Fp8: row scales of A (Mp), column scales of B (Np)
  const float* sb;
};

struct Bf16x3Mode {
  static constexpr int planes = 2;
  static constexpr int step_bytes = 32;   // bytes of a row one instruction consumes (16 x bf16)
  static constexpr int lane_bytes = 16;   // bytes per lane per operand
  static constexpr bool scaled = false;
};
struct Fp8Mode {
  static constexpr int planes = 1;
  static constexpr int step_bytes = 64;   // 64 x e4m3
  static constexpr int lane_bytes = 32;
  static constexpr bool scaled = true;
};

// kDepth: stages in flight in registers (1: the next stage's loads are
// issued before the current stage's matrix ops; 2: two stages ahead, which
// needs a second register staging set).  kWM x kWN waves share the tile,
// each computing a (kBM / kWM) x (kBN / kWN) part of it.  kPipe (scaled
// mode): each group of matrix ops has the LDS reads of the next group
// issued ahead of it.
template <int kBM, int kBN, int kBKB, class Mode, int kDepth = 2, int kWM = 2, int kWN = 2,
          bool kPipe = false>
struct NtCfg {
  using mode = Mode;
  static constexpr int bm = kBM, bn = kBN, bkb = kBKB, depth = kDepth;
  static constexpr bool pipe = kPipe;
  static_assert(!kPipe || (Mode::scaled && Mode::lane_bytes == 32), "pipelined form: scaled mode");
  static constexpr int wm = kWM, wn = kWN, threads = 64 * kWM * kWN;
  static constexpr int wtm = kBM / kWM, wtn = kBN / kWN;
  static constexpr int fm = wtm / 32, fn = wtn / 32;
  static constexpr int chunks = kBKB / 16;                 // 16-byte chunks per row
  static constexpr int rows_per_256 = 256 / kBKB;          // rows sharing one bank period
  static constexpr int pitch = kBKB;
  static constexpr int steps = kBKB / Mode::step_bytes;
  static constexpr int a_chunks = kBM * kBKB / 16 / threads;   // 16-byte chunks per thread per plane
  static constexpr int b_chunks = kBN * kBKB / 16 / threads;
  static constexpr int plane_bytes = (kBM + kBN) * pitch;
  static constexpr int stage_bytes = Mode::planes * plane_bytes;
  static constexpr int lds_bytes = 2 * stage_bytes;
  static_assert(steps >= 1 && kBKB % Mode::step_bytes == 0, "stage holds whole steps");
  static_assert(a_chunks >= 1 && b_chunks >= 1, "tile too small for the threads");
  static_assert(a_chunks * threads * 16 == kBM * kBKB && b_chunks * threads * 16 == kBN * kBKB,
                "stage divides evenly among the threads");
  static_assert(fm >= 1 && fn >= 1, "wave tile holds whole 32 x 32 fragments");
};

namespace gemm_nt {

template <int kBytes>
struct Frag;
template <>
struct Frag<16> {
  u32x4 v;
  __device__ __forceinline__ mfma::bf16x8 bf16() const {
    return __builtin_bit_cast(mfma::bf16x8, v);
  }
};
template <>
struct Frag<32> {
  u32x4 v0, v1;
  __device__ __forceinline__ mfma::i32x8 i8() const {
    mfma::i32x8 r;
    r[0] = v0[0]; r[1] = v0[1]; r[2] = v0[2]; r[3] = v0[3];
    r[4] = v1[0]; r[5] = v1[1]; r[6] = v1[2]; r[7] = v1[3];
    return r;
  }
};

// Stage sources.  A source fills the LDS buffer of one stage -- per plane,
// BM rows of A then BN rows of B^T, BKB bytes of K each as 16-byte chunks --
// in two steps: load(kt, R) issues the global loads of stage kt into
// registers, store(R, plane) writes them to the buffer whose plane pl is
// plane(pl).  stages() is the number of stages of the K loop.
//
// PlaneSource: padded planes prepared by an operand pre-pass (no guards).
// kBuf (a tile's rows of each plane span less than 2^31 bytes): the loads go
// through one buffer range per plane over the tile's rows, at per-lane byte
// offsets that are the same in every stage, the stage moving only the
// scalar offset.
template <class C, bool kBuf = false>
struct PlaneSource {
  using Mode = typename C::mode;
  static constexpr int P = Mode::planes, T = C::threads, CPR = C::chunks;
  struct Regs {
    u32x4 a[P][C::a_chunks], b[P][C::b_chunks];
  };
  static constexpr bool kStaticTail = false;
  const NtOperands& p;
  idx_t m0, n0;

  __device__ __forceinline__ idx_t stages() const { return p.row_bytes / C::bkb; }
  // 16-byte chunk q of a stage (q = thread + T i) is chunk q % CPR of row
  // q / CPR: consecutive lanes read consecutive bytes of a row.
  __device__ __forceinline__ void load(idx_t kt, Regs& R) const {
    const idx_t k0b = kt * C::bkb;
    const int t = (int)thread_x<T>().index();
    if constexpr (kBuf) {
      const BufferWindow<1> wa{(uint32_t)p.row_bytes, C::bm, (int32_t)p.row_bytes};
      const BufferWindow<1> wb{(uint32_t)p.row_bytes, C::bn, (int32_t)p.row_bytes};
#pragma unroll
      for (int pl = 0; pl < P; ++pl) {
        const auto ra = buffer_rsrc(&matrix(p.a[pl], 0, p.row_bytes).at(m0, 0), wa.bytes());
        const auto rb = buffer_rsrc(&matrix(p.b[pl], 0, p.row_bytes).at(n0, 0), wb.bytes());
#pragma unroll
        for (int i = 0; i < C::a_chunks; ++i) {
          const int q = t + T * i;
          R.a[pl][i] = __builtin_bit_cast(
              u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                         ra, (int)(wa.row(q / CPR) + wa.col_valid(16 * (q % CPR))), (int)k0b, 0));
        }
#pragma unroll
        for (int i = 0; i < C::b_chunks; ++i) {
          const int q = t + T * i;
          R.b[pl][i] = __builtin_bit_cast(
              u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                         rb, (int)(wb.row(q / CPR) + wb.col_valid(16 * (q % CPR))), (int)k0b, 0));
        }
      }
      return;
    }
#pragma unroll
    for (int pl = 0; pl < P; ++pl) {
      auto ag = matrix(p.a[pl], 0, p.row_bytes);
      auto bg = matrix(p.b[pl], 0, p.row_bytes);
#pragma unroll
      for (int i = 0; i < C::a_chunks; ++i) {
        const int q = t + T * i;
        R.a[pl][i] = *(const u32x4*)&ag.at(m0 + q / CPR, k0b + 16 * (q % CPR));
      }
#pragma unroll
      for (int i = 0; i < C::b_chunks; ++i) {
        const int q = t + T * i;
        R.b[pl][i] = *(const u32x4*)&bg.at(n0 + q / CPR, k0b + 16 * (q % CPR));
      }
    }
  }
  template <class PlaneFn>
  __device__ __forceinline__ void store(const Regs& R, PlaneFn&& plane) const {
    const int t = (int)thread_x<T>().index();
#pragma unroll
    for (int pl = 0; pl < P; ++pl) {
      auto s = plane(pl);
#pragma unroll
      for (int i = 0; i < C::a_chunks; ++i) {
        const int q = t + T * i;
        s.at(q / CPR, q % CPR) = R.a[pl][i];
      }
#pragma unroll
      for (int i = 0; i < C::b_chunks; ++i) {
        const int q = t + T * i;
        s.at(C::bm + q / CPR, q % CPR) = R.b[pl][i];
      }
    }
  }
};

// Row-major FP32 operands as the caller holds them: A (M x K, stride lda),
// B (K x N, stride ldb).
struct F32Operands {
  const float* A;
  int64_t lda;
  const float* B;
  int64_t ldb;
  int64_t M, N, K;
};

// The strides the split source accepts: its buffer offsets, at most 16 rows
// of A or 8 rows of B from a range's base, stay below 2^31.
constexpr int64_t kSplitMaxLd = int64_t(1) << 24;

// SplitSource (Bf16x3 mode): the FP32 operands split into hi and lo on the
// way into LDS, so no pre-pass and no planes in memory.  A stage is KS = 8 x
// chunks values of K; a thread takes whole octets (8 consecutive k of one row
// of A or column of B: one 16-byte chunk of each plane) and writes them,
// split, to chunk `octet` of row `row` (A) or BM + column (B^T).
//   A: octet q is octet q % CPR of row q / CPR.  The 16 rows one wave reads
//      per octet set are one buffer range (base at the stage's k0), read as
//      two 16-byte loads per octet when kVec (A 16-byte aligned, lda and K
//      multiples of 4), else as 8 single loads.
//   B: octet q is column q % BN, octet q / BN, which is one octet per wave:
//      its 8 rows are one buffer range, read as 8 single loads, each
//      coalesced over the wave's 64 consecutive columns.
// Edges: a range ends at the last valid element (past K in the last row of
// A, past the valid rows of A or B), so loads beyond it return zero; inside a
// range, k past K in the other rows of A and columns past N of B are sent
// outside it by their offsets.  Every load is unconditional: branches around
// loads would double the registers the staging sets take.  Any shape with M,
// N, K >= 1 and lda, ldb <= kSplitMaxLd.
template <class C, bool kVec>
struct SplitSource {
  static_assert(C::mode::planes == 2 && C::mode::step_bytes == 32, "Bf16x3 mode only");
  static constexpr int T = C::threads, CPR = C::chunks, KS = 8 * C::chunks;
  static constexpr int AO = C::bm * CPR / T, BO = C::bn * CPR / T;
  static_assert(AO >= 1 && BO >= 1 && AO * T == C::bm * CPR && BO * T == C::bn * CPR,
                "octets divide evenly among the threads");
  static_assert(CPR == 4 && kWave % CPR == 0 && C::bn % kWave == 0,
                "a wave covers 16 whole rows of A and one octet of B");
  struct Regs {
    f32x4 a[AO][2], b[BO][2];   // an octet as two groups of four values
  };
  static constexpr bool kStaticTail = true;
  const F32Operands& p;
  idx_t m0, n0;
  // What a wave's ranges keep over the whole K loop (uniform values): each
  // A row group's valid rows and its first row (A's first when it has
  // none); each B octet's valid columns, its first k in a stage, and B from
  // that k on at its first column (B itself when it has no valid column).
  // A stage's range bases are these views at the stage's k.
  int32_t a_rows[AO], b_cols[BO];
  idx_t b_k[BO];
  const float* a_first[AO];
  const float* b_first[BO];

  __device__ __forceinline__ SplitSource(const F32Operands& f, idx_t m0_, idx_t n0_)
      : p(f), m0(m0_), n0(n0_) {
    const int w = __builtin_amdgcn_readfirstlane((int)wave_of_block<T>().index());
#pragma unroll
    for (int i = 0; i < AO; ++i) {
      const idx_t r0 = m0 + (T / CPR) * i + (kWave / CPR) * w;  // first of the wave's rows
      const idx_t rv = max_i(min_i(p.M - r0, kWave / CPR), 0);   // its valid rows
      a_rows[i] = (int32_t)rv;
      a_first[i] = &matrix(p.A, p.M, p.lda).at(rv > 0 ? r0 : 0, 0);
    }
#pragma unroll
    for (int i = 0; i < BO; ++i) {
      const int q0 = T * i + kWave * w;                          // the wave's first octet index
      const idx_t c0 = n0 + q0 % C::bn;                           // the wave's first column
      const idx_t cv = max_i(min_i(p.N - c0, kWave), 0);          // valid columns of the wave
      b_cols[i] = (int32_t)cv;
      b_k[i] = 8 * (q0 / C::bn);
      b_first[i] = cv > 0 ? &matrix(p.B, p.K, p.ldb).at(b_k[i], c0) : p.B;
    }
  }

  __device__ __forceinline__ idx_t stages() const { return (p.K + KS - 1) / KS; }

  // Stage kt.  Every stage but a last partial one is full (all KS values of
  // k inside K): then each range's extent and a lane's offsets in it are
  // the same for every stage, and only the ranges' bases move with k.
  __device__ __forceinline__ void load(idx_t kt, Regs& R) const {
    const idx_t k0 = kt * KS;
    if (k0 + KS <= p.K) load_stage<true>(k0, R);
    else load_stage<false>(k0, R);
  }
  template <bool kFull>
  __device__ __forceinline__ void load_stage(idx_t k0, Regs& R) const {
    const int32_t cols = kFull ? KS : (int32_t)min_i(p.K - k0, KS);   // valid k of this stage
    const int lane = (int)lane_of_wave().index();
    const int lr = layout::split_a_row<CPR>(lane);               // row in the wave's 16
    const int ka = layout::split_a_k<CPR>(lane);                 // first k of the lane's octet
#pragma unroll
    for (int i = 0; i < AO; ++i) {
      const BufferWindow<4> win{(uint32_t)p.lda, a_rows[i], cols};
      // k0 < K: the base stays inside the group's first row (or A's)
      const auto rs = buffer_rsrc(&array(a_first[i], p.K).at(k0), win.bytes());
      const uint32_t row = win.row(lr);
      if constexpr (kVec) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
          R.a[i][h] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                    rs, (int)(row + win.col(ka + 4 * h)), 0, 0));
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          R.a[i][j / 4][j % 4] = __uint_as_float(
              __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(row + win.col(ka + j)), 0, 0));
      }
    }
#pragma unroll
    for (int i = 0; i < BO; ++i) {
      // valid k of the octet (all 8 in a full stage); an octet past K reads
      // nothing, and its base stays at the group's first row
      const int32_t rv = kFull ? 8 : (int32_t)max_i(min_i(p.K - k0 - b_k[i], 8), 0);
      const BufferWindow<4> win{(uint32_t)p.ldb, rv, b_cols[i]};
      const idx_t kr = kFull || rv > 0 ? k0 : 0;
      const auto rs = buffer_rsrc(&matrix(b_first[i], p.K, p.ldb).at(kr, 0), win.bytes());
      const uint32_t col = win.col(layout::split_b_col(lane));
#pragma unroll
      for (int j = 0; j < 8; ++j)
        R.b[i][j / 4][j % 4] = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(win.row(j) + col), 0, 0));
    }
  }
  __device__ __forceinline__ static idx_t min_i(idx_t x, idx_t y) { return x < y ? x : y; }
  __device__ __forceinline__ static idx_t max_i(idx_t x, idx_t y) { return x > y ? x : y; }

  template <class PlaneFn>
  __device__ __forceinline__ void store(const Regs& R, PlaneFn&& plane) const {
    const int t = (int)thread_x<T>().index();
    auto hi = plane(0);
    auto lo = plane(1);
    auto put = [&](idx_t row, int oct, f32x4 v, f32x4 w) {
      const lowp::Split4 x = lowp::split_bf16x4(v[0], v[1], v[2], v[3]);
      const lowp::Split4 y = lowp::split_bf16x4(w[0], w[1], w[2], w[3]);
      hi.at(row, oct) = join(x.hi, y.hi);
      lo.at(row, oct) = join(x.lo, y.lo);
    };
#pragma unroll
    for (int i = 0; i < AO; ++i) {
      const int q = t + T * i;
      put(q / CPR, q % CPR, R.a[i][0], R.a[i][1]);
    }
#pragma unroll
    for (int i = 0; i < BO; ++i) {
      const int q = t + T * i;
      put(C::bm + q % C::bn, q / C::bn, R.b[i][0], R.b[i][1]);
    }
  }
  __device__ __forceinline__ static u32x4 join(lowp::bf16x4_bits x, lowp::bf16x4_bits y) {
    const lowp::u32x2_bits a = __builtin_bit_cast(lowp::u32x2_bits, x);
    const lowp::u32x2_bits b = __builtin_bit_cast(lowp::u32x2_bits, y);
    return u32x4{a[0], a[1], b[0], b[1]};
  }
};

// Where the tile's FP32 result goes: C (M x N valid, stride ldc) and, in the
// scaled mode, the row scales of A and column scales of B.
struct NtEpilogue {
  float* C;
  int64_t ldc;
  int64_t M, N;
  const float* sa;
  const float* sb;
};

template <class C, class Src>
__device__ __forceinline__ void tile_from(const Src& src, const NtEpilogue& p, idx_t tm, idx_t tn,
                                          uint8_t* lds) {
  using Mode = typename C::mode;
  constexpr int P = Mode::planes, LB = Mode::lane_bytes;
  constexpr int T = C::threads;
  auto thread = thread_x<T>();
  auto wv = wave_of_block<T>();
  const int lane = (int)lane_of_wave().index();
  const int half = lane / 32, col32 = lane % 32;
  const int wm = (int)wv.index() / C::wn, wn = (int)wv.index() % C::wn;
  const idx_t m0 = tm * C::bm, n0 = tn * C::bn;

  // LDS: [stage][plane][A rows then B rows][chunks] of 16 bytes, swizzled
  auto sm = matrices((u32x4*)lds, 2 * P, C::bm + C::bn, C::chunks);
  auto plane = [&](int stage, int pl) {
    return sm.idx(stage * P + pl).template xor_swizzle<C::rows_per_256, C::chunks>();
  };

  // Two register staging sets: stage j travels through set j % 2.
  using Stage = typename Src::Regs;
  Stage R0, R1;
  auto load = [&](idx_t kt, Stage& R) { src.load(kt, R); };
  auto store = [&](const Stage& R, int stage) {
    src.store(R, [&](int pl) { return plane(stage, pl); });
  };

  mfma::f32x16 acc[C::fm][C::fn];
#pragma unroll
  for (int i = 0; i < C::fm; ++i)
#pragma unroll
    for (int j = 0; j < C::fn; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // Matrix ops of one stage from LDS buffer `stage`.  A lane's fragments of
  // one step lie whole 32-row blocks apart, where the swizzle repeats (its
  // period, rows_per_256 x chunks rows, divides 32): the view gives the
  // chunk addresses of the first fragment, the others are constant offsets
  // from them (LDS read immediates).
  static_assert(32 % (C::rows_per_256 * C::chunks) == 0, "the swizzle repeats every 32 rows");
  constexpr int kFragStride = 32 * C::chunks;   // 16-byte chunks between fragments
  auto compute = [&](int stage) {
#pragma unroll
    for (int st = 0; st < C::steps; ++st) {
      // this lane's chunk(s) of the step: LB bytes from byte st*step + half*LB
      const int ch = (st * Mode::step_bytes + half * LB) / 16;
      gemm_nt::Frag<LB> fa[P][C::fm], fb[P][C::fn];
#pragma unroll
      for (int pl = 0; pl < P; ++pl) {
        auto s = plane(stage, pl);
        const u32x4* a0 = &s.at(wm * C::wtm + col32, ch);
        const u32x4* b0 = &s.at(C::bm + wn * C::wtn + col32, ch);
        const u32x4* a1 = &s.at(wm * C::wtm + col32, ch + (LB == 32 ? 1 : 0));
        const u32x4* b1 = &s.at(C::bm + wn * C::wtn + col32, ch + (LB == 32 ? 1 : 0));
#pragma unroll
        for (int i = 0; i < C::fm; ++i) {
          if constexpr (LB == 16) fa[pl][i].v = a0[i * kFragStride];
          else { fa[pl][i].v0 = a0[i * kFragStride]; fa[pl][i].v1 = a1[i * kFragStride]; }
        }
#pragma unroll
        for (int j = 0; j < C::fn; ++j) {
          if constexpr (LB == 16) fb[pl][j].v = b0[j * kFragStride];
          else { fb[pl][j].v0 = b0[j * kFragStride]; fb[pl][j].v1 = b1[j * kFragStride]; }
        }
      }
#pragma unroll
      for (int i = 0; i < C::fm; ++i)
#pragma unroll
        for (int j = 0; j < C::fn; ++j) {
          if constexpr (Mode::scaled) {
            acc[i][j] = mfma::fp8_32x32x64(fa[0][i].i8(), fb[0][j].i8(), acc[i][j]);
          } else {
            acc[i][j] = mfma::bf16_32x32x16(fa[1][i].bf16(), fb[0][j].bf16(), acc[i][j]);
            acc[i][j] = mfma::bf16_32x32x16(fa[0][i].bf16(), fb[1][j].bf16(), acc[i][j]);
            acc[i][j] = mfma::bf16_32x32x16(fa[0][i].bf16(), fb[0][j].bf16(), acc[i][j]);
          }
        }
    }
  };

  // Pipelined matrix ops of one stage (scaled mode): a step's B fragments
  // stay in registers while its A fragments stream through two register
  // sets.  Group g is the fn matrix ops of one A fragment; the reads for
  // group g + 1 (the next A fragment, or the next step's B fragments and
  // first A fragment, into the other sets) are issued before group g's
  // matrix ops, so their LDS latency runs under those.  The scheduling
  // groups pin that order: the compiler would otherwise gather the reads.
  auto compute_pipe = [&](auto stage) {
    using F = gemm_nt::Frag<32>;
    auto s = plane(stage, 0);
    // Rows 32 apart share the swizzle (its period, rows_per_256 x chunks
    // rows, divides 32), so a lane's fragments of one step lie whole 32-row
    // blocks apart: the chunk addresses of its first fragment come from the
    // view, the others are constant offsets from them (LDS read immediates
    // instead of an address computation per read).
    const u32x4* first[2][C::steps][2];
#pragma unroll
    for (int st = 0; st < C::steps; ++st)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int ch = (st * Mode::step_bytes + half * LB) / 16 + e;
        first[0][st][e] = &s.at(wm * C::wtm + col32, ch);
        first[1][st][e] = &s.at(C::bm + wn * C::wtn + col32, ch);
      }
    auto read = [&](int op, int st, int k, F& f) {
      f.v0 = first[op][st][0][k * kFragStride];
      f.v1 = first[op][st][1][k * kFragStride];
    };
    auto read_a = [&](int st, int i, F& f) { read(0, st, i, f); };
    auto read_b = [&](int st, int j, F& f) { read(1, st, j, f); };
    constexpr unsigned kDsRead = 0x100, kMatrix = 0x008;   // sched_group_barrier masks
    F fa[2], fb[2][C::fn];
#pragma unroll
    for (int j = 0; j < C::fn; ++j) read_b(0, j, fb[0][j]);
    read_a(0, 0, fa[0]);
    __builtin_amdgcn_sched_group_barrier(kDsRead, 2 * C::fn + 2, 0);
#pragma unroll
    for (int st = 0; st < C::steps; ++st)
#pragma unroll
      for (int i = 0; i < C::fm; ++i) {
        const int g = st * C::fm + i;
        if (i + 1 < C::fm) {
          read_a(st, i + 1, fa[(g + 1) & 1]);
          __builtin_amdgcn_sched_group_barrier(kDsRead, 2, 0);
        } else if (st + 1 < C::steps) {
#pragma unroll
          for (int j = 0; j < C::fn; ++j) read_b(st + 1, j, fb[(st + 1) & 1][j]);
          read_a(st + 1, 0, fa[(g + 1) & 1]);
          __builtin_amdgcn_sched_group_barrier(kDsRead, 2 * C::fn + 2, 0);
        }
#pragma unroll
        for (int j = 0; j < C::fn; ++j)
          acc[i][j] = mfma::fp8_32x32x64(fa[g & 1].i8(), fb[st & 1][j].i8(), acc[i][j]);
        __builtin_amdgcn_sched_group_barrier(kMatrix, C::fn, 0);
      }
  };
  auto compute_stage = [&](int stage) {
    if constexpr (C::pipe) compute_pipe(stage);
    else compute(stage);
  };

  const idx_t nk = src.stages();
  if constexpr (C::depth == 1) {
    // One stage ahead: iteration kt loads stage kt+1 into registers, computes
    // stage kt from LDS and writes stage kt+1 to the other buffer; the last
    // stage is peeled so the loop body has no branch.
    load(0, R0);
    store(R0, 0);
    sync(thread);
    for (idx_t kt = 0; kt + 1 < nk; ++kt) {
      const int stage = (int)(kt & 1);
      load(kt + 1, R0);
      __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the matrix ops
      compute_stage(stage);
      __builtin_amdgcn_sched_barrier(0);
      store(R0, stage ^ 1);
      sync(thread);
    }
    compute_stage((int)((nk - 1) & 1));
  } else {
    // Two stages deep: at the start of iteration kt, LDS buffer kt % 2 holds
    // stage kt and register set (kt+1) % 2 holds stage kt+1 (its loads issued
    // one iteration earlier).  Iteration kt issues the loads of stage kt+2,
    // computes stage kt, writes stage kt+1 to the other LDS buffer and
    // synchronises, so a global load has two stages of matrix ops to arrive.
    // The steady state runs in pairs of iterations (register sets named
    // statically) without branches; the last iterations are peeled.
    load(0, R0);
    store(R0, 0);
    if (nk > 1) load(1, R1);
    sync(thread);
    idx_t kt = 0;
    for (; kt + 3 < nk; kt += 2) {
      load(kt + 2, R0);
      __builtin_amdgcn_sched_barrier(0);
      compute_stage(0);
      __builtin_amdgcn_sched_barrier(0);
      store(R1, 1);
      sync(thread);
      load(kt + 3, R1);
      __builtin_amdgcn_sched_barrier(0);
      compute_stage(1);
      __builtin_amdgcn_sched_barrier(0);
      store(R0, 0);
      sync(thread);
    }
    // At most three iterations are left, kt even.  With the split source
    // they are written out so that each names its register sets statically:
    // a set chosen at run time lives in memory when its values are not plain
    // copies.  The plane source keeps the loop, which allocates better there.
    if constexpr (Src::kStaticTail) {
      if (kt < nk) {
        if (kt + 2 < nk) load(kt + 2, R0);
        compute_stage(0);
        if (kt + 1 < nk) store(R1, 1);
        sync(thread);
      }
      if (kt + 1 < nk) {
        compute_stage(1);
        if (kt + 2 < nk) store(R0, 0);
        sync(thread);
      }
      if (kt + 2 < nk) {
        compute_stage(0);
        sync(thread);
      }
    } else {
      for (; kt < nk; ++kt) {
        const bool even = (kt & 1) == 0;
        if (kt + 2 < nk) load(kt + 2, even ? R0 : R1);
        compute_stage((int)(kt & 1));
        if (kt + 1 < nk) store(even ? R1 : R0, (int)((kt + 1) & 1));
        sync(thread);
      }
    }
  }

  // Epilogue.  The scales are padded to whole tiles, so a lane's scale loads
  // are issued together, before its stores: all of them when the wave tile
  // has at most two fragment rows, one fragment row at a time otherwise (the
  // row scales of four fragment rows would take 64 registers).  A tile wholly
  // inside C stores without guards.
  auto c_g = matrix(p.C, p.M, p.ldc);
  constexpr int EB = C::fm > 2 ? 1 : C::fm;   // fragment rows per batch
  const bool full = m0 + C::bm <= p.M && n0 + C::bn <= p.N;
  float sbv[C::fn];
  if constexpr (Mode::scaled) {
    auto sb = array(p.sb, 0);
#pragma unroll
    for (int j = 0; j < C::fn; ++j) sbv[j] = sb[n0 + wn * C::wtn + j * 32 + col32];
  }
#pragma unroll
  for (int i0 = 0; i0 < C::fm; i0 += EB) {
    float sav[EB][16];
    if constexpr (Mode::scaled) {
      auto sa = array(p.sa, 0);
#pragma unroll
      for (int i = 0; i < EB; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          sav[i][r] = sa[m0 + wm * C::wtm + (i0 + i) * 32 + mfma::acc_row(r, lane)];
    }
    auto value = [&](int i, int j, int r) {
      float v = acc[i0 + i][j][r];
      if constexpr (Mode::scaled) v = (v * sav[i][r]) * sbv[j];
      return v;
    };
    if (full) {
#pragma unroll
      for (int i = 0; i < EB; ++i)
#pragma unroll
        for (int j = 0; j < C::fn; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            c_g.at(m0 + wm * C::wtm + (i0 + i) * 32 + mfma::acc_row(r, lane),
                   n0 + wn * C::wtn + j * 32 + col32) = value(i, j, r);
    } else {
#pragma unroll
      for (int i = 0; i < EB; ++i)
#pragma unroll
        for (int j = 0; j < C::fn; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const idx_t row = m0 + wm * C::wtm + (i0 + i) * 32 + mfma::acc_row(r, lane);
            const idx_t col = n0 + wn * C::wtn + j * 32 + col32;
            if (row < p.M && col < p.N) c_g.at(row, col) = value(i, j, r);
          }
    }
  }
}

// A tile of C from padded planes (the operand pre-pass layout).
template <class C, bool kBuf = false>
__device__ __forceinline__ void tile(const NtOperands& p, idx_t tm, idx_t tn, uint8_t* lds) {
  const PlaneSource<C, kBuf> src{p, tm * C::bm, tn * C::bn};
  tile_from<C>(src, NtEpilogue{p.C, p.ldc, p.M, p.N, p.sa, p.sb}, tm, tn, lds);
}

// A tile of C = A * B in the Bf16x3 mode straight from FP32 operands
// (M, N, K >= 1).  kVec: A read in 16-byte groups (A 16-byte aligned, lda
// and K multiples of 4).
template <class C, bool kVec>
__device__ __forceinline__ void tile_split(const F32Operands& f, float* Cp, int64_t ldc, idx_t tm,
                                           idx_t tn, uint8_t* lds) {
  const SplitSource<C, kVec> src{f, tm * C::bm, tn * C::bn};
  tile_from<C>(src, NtEpilogue{Cp, ldc, f.M, f.N, nullptr, nullptr}, tm, tn, lds);
}

}  // namespace gemm_nt
}  // namespace desc
