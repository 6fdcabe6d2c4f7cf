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
#include "mfma.hpp"
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
// each computing a (kBM / kWM) x (kBN / kWN) part of it.
template <int kBM, int kBN, int kBKB, class Mode, int kDepth = 2, int kWM = 2, int kWN = 2>
struct NtCfg {
  using mode = Mode;
  static constexpr int bm = kBM, bn = kBN, bkb = kBKB, depth = kDepth;
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

template <class C>
__device__ __forceinline__ void tile(const NtOperands& p, idx_t tm, idx_t tn, uint8_t* lds) {
  using Mode = typename C::mode;
  constexpr int P = Mode::planes, LB = Mode::lane_bytes, BKB = C::bkb;
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
  struct Stage {
    u32x4 a[P][C::a_chunks], b[P][C::b_chunks];
  };
  Stage R0, R1;
  // 16-byte chunk q of a stage (q = thread + T i) is chunk q % CPR of row
  // q / CPR: consecutive lanes read consecutive bytes of a row.
  constexpr int CPR = C::chunks;
  auto load = [&](idx_t k0b, Stage& R) {
#pragma unroll
    for (int pl = 0; pl < P; ++pl) {
      auto ag = matrix(p.a[pl], 0, p.row_bytes);
      auto bg = matrix(p.b[pl], 0, p.row_bytes);
#pragma unroll
      for (int i = 0; i < C::a_chunks; ++i) {
        const int q = (int)thread.index() + T * i;
        R.a[pl][i] = *(const u32x4*)&ag.at(m0 + q / CPR, k0b + 16 * (q % CPR));
      }
#pragma unroll
      for (int i = 0; i < C::b_chunks; ++i) {
        const int q = (int)thread.index() + T * i;
        R.b[pl][i] = *(const u32x4*)&bg.at(n0 + q / CPR, k0b + 16 * (q % CPR));
      }
    }
  };
  auto store = [&](const Stage& R, int stage) {
#pragma unroll
    for (int pl = 0; pl < P; ++pl) {
      auto s = plane(stage, pl);
#pragma unroll
      for (int i = 0; i < C::a_chunks; ++i) {
        const int q = (int)thread.index() + T * i;
        s.at(q / CPR, q % CPR) = R.a[pl][i];
      }
#pragma unroll
      for (int i = 0; i < C::b_chunks; ++i) {
        const int q = (int)thread.index() + T * i;
        s.at(C::bm + q / CPR, q % CPR) = R.b[pl][i];
      }
    }
  };

  mfma::f32x16 acc[C::fm][C::fn];
#pragma unroll
  for (int i = 0; i < C::fm; ++i)
#pragma unroll
    for (int j = 0; j < C::fn; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // Matrix ops of one stage from LDS buffer `stage`.
  auto compute = [&](int stage) {
#pragma unroll
    for (int st = 0; st < C::steps; ++st) {
      // this lane's chunk(s) of the step: LB bytes from byte st*step + half*LB
      const int ch = (st * Mode::step_bytes + half * LB) / 16;
      gemm_nt::Frag<LB> fa[P][C::fm], fb[P][C::fn];
#pragma unroll
      for (int pl = 0; pl < P; ++pl) {
        auto s = plane(stage, pl);
#pragma unroll
        for (int i = 0; i < C::fm; ++i) {
          const idx_t row = wm * C::wtm + i * 32 + col32;
          if constexpr (LB == 16) fa[pl][i].v = s.at(row, ch);
          else { fa[pl][i].v0 = s.at(row, ch); fa[pl][i].v1 = s.at(row, ch + 1); }
        }
#pragma unroll
        for (int j = 0; j < C::fn; ++j) {
          const idx_t row = C::bm + wn * C::wtn + j * 32 + col32;
          if constexpr (LB == 16) fb[pl][j].v = s.at(row, ch);
          else { fb[pl][j].v0 = s.at(row, ch); fb[pl][j].v1 = s.at(row, ch + 1); }
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

  const idx_t nk = p.row_bytes / BKB;
  if constexpr (C::depth == 1) {
    // One stage ahead: iteration kt loads stage kt+1 into registers, computes
    // stage kt from LDS and writes stage kt+1 to the other buffer; the last
    // stage is peeled so the loop body has no branch.
    load(0, R0);
    store(R0, 0);
    sync(thread);
    for (idx_t kt = 0; kt + 1 < nk; ++kt) {
      const int stage = (int)(kt & 1);
      load((kt + 1) * BKB, R0);
      __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the matrix ops
      compute(stage);
      __builtin_amdgcn_sched_barrier(0);
      store(R0, stage ^ 1);
      sync(thread);
    }
    compute((int)((nk - 1) & 1));
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
    if (nk > 1) load(BKB, R1);
    sync(thread);
    idx_t kt = 0;
    for (; kt + 3 < nk; kt += 2) {
      load((kt + 2) * BKB, R0);
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      __builtin_amdgcn_sched_barrier(0);
      store(R1, 1);
      sync(thread);
      load((kt + 3) * BKB, R1);
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      __builtin_amdgcn_sched_barrier(0);
      store(R0, 0);
      sync(thread);
    }
    for (; kt < nk; ++kt) {            // at most three iterations left
      const bool even = (kt & 1) == 0;
      if (kt + 2 < nk) load((kt + 2) * BKB, even ? R0 : R1);
      compute((int)(kt & 1));
      if (kt + 1 < nk) store(even ? R1 : R0, (int)((kt + 1) & 1));
      sync(thread);
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

}  // namespace gemm_nt
}  // namespace desc
