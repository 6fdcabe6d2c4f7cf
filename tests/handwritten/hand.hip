// hand.hip -- hand-indexed twins of the view-based reduce, scan and
// transpose kernels: the baseline of the evaluation of Sec. 5, which compares
// the kernels written against views with the same algorithms written directly
// in the kernel programming model, with raw index arithmetic.
//
// Each twin has the algorithm, tile shape, memory-access order, index types
// (int64) and synchronisation of the view kernel it mirrors, in one of that
// kernel's configurations:
//   reduce     256 threads, 4 int32x4 per lane per tile, non-temporal loads;
//   scan       1024 threads x 16 rounds x 4 int32 per tile (64K elements),
//              non-temporal loads and stores, 256-word look-back window
//              (the configuration the library runs from 2^24 elements);
//   transpose  128 x 128 tiles, LDS pitch 129, 256 threads as [8][32];
//   FP32 GEMM  128 x 128 x 16 tiles, 2 x 2 waves of 16 x 16 x 4
//              instructions, A row-major in LDS, loads two stages ahead,
//              interior tiles through buffer ranges (the configuration the
//              library runs from 2^30 M N K on).
// Only the index expressions differ: here they are written out by hand
// instead of being derived from a composition of views.  The helpers shared
// with the library (relaxed status-word atomics, DPP wave sums) hold no index
// arithmetic.
//
// The twins are measurement infrastructure, not part of the library; they
// are exported with a minimal C interface that does no argument checking.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "lowp.hpp"
#include "wave.hpp"

namespace hand {
using desc::i32x4;
using desc::u32x4;
using desc::kWave;
using desc::WsHeader;
using desc::CallState;

// ---------------------------------------------------------------- reduce
constexpr int kRBlock = 256, kRUnroll = 4;
constexpr int kRTileVec = kRBlock * kRUnroll, kRTile = kRTileVec * 4;
constexpr int kValueBits = 51;
constexpr uint64_t kValueMask = (1ull << kValueBits) - 1;
constexpr uint32_t kTagPeriod = 8191;

__device__ __forceinline__ uint64_t tag_of(uint32_t gen) { return 1u + gen % kTagPeriod; }

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* lds) {
  v = desc::wave::sum_i64(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x / 64] = v;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int w = 0; w < kRBlock / kWave; ++w) s += lds[w];
  return s;
}

__global__ __launch_bounds__(kRBlock) void reduce_i32_hand(
    const i32x4* __restrict__ body, int64_t ntiles, const int32_t* __restrict__ head,
    int64_t nhead, const int32_t* __restrict__ tail, int64_t ntail, int64_t* __restrict__ out,
    WsHeader* __restrict__ hdr, uint64_t* __restrict__ partials) {
  __shared__ int64_t lds[kRBlock / kWave];
  __shared__ CallState s_call;
  const int64_t b = blockIdx.x, nb = gridDim.x, tid = threadIdx.x;
  if (tid == 0) s_call = desc::read_call_state(hdr);
  int64_t acc = 0;
  for (int64_t t = b; t < ntiles; t += nb) {
    const i32x4* p = body + t * kRTileVec + tid;
    i32x4 q[kRUnroll];
#pragma unroll
    for (int u = 0; u < kRUnroll; ++u) q[u] = __builtin_nontemporal_load(p + u * kRBlock);
#pragma unroll
    for (int u = 0; u < kRUnroll; ++u)
      acc += (int64_t)q[u].x + (int64_t)q[u].y + (int64_t)q[u].z + (int64_t)q[u].w;
  }
  const bool last = b == nb - 1;
  if (last) {
    for (int64_t i = tid; i < nhead; i += kRBlock) acc += head[i];
    for (int64_t i = tid; i < ntail; i += kRBlock) acc += tail[i];
  }
  const int64_t s = block_sum(acc, lds);
  const uint32_t gen = s_call.gen;
  if (!last) {
    if (tid == 0)
      desc::store_status(&partials[b], (tag_of(gen) << kValueBits) | ((uint64_t)s & kValueMask));
    return;
  }
  const uint64_t want = tag_of(gen);
  const uint32_t maxp = s_call.polls;
  int64_t acc2 = tid == 0 ? s : 0;
  for (int64_t i = tid; i < nb - 1; i += kRBlock) {
    uint64_t w = 0;
    for (uint32_t polls = 0;; ++polls) {
      if (polls == maxp) {
        desc::set_error(hdr, desc::kDevWaitLimit);
        w = 0;
        break;
      }
      w = desc::load_status(&partials[i]);
      if ((w >> kValueBits) == want) {
        desc::store_status(&partials[i], 0);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    acc2 += (int64_t)(w << (64 - kValueBits)) >> (64 - kValueBits);
  }
  __syncthreads();
  const int64_t total = block_sum(acc2, lds);
  if (tid == 0) {
    out[0] = total;
    desc::store_u32(&hdr->gen, desc::next_gen(gen));
  }
}

// ---------------------------------------------------------------- scan
constexpr uint64_t kFlagAggregate = 1, kFlagPrefix = 2;
constexpr uint32_t kTagMask = 0x3fffffffu;
constexpr int kLookWords = 4, kWindow = kWave * kLookWords;
constexpr int kSBlock = 1024, kSRounds = 16, kSWaves = kSBlock / kWave;
constexpr int kSTile = kSBlock * kSRounds * 4;

__device__ __forceinline__ uint64_t pack(uint64_t flag, uint32_t gen, uint32_t v) {
  return (flag << 62) | ((uint64_t)(gen & kTagMask) << 32) | (uint64_t)v;
}

__device__ __forceinline__ uint32_t look_back(const uint64_t* __restrict__ status, int64_t tile,
                                              uint32_t gen, uint32_t max_polls,
                                              WsHeader* __restrict__ hdr) {
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t tag = gen & kTagMask;
  uint32_t excl = 0;
  int64_t pos = tile - 1;
  for (uint32_t polls = 0;; ++polls) {
    if (polls == max_polls) {
      if (lane == 0) desc::set_error(hdr, desc::kDevWaitLimit);
      break;
    }
    uint64_t w[kLookWords];
#pragma unroll
    for (int q = 0; q < kLookWords; ++q) {
      const int64_t j = pos - (q * kWave + lane);
      w[q] = j >= 0 ? desc::load_status(&status[j]) : pack(kFlagPrefix, gen, 0u);
    }
    int first_p = kWindow;
    bool missing = false;
#pragma unroll
    for (int q = kLookWords - 1; q >= 0; --q) {
      const uint32_t flag = (uint32_t)(w[q] >> 62);
      const bool valid = flag != 0 && (uint32_t)((w[q] >> 32) & kTagMask) == tag;
      const uint64_t pm = __ballot(valid && flag == kFlagPrefix);
      if (pm) first_p = q * kWave + __builtin_ctzll(pm);
    }
#pragma unroll
    for (int q = 0; q < kLookWords; ++q) {
      const uint32_t flag = (uint32_t)(w[q] >> 62);
      const bool valid = flag != 0 && (uint32_t)((w[q] >> 32) & kTagMask) == tag;
      missing |= __ballot(!valid && q * kWave + lane <= first_p) != 0;
    }
    if (missing) {
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    uint32_t part = 0;
#pragma unroll
    for (int q = 0; q < kLookWords; ++q) part += (q * kWave + lane <= first_p) ? (uint32_t)w[q] : 0u;
    excl += desc::wave::sum_u32(part);
    if (first_p < kWindow) break;
    pos -= kWindow;
  }
  return excl;
}

template <bool kVec>
__global__ __launch_bounds__(kSBlock) void scan_i32_hand(const int32_t* __restrict__ in,
                                                         int32_t* __restrict__ out, int64_t n,
                                                         WsHeader* __restrict__ hdr,
                                                         uint64_t* __restrict__ status) {
  constexpr int R = kSRounds, NW = kSWaves;
  __shared__ CallState s_call;
  __shared__ uint32_t s_prefix;
  __shared__ uint32_t s_wtot[NW];
  const int64_t ntiles = gridDim.x, tile = blockIdx.x, tid = threadIdx.x;
  const int64_t wv = tid / kWave, lane = tid % kWave;
  if (tid == 0) s_call = desc::read_call_state(hdr);
  __syncthreads();
  const CallState call = s_call;
  const uint32_t gen = call.gen;

  // group g = ((tile * NW + wave) * R + r) * 64 + lane holds elements 4g..4g+3
  const int64_t g0 = ((tile * NW + wv) * R) * kWave + lane;
  const bool full = kVec && (tile + 1) * kSTile <= n;
  uint32_t x[R][4];
  if (full) {
    const i32x4* p = (const i32x4*)in + g0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const i32x4 q = __builtin_nontemporal_load(p + r * kWave);
      x[r][0] = (uint32_t)q.x; x[r][1] = (uint32_t)q.y;
      x[r][2] = (uint32_t)q.z; x[r][3] = (uint32_t)q.w;
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t e = 4 * (g0 + r * kWave);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[r][k] = e + k < n ? (uint32_t)in[e + k] : 0u;
    }
  }

  uint32_t lsum = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) lsum += x[r][0] + x[r][1] + x[r][2] + x[r][3];
  const uint32_t wsum = desc::wave::sum_u32(lsum);
  if (lane == 0) s_wtot[wv] = wsum;
  __syncthreads();
  uint32_t wex = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t v = s_wtot[w];
    wex += (w < wv) ? v : 0u;
    agg += v;
  }

  if (wv == 0) {
    uint32_t excl = 0;
    if (tile == 0) {
      if (lane == 0) desc::store_status(&status[0], pack(kFlagPrefix, gen, agg));
    } else {
      if (lane == 0) desc::store_status(&status[tile], pack(kFlagAggregate, gen, agg));
      excl = look_back(status, tile, gen, call.polls, hdr);
      if (lane == 0) desc::store_status(&status[tile], pack(kFlagPrefix, gen, excl + agg));
    }
    if (lane == 0) s_prefix = excl;
    if (tile == ntiles - 1) {
      const uint64_t hw = __hip_atomic_load(&hdr->hw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int64_t i = ntiles + (uint32_t)lane; i < (int64_t)hw; i += kWave)
        __hip_atomic_store(&status[i], (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (lane == 0) {
        __hip_atomic_store(&hdr->hw, (uint64_t)ntiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        desc::store_u32(&hdr->gen, desc::next_gen(gen));
      }
    }
  }

  uint32_t carry = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    x[r][1] += x[r][0];
    x[r][2] += x[r][1];
    x[r][3] += x[r][2];
    const uint32_t t = x[r][3];
    const uint32_t incl = desc::wave::inclusive_add_u32(t);
    const uint32_t ex = carry + incl - t;
#pragma unroll
    for (int k = 0; k < 4; ++k) x[r][k] += ex;
    carry += desc::wave::lane_read_u32(incl, kWave - 1);
  }
  __syncthreads();
  const uint32_t add = s_prefix + wex;

  if (full) {
    i32x4* p = (i32x4*)out + g0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      i32x4 q;
      q.x = (int32_t)(x[r][0] + add); q.y = (int32_t)(x[r][1] + add);
      q.z = (int32_t)(x[r][2] + add); q.w = (int32_t)(x[r][3] + add);
      __builtin_nontemporal_store(q, p + r * kWave);
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t e = 4 * (g0 + r * kWave);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (e + k < n) out[e + k] = (int32_t)(x[r][k] + add);
    }
  }
}

// ---------------------------------------------------------------- transpose
constexpr int kT = 128, kPitch = kT + 1, kTX = kT / 4, kTY = 256 / kTX, kIT = kT / kTY;

template <bool kVec>
__global__ __launch_bounds__(256) void transpose32_hand(const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, int64_t rows,
                                                        int64_t cols) {
  __shared__ uint32_t lds[kT * kPitch];
  // column tiles in diagonal order, as in the library's kernel
  const int64_t bx = ((int64_t)blockIdx.x + blockIdx.y) % gridDim.x, by = blockIdx.y,
                bz = blockIdx.z, tid = threadIdx.x;
  const bool full = kVec && (by + 1) * kT <= rows && (bx + 1) * kT <= cols;
  if (full) {
    const int64_t y = tid / kTX, x = tid % kTX, c4 = cols / 4, r4 = rows / 4;
    // row y of input tile (by, bx) and row y of output tile (bx, by)
    const u32x4* a = (const u32x4*)in + (bz * rows + by * kT + y) * c4 + bx * kTX + x;
    u32x4* b = (u32x4*)out + (bz * cols + bx * kT + y) * r4 + by * kTX + x;
    u32x4 v[kIT];
#pragma unroll
    for (int i = 0; i < kIT; ++i) v[i] = a[kTY * i * c4];
#pragma unroll
    for (int i = 0; i < kIT; ++i) {
      uint32_t* l = &lds[(y + kTY * i) * kPitch + 4 * x];
      l[0] = v[i].x; l[1] = v[i].y; l[2] = v[i].z; l[3] = v[i].w;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kIT; ++i) {
      const uint32_t* l = &lds[4 * x * kPitch + y + kTY * i];
      u32x4 w;
      w.x = l[0]; w.y = l[kPitch]; w.z = l[2 * kPitch]; w.w = l[3 * kPitch];
      b[kTY * i * r4] = w;
    }
  } else {
    const int64_t r0 = by * kT, c0 = bx * kT;
    const uint32_t* a = in + (bz * rows + r0) * cols + c0;
    uint32_t* b = out + (bz * cols + c0) * rows + r0;
    for (int64_t e = tid; e < kT * kT; e += 256) {
      const int64_t r = e / kT, c = e % kT;
      if (r0 + r < rows && c0 + c < cols) lds[r * kPitch + c] = a[r * cols + c];
    }
    __syncthreads();
    for (int64_t e = tid; e < kT * kT; e += 256) {
      const int64_t c = e / kT, r = e % kT;
      if (r0 + r < rows && c0 + c < cols) b[c * rows + r] = lds[r * kPitch + c];
    }
  }
}

// ---------------------------------------------------------------- FP32 GEMM
// Twin of gemm_f32w_kernel<GemmCfgF32W<128, 128, 16, 2, 2, 2, true>> (the
// library's FP32 GEMM from 2^30 M N K on): 256 threads as 2 x 2 waves of
// 64 x 64 in 16 x 16 fragments, A staged in LDS as [m][k] (pitch 20 words)
// and B as [k][n] (pitch 132), two LDS buffers, loads two stages ahead
// through two register sets, the 16 x 16 x 4 instruction's four k slots
// taking the four quarters of a stage.
constexpr int kGM = 128, kGN = 128, kGK = 16, kGT = 256, kGWN = 2;
constexpr int kGWTM = kGM / 2, kGWTN = kGN / 2, kGFM = kGWTM / 16, kGFN = kGWTN / 16;
constexpr int kGPA = kGK + 4, kGPB = kGN + 4;
constexpr int kGAV = kGM * kGK / 4 / kGT, kGBV = kGK * kGN / 4 / kGT;
constexpr int kGLds = 2 * kGM * kGPA + 2 * kGK * kGPB;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int64_t gemm_tile_of(int64_t u, int64_t tiles_m, int64_t tiles_n) {
  const int64_t T = tiles_m * tiles_n;
  if (T % 8 == 0) u = (u % 8) * (T / 8) + u / 8;
  const int64_t per_group = 8 * tiles_n, g = u / per_group, first_m = g * 8;
  const int64_t gsize = tiles_m - first_m < 8 ? tiles_m - first_m : 8;
  const int64_t r = u - g * per_group;
  return (first_m + r % gsize) * tiles_n + r / gsize;
}

// Interior tiles (the whole tile inside C, K a multiple of 16, each
// operand's span below 2^31 bytes, 16-byte aligned operands with leading
// dimensions that are multiples of 4): the loads are buffer loads at fixed
// per-lane byte offsets, the stage moving only the scalar offset.
template <bool kVec, bool kInterior>
__device__ __forceinline__ void gemm_f32_hand_tile(
    const float* __restrict__ A, int64_t lda, const float* __restrict__ B, int64_t ldb,
    float* __restrict__ Cm, int64_t ldc, int64_t M, int64_t N, int64_t K, int64_t m0, int64_t n0,
    float* lds) {
  float* const a_lds = lds;                          // [2][128][20]
  float* const b_lds = lds + 2 * kGM * kGPA;         // [2][16][132]
  const int tid = (int)threadIdx.x, lane = tid % 64, w = tid / 64;
  const int half = lane / 32, col32 = lane % 32, wm = w / kGWN, wn = w % kGWN;
  struct Regs {
    f32x4 a[kGAV], b[kGBV];
  };
  Regs R0, R1;
  __amdgpu_buffer_rsrc_t rs_a, rs_b;
  uint32_t off_a[kGAV], off_b[kGBV];
  if constexpr (kInterior) {
    rs_a = __builtin_amdgcn_make_buffer_rsrc((void*)(A + m0 * lda), 0,
                                             (int)(((kGM - 1) * lda + K) * 4), 0x00020000);
    rs_b = __builtin_amdgcn_make_buffer_rsrc((void*)(B + n0), 0,
                                             (int)(((K - 1) * ldb + kGN) * 4), 0x00020000);
#pragma unroll
    for (int i = 0; i < kGAV; ++i) {
      const int q = tid + kGT * i;
      off_a[i] = (uint32_t)(q / (kGK / 4)) * (uint32_t)lda * 4u + 16u * (uint32_t)(q % (kGK / 4));
    }
#pragma unroll
    for (int i = 0; i < kGBV; ++i) {
      const int q = tid + kGT * i;
      off_b[i] = (uint32_t)(q / (kGN / 4)) * (uint32_t)ldb * 4u + 16u * (uint32_t)(q % (kGN / 4));
    }
  }
  auto load = [&](int64_t kt, Regs& R) {
    const int64_t k0 = kt * kGK;
    if constexpr (kInterior) {
      const int sa = (int)(k0 * 4), sb = (int)((uint32_t)k0 * (uint32_t)ldb * 4u);
#pragma unroll
      for (int i = 0; i < kGAV; ++i)
        R.a[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs_a, (int)off_a[i],
                                                                                  sa, 0));
#pragma unroll
      for (int i = 0; i < kGBV; ++i)
        R.b[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs_b, (int)off_b[i],
                                                                                  sb, 0));
      return;
    }
#pragma unroll
    for (int i = 0; i < kGAV; ++i) {
      const int q = tid + kGT * i;
      const int64_t r = m0 + q / (kGK / 4), c = k0 + 4 * (q % (kGK / 4));
      if constexpr (kVec) {
        const bool in = r < M && c < K;
        const f32x4 v = *(const f32x4*)(A + (r < M ? r : M - 1) * lda + (c < K ? c : K - 4));
#pragma unroll
        for (int j = 0; j < 4; ++j) R.a[i][j] = in ? v[j] : 0.f;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) R.a[i][j] = (r < M && c + j < K) ? A[r * lda + c + j] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < kGBV; ++i) {
      const int q = tid + kGT * i;
      const int64_t r = k0 + q / (kGN / 4), c = n0 + 4 * (q % (kGN / 4));
      if constexpr (kVec) {
        const bool in = r < K && c < N;
        const f32x4 v = *(const f32x4*)(B + (r < K ? r : K - 1) * ldb + (c < N ? c : N - 4));
#pragma unroll
        for (int j = 0; j < 4; ++j) R.b[i][j] = in ? v[j] : 0.f;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) R.b[i][j] = (r < K && c + j < N) ? B[r * ldb + c + j] : 0.f;
      }
    }
  };
  auto store = [&](const Regs& R, int buf) {
#pragma unroll
    for (int i = 0; i < kGAV; ++i) {
      const int q = tid + kGT * i;
      *(f32x4*)(a_lds + (buf * kGM + q / (kGK / 4)) * kGPA + 4 * (q % (kGK / 4))) = R.a[i];
    }
#pragma unroll
    for (int i = 0; i < kGBV; ++i) {
      const int q = tid + kGT * i;
      *(f32x4*)(b_lds + (buf * kGK + q / (kGN / 4)) * kGPB + 4 * (q % (kGN / 4))) = R.b[i];
    }
  };
  f32x4 acc[kGFM][kGFN];
#pragma unroll
  for (int i = 0; i < kGFM; ++i)
#pragma unroll
    for (int j = 0; j < kGFN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.f;
  const int quarter = lane / 16, c16 = lane % 16;
  auto compute = [&](int buf) {
    f32x4 a[kGFM];
#pragma unroll
    for (int i = 0; i < kGFM; ++i)
      a[i] = *(const f32x4*)(a_lds + (buf * kGM + wm * kGWTM + i * 16 + c16) * kGPA +
                             quarter * (kGK / 4));
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      float b[kGFN];
#pragma unroll
      for (int j = 0; j < kGFN; ++j)
        b[j] = b_lds[(buf * kGK + quarter * (kGK / 4) + kk) * kGPB + wn * kGWTN + j * 16 + c16];
#pragma unroll
      for (int i = 0; i < kGFM; ++i)
#pragma unroll
        for (int j = 0; j < kGFN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][kk], b[j], acc[i][j], 0, 0, 0);
    }
  };
  const int64_t nk = (K + kGK - 1) / kGK;
  if (nk > 0) {
    load(0, R0);
    store(R0, 0);
  }
  if (nk > 1) load(1, R1);
  __syncthreads();
  int64_t kt = 0;
  for (; kt + 3 < nk; kt += 2) {
    load(kt + 2, R0);
    compute(0);
    store(R1, 1);
    __syncthreads();
    load(kt + 3, R1);
    compute(1);
    store(R0, 0);
    __syncthreads();
  }
  if (kt < nk) {
    if (kt + 2 < nk) load(kt + 2, R0);
    compute(0);
    if (kt + 1 < nk) store(R1, 1);
    __syncthreads();
  }
  if (kt + 1 < nk) {
    compute(1);
    if (kt + 2 < nk) store(R0, 0);
    __syncthreads();
  }
  if (kt + 2 < nk) {
    compute(0);
    __syncthreads();
  }
  // accumulator register r of lane l: row 4 (l / 16) + r, column l % 16
  if (m0 + kGM <= M && n0 + kGN <= N) {
#pragma unroll
    for (int i = 0; i < kGFM; ++i)
#pragma unroll
      for (int j = 0; j < kGFN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Cm[(m0 + wm * kGWTM + i * 16 + 4 * quarter + r) * ldc + n0 + wn * kGWTN + j * 16 + c16] =
              acc[i][j][r];
  } else {
#pragma unroll
    for (int i = 0; i < kGFM; ++i)
#pragma unroll
      for (int j = 0; j < kGFN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + wm * kGWTM + i * 16 + 4 * quarter + r;
          const int64_t col = n0 + wn * kGWTN + j * 16 + c16;
          if (row < M && col < N) Cm[row * ldc + col] = acc[i][j][r];
        }
  }
}

template <bool kVec>
__global__ __launch_bounds__(kGT) __attribute__((amdgpu_waves_per_eu(2)))
void gemm_f32_hand(const float* __restrict__ A, int64_t lda, const float* __restrict__ B,
                   int64_t ldb, float* __restrict__ Cm, int64_t ldc, int64_t M, int64_t N,
                   int64_t K) {
  __shared__ __attribute__((aligned(16))) float lds[kGLds];
  const int64_t tiles_n = (N + kGN - 1) / kGN;
  const int64_t t = gemm_tile_of(blockIdx.x, (M + kGM - 1) / kGM, tiles_n);
  const int64_t m0 = t / tiles_n * kGM, n0 = t % tiles_n * kGN;
  constexpr int64_t kSpan = int64_t(1) << 29;
  const bool interior = m0 + kGM <= M && n0 + kGN <= N && K > 0 && K % kGK == 0 &&
                        (kGM - 1) * lda + K < kSpan && (K - 1) * ldb + kGN < kSpan &&
                        ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && lda % 4 == 0 &&
                        ldb % 4 == 0;
  if (kVec && interior)
    gemm_f32_hand_tile<true, true>(A, lda, B, ldb, Cm, ldc, M, N, K, m0, n0, lds);
  else
    gemm_f32_hand_tile<kVec, false>(A, lda, B, ldb, Cm, ldc, M, N, K, m0, n0, lds);
}

// ---------------------------------------------------------------- e4m3 check
// The library's e4m3 quantisers use the hardware conversion for groups whose
// magnitudes are all finite and <= 448 and the software encoder otherwise.
// This kernel compares the two over all 2^32 binary32 inputs: counts[0]
// gets the disagreements at finite |x| <= 448, counts[1] the others.  One
// atomic per block and counter.
constexpr int kCvtThreads = 256, kCvtPer = 64;
constexpr uint64_t kCvtBlocks = (1ull << 32) / (kCvtThreads * kCvtPer);

__global__ __launch_bounds__(kCvtThreads) void e4m3_all_inputs(unsigned long long* counts) {
  __shared__ unsigned long long s_in, s_out;
  if (threadIdx.x == 0) { s_in = 0; s_out = 0; }
  __syncthreads();
  unsigned long long n_in = 0, n_out = 0;
  const uint64_t base = (uint64_t)blockIdx.x * kCvtThreads * kCvtPer;
  for (int j = 0; j < kCvtPer; ++j) {
    const uint32_t i = (uint32_t)(base + (uint64_t)j * kCvtThreads + threadIdx.x);
    const float x = __uint_as_float(i);
    const uint32_t sw = desc::lowp::e4m3_rne_sat(x);
    const uint32_t hw = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x, x, 0, false) & 0xffu;
    if (sw != hw) {
      if (fabsf(x) <= 448.0f) ++n_in; else ++n_out;
    }
  }
  atomicAdd(&s_in, n_in);
  atomicAdd(&s_out, n_out);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&counts[0], s_in);
    atomicAdd(&counts[1], s_out);
  }
}

// The hardware bf16 conversion against the library's software rounding:
// every input x is converted once in the low and once in the high half
// (paired with the bit-reversed pattern).  counts[0]: disagreements on
// inputs that are not NaNs, counts[1]: on NaNs.
__global__ __launch_bounds__(kCvtThreads) void bf16_all_inputs(unsigned long long* counts) {
  __shared__ unsigned long long s_num, s_nan;
  if (threadIdx.x == 0) { s_num = 0; s_nan = 0; }
  __syncthreads();
  unsigned long long n_num = 0, n_nan = 0;
  const uint64_t base = (uint64_t)blockIdx.x * kCvtThreads * kCvtPer;
  for (int j = 0; j < kCvtPer; ++j) {
    const uint32_t i = (uint32_t)(base + (uint64_t)j * kCvtThreads + threadIdx.x);
    const float x = __uint_as_float(i), y = __uint_as_float(__brev(i));
    const uint32_t hw1 = desc::lowp::bf16x2_hw(x, y), hw2 = desc::lowp::bf16x2_hw(y, x);
    const uint32_t sx = desc::lowp::bf16_rne(x), sy = desc::lowp::bf16_rne(y);
    const bool bad_x = (hw1 & 0xffffu) != sx || (hw2 >> 16) != sx;
    const bool bad_y = (hw1 >> 16) != sy || (hw2 & 0xffffu) != sy;
    if (bad_x) { if (__builtin_isnan(x)) ++n_nan; else ++n_num; }
    if (bad_y) { if (__builtin_isnan(y)) ++n_nan; else ++n_num; }
  }
  atomicAdd(&s_num, n_num);
  atomicAdd(&s_nan, n_nan);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&counts[0], s_num);
    atomicAdd(&counts[1], s_nan);
  }
}

}  // namespace hand

// ---------------------------------------------------------------- C interface
// All return a hipError_t value.  Workspaces follow the library's contract:
// zero-filled before the first call, then reused.

extern "C" {

size_t hand_reduce_i32_workspace(int64_t n) {
  const int64_t ntiles = n / hand::kRTile;
  int64_t grid = ntiles < 2048 ? ntiles : 2048;
  const int64_t need = (n + (1 << 19) - 1) >> 19;
  if (grid < need) grid = need;
  if (grid < 1) grid = 1;
  return sizeof(hand::WsHeader) + 8 * (size_t)grid;
}

int hand_reduce_i32(const int32_t* in, int64_t n, int64_t* out, void* ws, hipStream_t s) {
  const uintptr_t addr = (uintptr_t)in;
  int64_t nhead = (int64_t)(((16 - (addr & 15)) & 15) / 4);
  if (nhead > n) nhead = n;
  const int64_t rest = n - nhead, ntiles = rest / hand::kRTile;
  const int64_t ntail = rest - ntiles * hand::kRTile;
  const int64_t grid = (int64_t)(hand_reduce_i32_workspace(n) - sizeof(hand::WsHeader)) / 8;
  hipLaunchKernelGGL(hand::reduce_i32_hand, dim3((unsigned)grid), dim3(hand::kRBlock), 0, s,
                     (const hand::i32x4*)(in + nhead), ntiles, in, nhead,
                     in + nhead + ntiles * hand::kRTile, ntail, out, (hand::WsHeader*)ws,
                     (uint64_t*)((char*)ws + sizeof(hand::WsHeader)));
  return (int)hipGetLastError();
}

size_t hand_scan_i32_workspace(int64_t n) {
  const int64_t ntiles = (n + hand::kSTile - 1) / hand::kSTile;
  return sizeof(hand::WsHeader) + 8 * (size_t)(ntiles > 0 ? ntiles : 1);
}

int hand_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s) {
  if (n == 0) return 0;
  const int64_t ntiles = (n + hand::kSTile - 1) / hand::kSTile;
  hand::WsHeader* hdr = (hand::WsHeader*)ws;
  uint64_t* status = (uint64_t*)((char*)ws + sizeof(hand::WsHeader));
  if ((((uintptr_t)in | (uintptr_t)out) & 15) == 0)
    hipLaunchKernelGGL(hand::scan_i32_hand<true>, dim3((unsigned)ntiles), dim3(hand::kSBlock), 0,
                       s, in, out, n, hdr, status);
  else
    hipLaunchKernelGGL(hand::scan_i32_hand<false>, dim3((unsigned)ntiles), dim3(hand::kSBlock),
                       0, s, in, out, n, hdr, status);
  return (int)hipGetLastError();
}

int hand_transpose_f32(const float* in, float* out, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return 0;
  const dim3 grid((unsigned)((cols + hand::kT - 1) / hand::kT),
                  (unsigned)((rows + hand::kT - 1) / hand::kT), 1);
  const bool vec = rows % 4 == 0 && cols % 4 == 0 && (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(hand::transpose32_hand<true>, grid, dim3(256), 0, s,
                       (const uint32_t*)in, (uint32_t*)out, rows, cols);
  else
    hipLaunchKernelGGL(hand::transpose32_hand<false>, grid, dim3(256), 0, s,
                       (const uint32_t*)in, (uint32_t*)out, rows, cols);
  return (int)hipGetLastError();
}

int hand_gemm_f32(const float* A, int64_t lda, const float* B, int64_t ldb, float* C,
                  int64_t ldc, int64_t M, int64_t N, int64_t K, hipStream_t s) {
  if (M == 0 || N == 0) return 0;
  const int64_t tiles = ((M + hand::kGM - 1) / hand::kGM) * ((N + hand::kGN - 1) / hand::kGN);
  const bool vec = ((((uintptr_t)A) | ((uintptr_t)B)) & 15) == 0 && lda % 4 == 0 &&
                   ldb % 4 == 0 && K % 4 == 0 && N % 4 == 0 && K > 0;
  if (vec)
    hipLaunchKernelGGL(hand::gemm_f32_hand<true>, dim3((unsigned)tiles), dim3(hand::kGT), 0, s, A,
                       lda, B, ldb, C, ldc, M, N, K);
  else
    hipLaunchKernelGGL(hand::gemm_f32_hand<false>, dim3((unsigned)tiles), dim3(hand::kGT), 0, s,
                       A, lda, B, ldb, C, ldc, M, N, K);
  return (int)hipGetLastError();
}

// counts: two zeroed unsigned 64-bit counters in GPU memory.
int hand_e4m3_all_inputs(unsigned long long* counts, hipStream_t s) {
  hipLaunchKernelGGL(hand::e4m3_all_inputs, dim3((unsigned)hand::kCvtBlocks),
                     dim3(hand::kCvtThreads), 0, s, counts);
  return (int)hipGetLastError();
}

// counts: two zeroed unsigned 64-bit counters in GPU memory.
int hand_bf16_all_inputs(unsigned long long* counts, hipStream_t s) {
  hipLaunchKernelGGL(hand::bf16_all_inputs, dim3((unsigned)hand::kCvtBlocks),
                     dim3(hand::kCvtThreads), 0, s, counts);
  return (int)hipGetLastError();
}

}  // extern "C"
