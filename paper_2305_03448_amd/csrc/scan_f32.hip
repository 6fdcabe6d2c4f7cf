// scan_f32.hip -- inclusive prefix sum of float32 values (the scan of Sec. 5
// over floats), accumulated in FP64 and rounded once to float32, in an order
// fixed by the element indices and n alone: equal inputs give bit-equal
// outputs on every run and at every address.
//
// A single pass (read n, write n) like the integer scan, but its look-back
// cannot take "the nearest inclusive prefix that has been published": which
// one that is depends on timing, and floating-point addition is not
// associative.  Here every tile's carry is a fixed expression:
//
//   * Tiles of 65536 elements, [16 waves][16 rounds][64 lanes][4]: each wave
//     owns a contiguous sub-tile, as in the integer scan.  T tiles; tile t
//     is in group g = t / 64 at place p = t % 64.
//   * A_t, the tile aggregate: lane sums (the lane's 64 elements added in
//     order from 0.0), a butterfly over the wave (lane i adds lane i ^ 32,
//     then i ^ 16, ..., 1), and the 16 wave values added in order from 0.0.
//   * Q_g, the sum of every tile before group g: Q_0 = 0 and
//     Q_{g+1} = Q_g + S_g, S_g the butterfly over the group's 64 aggregates.
//     The last tile of group g publishes Q_{g+1}; so the serial chain
//     advances one group (64 tiles) per hand-over, not one tile.
//   * The carry of tile t: P_t = Q_g + E_p, E_p the butterfly over the
//     aggregates of places 0 .. p-1 of the group (zeros elsewhere).
//   * Inside the tile, for the element at (wave w, round r, lane l, e):
//     s_e = the lane's four values added in order; I_l = the wave's
//     inclusive scan of s_3 (DPP row shifts 1, 2, 4, 8, then the row
//     broadcasts of lanes 15 and 31); X_l = I_{l-1} (0 for lane 0);
//     C_r = c_r + X_l with c_0 = 0, c_{r+1} = c_r + I_63; B_w = P_t + wex_w,
//     wex_w the wave values of waves before w added in order from 0.0.
//     The output is fl32(B_w + (C_r + s_e)).
//
// The error against the exact prefix S_i is at most 2^-24 |S_i| (the final
// rounding) + 2^-149 + d 2^-53 sum_{k<=i} |x_k|, d = ceil(T / 64) + 160 the
// longest chain of FP64 additions.  Zero prefixes come out as +0.
//
// Hand-over as in the other reductions: each published FP64 value is two
// 64-bit words {tag:32, half:32} (per tile: its aggregate; per group: Q),
// written and read with single relaxed atomics, the tag naming the call's
// generation.  Tile t waits only on tiles before it (blocks are dispatched in
// order); the last tile advances the generation once everything before it
// has published.  Every word of a call's region (T aggregates, then one Q per
// group, the last, partial group's included) is written by the call, and the
// last tile clears what the previous call left beyond that region, so no
// word older than the previous call survives to match a later call's tag.
#include "common.hpp"
#include "handover.hpp"
#include "launch.hpp"
#include "layouts.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / kWave;      // 16
constexpr int kRounds = 16;
constexpr int kTile = kWaves * kRounds * kWave * 4;   // 65536
constexpr int kGroup = 64;                  // tiles per look-back group

// A DPP move of an FP64 value (both halves with the same control); lanes
// that receive nothing get +0.0.
template <int kCtrl, int kRowMask, bool kBound>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, kCtrl,
                                                            kRowMask, 0xf, kBound);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), kCtrl,
                                                            kRowMask, 0xf, kBound);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Inclusive scan over the 64 lanes in the fixed DPP order.
__device__ __forceinline__ double wave_incl_f64(double v) {
  v = v + dpp_f64<wave::kRowShr1, 0xf, true>(v);
  v = v + dpp_f64<wave::kRowShr2, 0xf, true>(v);
  v = v + dpp_f64<wave::kRowShr4, 0xf, true>(v);
  v = v + dpp_f64<wave::kRowShr8, 0xf, true>(v);
  v = v + dpp_f64<wave::kRowBcast15, 0xa, false>(v);
  v = v + dpp_f64<wave::kRowBcast31, 0xc, false>(v);
  return v;
}

// Butterfly sum over the 64 lanes (the two lanes of a pair compute the same
// sum, so every lane ends with the same value).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = v + __shfl_xor(v, m, kWave);
  return v;
}

__device__ __forceinline__ double lane_read_f64(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ uint64_t bits(double v) { return (uint64_t)__double_as_longlong(v); }
__device__ __forceinline__ double from_bits(uint64_t u) { return __longlong_as_double((long long)u); }

// Marks the loaded values as changed, so that the compiler converts them to
// FP64 again where they are used next instead of keeping 64 converted
// values (128 registers) alive across the phases of the tile.
__device__ __forceinline__ void reload_barrier(float (&x)[kRounds][4]) {
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(x[r][k]));
}

struct ScanF32Lds {
  double wtot[kWaves];
  double carry;     // P_t
};

// One tile; kFull: a whole tile of 16-byte-aligned input and output, read
// and written with 16-byte accesses (else element by element, zeros past n).
// The two forms are separate inlined bodies, so that the register allocation
// of one does not constrain the other.
template <bool kFull>
__device__ __forceinline__ void scan_f32_tile(const float* __restrict__ in,
                                              float* __restrict__ out, int64_t n,
                                              WsHeader* __restrict__ hdr,
                                              uint64_t* __restrict__ aggs,
                                              uint64_t* __restrict__ groups, ScanF32Lds& sl,
                                              const CallState& s_call) {
  auto tile_res = block_x();
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  auto lane = lane_of_wave();
  const idx_t tile = tile_res.index(), ntiles = tile_res.count();

  // [tiles][waves][rounds][lanes] groups of four; this lane's [rounds]
  float x[kRounds][4];
  if constexpr (kFull) {
    auto mine = layout::wave_striped<kWaves, kRounds>(array((const f32x4*)in, ntiles * (kTile / 4)),
                                                      tile, wv, lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const f32x4 q = __builtin_nontemporal_load(&mine[r]);
      x[r][0] = q.x; x[r][1] = q.y; x[r][2] = q.z; x[r][3] = q.w;
    }
  } else {
    auto mine = layout::wave_striped<kWaves, kRounds>(array(in, ntiles * kTile).group<4>(), tile,
                                                      wv, lane);        // [rounds][4]
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      auto grp = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[r][k] = grp.pos(k) < n ? grp[k] : 0.0f;
    }
  }

  // A_t: lane sums in order, the wave butterfly, the waves in order.
  double ls = 0.0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) ls = ls + (double)x[r][k];
  reload_barrier(x);
  const double wsum = wave_sum_f64(ls);
  if (lane.index() == 0) sl.wtot[wv.index()] = wsum;
  sync(thread);   // (also publishes s_call)
  const uint32_t gen = s_call.gen;
  double wex = 0.0, agg = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const double v = sl.wtot[w];
    if (w < wv.index()) wex = wex + v;
    agg = agg + v;
  }

  // Wave 0: publish A_t, gather the group's earlier aggregates and Q_g.
  if (wv.index() == 0) {
    const uint64_t tag = handover::tag_of(gen);
    const idx_t g = tile / kGroup;
    const int p = (int)(tile % kGroup);
    auto ag = array(aggs, 2 * ntiles).group<2>();                         // [T][2]
    auto gq = array(groups, 2 * ((ntiles + kGroup - 1) / kGroup)).group<2>();
    if (lane.index() == 0) handover::publish(&ag.idx(tile)[0], tag, bits(agg));
    bool ok = true;
    uint64_t vb = bits(lane.index() == p ? agg : 0.0), qb = bits(0.0);
    if (lane.index() < p)
      ok = handover::poll(&ag.idx(layout::handover_peer<kGroup>(tile, lane.index()))[0], tag, vb,
                          s_call.polls);
    if (g > 0 && lane.index() == 0)
      ok = handover::poll(&gq.idx(g - 1)[0], tag, qb, s_call.polls) && ok;
    const double v = from_bits(vb);
    double q = from_bits(qb);
    if (__ballot(!ok) != 0 && lane.index() == 0) set_error(hdr, kDevWaitLimit);
    q = lane_read_f64(q, 0);
    const double e = wave_sum_f64(lane.index() < p ? v : 0.0);
    const double carry = q + e;
    if (layout::handover_publishes_group<kGroup>(tile, ntiles)) {   // (the last Q is not read)
      const double s = wave_sum_f64(v);
      if (lane.index() == 0) handover::publish(&gq.idx(g)[0], tag, bits(q + s));
    }
    if (lane.index() == 0) sl.carry = carry;
    if (tile == ntiles - 1) {
      // Everything before the last tile has published (the last tile has
      // seen its group's aggregates and the chain of Q), so every block of
      // this call has read the generation: advance it, and clear what the
      // previous call left past this call's region.
      const uint64_t used = (uint64_t)layout::handover_words<kGroup>(ntiles);
      const uint64_t hw = __hip_atomic_load(&hdr->hw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      clear_words<kWave>(aggs, used, hw, lane.index());
      if (lane.index() == 0) {
        __hip_atomic_store(&hdr->hw, used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        store_u32(&hdr->gen, next_gen(gen));
      }
    }
  }

  // Per round: C_r = c_r + X_l, kept until the carry is known.
  double cr[kRounds];
  double c = 0.0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const double s3 = (((double)x[r][0] + (double)x[r][1]) + (double)x[r][2]) + (double)x[r][3];
    const double incl = wave_incl_f64(s3);
    const double xl = __shfl_up(incl, 1, kWave);
    cr[r] = c + (lane.index() == 0 ? 0.0 : xl);
    c = c + lane_read_f64(incl, kWave - 1);
  }
  reload_barrier(x);
  sync(thread);
  const double base = sl.carry + wex;

  // fl32(B_w + (C_r + s_e)), stored.
  if constexpr (kFull) {
    auto mine = layout::wave_striped<kWaves, kRounds>(array((f32x4*)out, ntiles * (kTile / 4)),
                                                      tile, wv, lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      double s = (double)x[r][0];
      f32x4 y;
      y.x = (float)(base + (cr[r] + s));
      s = s + (double)x[r][1];
      y.y = (float)(base + (cr[r] + s));
      s = s + (double)x[r][2];
      y.z = (float)(base + (cr[r] + s));
      s = s + (double)x[r][3];
      y.w = (float)(base + (cr[r] + s));
      __builtin_nontemporal_store(y, &mine[r]);
    }
  } else {
    auto mine = layout::wave_striped<kWaves, kRounds>(array(out, ntiles * kTile).group<4>(), tile,
                                                      wv, lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      auto grp = mine.idx(r);
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s = k == 0 ? (double)x[r][0] : s + (double)x[r][k];
        if (grp.pos(k) < n) grp[k] = (float)(base + (cr[r] + s));
      }
    }
  }
}

template <bool kVec>
__global__ __launch_bounds__(kBlock) void scan_f32_kernel(const float* __restrict__ in,
                                                          float* __restrict__ out, int64_t n,
                                                          WsHeader* __restrict__ hdr,
                                                          uint64_t* __restrict__ aggs,
                                                          uint64_t* __restrict__ groups) {
  __shared__ CallState s_call;
  __shared__ ScanF32Lds sl;
  if (thread_x<kBlock>().index() == 0) s_call = read_call_state(hdr);
  if (kVec && ((int64_t)block_x().index() + 1) * kTile <= n)
    scan_f32_tile<true>(in, out, n, hdr, aggs, groups, sl, s_call);
  else
    scan_f32_tile<false>(in, out, n, hdr, aggs, groups, sl, s_call);
}

int64_t tiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

}  // namespace

namespace launch {

size_t scan_f32_workspace(int64_t n) {
  const int64_t t = tiles_of(n < 0 ? 0 : n);
  const int64_t g = (t + kGroup - 1) / kGroup;
  return sizeof(WsHeader) + 16 * (size_t)(t > 0 ? t : 1) + 16 * (size_t)(g > 0 ? g : 1);
}

hipError_t scan_f32(const float* in, float* out, int64_t n, void* ws, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t t = tiles_of(n);
  WsHeader* hdr = (WsHeader*)ws;
  uint64_t* aggs = (uint64_t*)((char*)ws + sizeof(WsHeader));
  uint64_t* groups = aggs + 2 * t;
  const bool vec = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(scan_f32_kernel<true>, dim3((unsigned)t), dim3(kBlock), 0, s, in, out, n,
                       hdr, aggs, groups);
  else
    hipLaunchKernelGGL(scan_f32_kernel<false>, dim3((unsigned)t), dim3(kBlock), 0, s, in, out, n,
                       hdr, aggs, groups);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
