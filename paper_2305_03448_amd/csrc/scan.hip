// scan.hip -- inclusive prefix sum of int32 values, wrapping modulo 2^32
// (the "scan" benchmark of Sec. 5).
//
// The paper's scan runs as two kernels; here it is one pass over the data
// (read n, write n) with decoupled look-back between tiles:
//
//   * A block takes the next tile id from a counter in the workspace, so a
//     tile only ever waits on tiles whose blocks are already running.
//   * A tile is [waves][rounds][64 lanes][4] int32: each wave owns a
//     contiguous sub-tile and reads it with 16-byte loads, a whole wave
//     covering 1 KiB per round.  Per round a lane adds its 4 values in order,
//     the wave scans the lane totals with DPP, and the running wave total
//     carries into the next round.
//   * Wave totals meet in LDS; the tile aggregate is published at once in
//     the tile's status word, then wave 0 walks back over the predecessors'
//     words 64 at a time until it meets an inclusive prefix, and publishes
//     the tile's own inclusive prefix.
//   * A status word holds {flag:2, generation tag:30, value:32} and is read
//     and written with single 64-bit relaxed atomics, so no fence is needed
//     to make the value visible to blocks on other XCDs.  Words whose tag is
//     not the current generation read as "not ready", which is what lets the
//     next call reuse the workspace without a clearing pass.
//
// Integer addition modulo 2^32 is associative, so the result equals the
// sequential definition bit for bit.
#include "common.hpp"
#include "launch.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 4;
constexpr int kWaves = kBlock / kWave;
constexpr int kSub = kWave * 4 * kRounds;        // int32 per wave
constexpr int kTile = kWaves * kSub;             // int32 per tile

constexpr uint64_t kFlagAggregate = 1, kFlagPrefix = 2;
constexpr uint32_t kTagMask = 0x3fffffffu;

__device__ __forceinline__ uint64_t pack(uint64_t flag, uint32_t gen, uint32_t v) {
  return (flag << 62) | ((uint64_t)(gen & kTagMask) << 32) | (uint64_t)v;
}

// Exclusive prefix of tile `tile` from the status words of its predecessors.
// Called by one whole wave; the result is valid in every lane.
__device__ __forceinline__ uint32_t look_back(const uint64_t* __restrict__ status, idx_t tile,
                                              uint32_t gen, WsHeader* __restrict__ hdr) {
  const int lane = wave::lane_id();
  const uint32_t tag = gen & kTagMask;
  uint32_t excl = 0;
  idx_t pos = tile - 1;
  for (uint32_t polls = 0;; ++polls) {
    if (polls == kSpinLimit) {     // inconsistent workspace: give up, flag it
      if (lane == 0) store_u32(&hdr->error, 1u);
      break;
    }
    const idx_t j = pos - lane;
    const uint64_t s = j >= 0 ? load_status(&status[j]) : pack(kFlagPrefix, gen, 0u);
    const uint32_t flag = (uint32_t)(s >> 62);
    const bool valid = flag != 0 && (uint32_t)((s >> 32) & kTagMask) == tag;
    const uint64_t pmask = __ballot(valid && flag == kFlagPrefix);
    const uint64_t imask = __ballot(!valid);
    const int first_p = pmask ? __builtin_ctzll(pmask) : 63;
    const uint64_t need = first_p == 63 ? ~0ull : ((2ull << first_p) - 1);
    if (imask & need) {            // a predecessor we need has not published yet
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += wave::sum_u32(lane <= first_p ? (uint32_t)s : 0u);
    if (pmask) break;
    pos -= kWave;
  }
  return excl;
}

// The block that finishes last prepares the workspace for the next call.
__device__ __forceinline__ void finish(WsHeader* hdr, uint32_t gen, idx_t ntiles) {
  const uint32_t d = fetch_add_u32(&hdr->done, 1u);
  if (d == (uint32_t)(ntiles - 1)) {
    store_u32(&hdr->next, 0u);
    store_u32(&hdr->done, 0u);
    store_u32(&hdr->gen, gen + 1u);
  }
}

template <bool kVec>
__global__ __launch_bounds__(kBlock) void scan_i32_kernel(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out, int64_t n,
                                                          WsHeader* __restrict__ hdr,
                                                          uint64_t* __restrict__ status) {
  __shared__ uint32_t s_tile, s_gen, s_prefix;
  __shared__ uint32_t s_wtot[kWaves];
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  auto lane = lane_of_wave();
  const idx_t ntiles = block_x().count();

  if (thread.index() == 0) {
    s_tile = fetch_add_u32(&hdr->next, 1u);
    s_gen = load_u32(&hdr->gen);
  }
  sync(thread);
  const idx_t tile = s_tile;
  const uint32_t gen = s_gen;
  if (tile >= ntiles) {          // only possible with a workspace that was not zeroed
    if (thread.index() == 0) {
      store_u32(&hdr->error, 1u);
      finish(hdr, gen, ntiles);
    }
    return;
  }

  // [tiles][waves][rounds][lanes] of 4-element groups; the last tile may be
  // partial, so the nominal extent is rounded up and positions >= n guarded.
  const bool full = kVec && (tile + 1) * kTile <= n;
  uint32_t x[kRounds][4];
  if (full) {
    auto mine = array((const i32x4*)in, ntiles * (kTile / 4))
                    .group<kWave>().group<kRounds>().group<kWaves>()
                    .idx(tile).select(wv).transpose().select(lane);     // [rounds]
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const i32x4 q = __builtin_nontemporal_load(&mine[r]);
      x[r][0] = (uint32_t)q.x; x[r][1] = (uint32_t)q.y;
      x[r][2] = (uint32_t)q.z; x[r][3] = (uint32_t)q.w;
    }
  } else {
    auto mine = array(in, ntiles * kTile)
                    .group<4>().group<kWave>().group<kRounds>().group<kWaves>()
                    .idx(tile).select(wv).transpose().select(lane);     // [rounds][4]
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      auto grp = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[r][k] = grp.pos(k) < n ? (uint32_t)grp[k] : 0u;
    }
  }

  // Scan inside the wave's sub-tile, round by round.
  uint32_t carry = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    x[r][1] += x[r][0];
    x[r][2] += x[r][1];
    x[r][3] += x[r][2];
    const uint32_t t = x[r][3];
    const uint32_t incl = wave::inclusive_add_u32(t);
    const uint32_t ex = carry + incl - t;
#pragma unroll
    for (int k = 0; k < 4; ++k) x[r][k] += ex;
    carry += wave::lane_read_u32(incl, kWave - 1);
  }
  if (lane.index() == 0) s_wtot[wv.index()] = carry;
  sync(thread);
  uint32_t wex = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t v = s_wtot[w];
    wex += (w < wv.index()) ? v : 0u;
    agg += v;
  }

  // Publish and look back (wave 0).
  auto st = array(status, ntiles);
  if (wv.index() == 0) {
    uint32_t excl = 0;
    if (tile == 0) {
      if (lane.index() == 0) store_status(&st[0], pack(kFlagPrefix, gen, agg));
    } else {
      if (lane.index() == 0) store_status(&st[tile], pack(kFlagAggregate, gen, agg));
      excl = look_back(status, tile, gen, hdr);
      if (lane.index() == 0) store_status(&st[tile], pack(kFlagPrefix, gen, excl + agg));
    }
    if (lane.index() == 0) s_prefix = excl;
  }
  sync(thread);
  const uint32_t add = s_prefix + wex;

  if (full) {
    auto mine = array((i32x4*)out, ntiles * (kTile / 4))
                    .group<kWave>().group<kRounds>().group<kWaves>()
                    .idx(tile).select(wv).transpose().select(lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      i32x4 q;
      q.x = (int32_t)(x[r][0] + add); q.y = (int32_t)(x[r][1] + add);
      q.z = (int32_t)(x[r][2] + add); q.w = (int32_t)(x[r][3] + add);
      __builtin_nontemporal_store(q, &mine[r]);
    }
  } else {
    auto mine = array(out, ntiles * kTile)
                    .group<4>().group<kWave>().group<kRounds>().group<kWaves>()
                    .idx(tile).select(wv).transpose().select(lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      auto grp = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (grp.pos(k) < n) grp[k] = (int32_t)(x[r][k] + add);
    }
  }

  if (thread.index() == 0) finish(hdr, gen, ntiles);
}

}  // namespace

namespace launch {

size_t scan_i32_workspace(int64_t n) {
  const int64_t ntiles = (n + kTile - 1) / kTile;
  return sizeof(WsHeader) + sizeof(uint64_t) * (size_t)(ntiles > 0 ? ntiles : 1);
}

hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t ntiles = (n + kTile - 1) / kTile;
  WsHeader* hdr = (WsHeader*)ws;
  uint64_t* status = (uint64_t*)((char*)ws + sizeof(WsHeader));
  const bool vec = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(scan_i32_kernel<true>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, in, out,
                       n, hdr, status);
  else
    hipLaunchKernelGGL(scan_i32_kernel<false>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, in,
                       out, n, hdr, status);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
