// scan.hip -- inclusive prefix sum of int32 values, wrapping modulo 2^32
// (the "scan" benchmark of Sec. 5).
//
// The paper's scan runs as two kernels; here it is one pass over the data
// (read n, write n) with decoupled look-back between tiles:
//
//   * Block b scans tile b.  Blocks are dispatched in the order of their ids
//     (round-robin over the XCDs, in order within each), so a tile only
//     waits on tiles whose blocks are already running; no shared counter is
//     needed to hand out tile ids.
//   * A tile is [waves][rounds][64 lanes][4] int32: each wave owns a
//     contiguous sub-tile and reads it with 16-byte loads, a whole wave
//     covering 1 KiB per round.  Per round a lane adds its 4 values in order,
//     the wave scans the lane totals with DPP, and the running wave total
//     carries into the next round.
//   * The tile aggregate is formed first (lane sums, a DPP wave sum, LDS
//     across waves) and published in the tile's status word at once.  Wave 0
//     then walks back over the predecessors' words, 256 per poll (four per
//     lane), until it meets an inclusive prefix, and publishes the tile's own
//     inclusive prefix; meanwhile the other waves scan their sub-tiles.
//   * Tiles are large (8192 to 65536 elements, picked per size class by the
//     tuning table) so that the prefixes travel faster than the tiles are
//     consumed: a poll costs a device-coherent round trip across XCDs, and
//     with the look-back removed every shape streams at the copy ceiling, so
//     the look-back is what the tile size has to amortise.
//   * A status word holds {flag:2, generation tag:30, value:32} and is read
//     and written with single 64-bit relaxed atomics, so no fence is needed
//     to make the value visible to blocks on other XCDs.  Words whose tag is
//     not the current generation read as "not ready", which is what lets the
//     next call reuse the workspace without a clearing pass.  The last tile
//     also clears the words an earlier, larger call left past this call's
//     tiles, so only the previous call's tag or zero is ever found.
//
// Integer addition modulo 2^32 is associative, so the result equals the
// sequential definition bit for bit.
#include "common.hpp"
#include "launch.hpp"
#include "layouts.hpp"
#include "lookback.hpp"
#include "tuning.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

using namespace scan_detail;

// A tile is kBlock threads x kRounds rounds x 4 int32; kNt selects
// non-temporal (streaming) global loads and stores.
template <int kBlock, int kRounds, bool kNt>
struct ScanCfg {
  static constexpr int block = kBlock;
  static constexpr int rounds = kRounds;
  static constexpr bool nt = kNt;
  static constexpr int waves = kBlock / kWave;
  static constexpr int tile = waves * kWave * 4 * kRounds;   // int32 per tile
};
constexpr int kMinTile = 8192;   // smallest tile of any configuration below

// A tile's values: [tiles][waves][rounds][lanes] of 4-element groups; the
// last tile may be partial, so the nominal extent is rounded up and
// positions >= n read as zero.
template <class C, bool kVec>
__device__ __forceinline__ void load_tile(const int32_t* __restrict__ in, int64_t n, idx_t tile,
                                          idx_t ntiles, uint32_t (&x)[C::rounds][4]) {
  constexpr int R = C::rounds, NW = C::waves, TILE = C::tile;
  auto wv = wave_of_block<C::block>();
  auto lane = lane_of_wave();
  if (kVec && (tile + 1) * TILE <= n) {
    auto mine = layout::wave_striped<NW, R>(array((const i32x4*)in, ntiles * (TILE / 4)), tile,
                                            wv, lane);                   // [rounds]
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const i32x4 q = load16<C::nt>(&mine[r]);
      x[r][0] = (uint32_t)q.x; x[r][1] = (uint32_t)q.y;
      x[r][2] = (uint32_t)q.z; x[r][3] = (uint32_t)q.w;
    }
  } else {
    auto mine = layout::wave_striped<NW, R>(array(in, ntiles * TILE).group<4>(), tile, wv,
                                            lane);                       // [rounds][4]
#pragma unroll
    for (int r = 0; r < R; ++r) {
      auto grp = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[r][k] = grp.pos(k) < n ? (uint32_t)grp[k] : 0u;
    }
  }
}

// The scan of one loaded tile, from its aggregate to its stores.  kExcl:
// exclusive scan (out[i] = sum of the elements before i), the same pass
// with each group of four shifted by one place after its in-group scan.
// The LDS words are reused by the block's next tile: every read of them
// comes before the second barrier here.
constexpr int kWaveMax = 1024 / kWave;   // waves of the largest block
struct alignas(16) ScanLds {
  uint32_t wtot[kWaveMax];   // first: 16-byte aligned, read as 16-byte words
  uint32_t prefix;
};
template <class C, bool kVec, bool kExcl>
__device__ __forceinline__ void scan_tile(int32_t* __restrict__ out, int64_t n, idx_t tile,
                                          idx_t ntiles, CallState call,
                                          WsHeader* __restrict__ hdr,
                                          uint64_t* __restrict__ status,
                                          uint32_t (&x)[C::rounds][4], ScanLds& sl) {
  constexpr int R = C::rounds, NW = C::waves, TILE = C::tile;
  auto thread = thread_x<C::block>();
  auto wv = wave_of_block<C::block>();
  auto lane = lane_of_wave();
  const bool full = kVec && (tile + 1) * TILE <= n;

  // Tile aggregate first, so that it can be published before the scan.
  uint32_t lsum = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) lsum += x[r][0] + x[r][1] + x[r][2] + x[r][3];
  const uint32_t wsum = wave::sum_u32(lsum);
  if (lane.index() == 0) sl.wtot[wv.index()] = wsum;
  sync(thread);
  uint32_t wex = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t v = sl.wtot[w];
    wex += (w < wv.index()) ? v : 0u;
    agg += v;
  }

  // Wave 0 publishes and looks back while the other waves scan.
  auto st = array(status, ntiles);
  if (wv.index() == 0) {
    uint32_t excl = 0;
    if (tile == 0) {
      if (lane.index() == 0) store_status(&st[0], pack(kFlagPrefix, call.gen, agg));
    } else {
      if (lane.index() == 0) store_status(&st[tile], pack(kFlagAggregate, call.gen, agg));
      excl = look_back(status, tile, call.gen, call.polls, hdr);
      if (lane.index() == 0) store_status(&st[tile], pack(kFlagPrefix, call.gen, excl + agg));
    }
    if (lane.index() == 0) sl.prefix = excl;
    if (tile == ntiles - 1) {
      // Every tile before the last has published, so every block of this
      // call has read the generation: the last tile may advance it, and
      // clear what the previous call left past this call's tiles.
      const uint64_t hw = __hip_atomic_load(&hdr->hw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      clear_words<kWave>(status, (uint64_t)ntiles, hw, lane.index());
      if (lane.index() == 0) {
        __hip_atomic_store(&hdr->hw, (uint64_t)ntiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        store_u32(&hdr->gen, next_gen(call.gen));
      }
    }
  }

  // Scan inside the wave's sub-tile, round by round.
  uint32_t carry = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    x[r][1] += x[r][0];
    x[r][2] += x[r][1];
    x[r][3] += x[r][2];
    const uint32_t t = x[r][3];
    const uint32_t incl = wave::inclusive_add_u32(t);
    const uint32_t ex = carry + incl - t;
    if constexpr (kExcl) {
      x[r][3] = x[r][2];
      x[r][2] = x[r][1];
      x[r][1] = x[r][0];
      x[r][0] = 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[r][k] += ex;
    carry += wave::lane_read_u32(incl, kWave - 1);
  }
  sync(thread);
  const uint32_t add = sl.prefix + wex;

  if (full) {
    auto mine = layout::wave_striped<NW, R>(array((i32x4*)out, ntiles * (TILE / 4)), tile, wv,
                                            lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      i32x4 q;
      q.x = (int32_t)(x[r][0] + add); q.y = (int32_t)(x[r][1] + add);
      q.z = (int32_t)(x[r][2] + add); q.w = (int32_t)(x[r][3] + add);
      store16<C::nt>(q, &mine[r]);
    }
  } else {
    auto mine = layout::wave_striped<NW, R>(array(out, ntiles * TILE).group<4>(), tile, wv, lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      auto grp = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (grp.pos(k) < n) grp[k] = (int32_t)(x[r][k] + add);
    }
  }
}

// One block per tile.
template <class C, bool kVec, bool kExcl>
__global__ __launch_bounds__(C::block) void scan_i32_kernel(const int32_t* __restrict__ in,
                                                            int32_t* __restrict__ out, int64_t n,
                                                            WsHeader* __restrict__ hdr,
                                                            uint64_t* __restrict__ status) {
  __shared__ CallState s_call;
  __shared__ ScanLds sl;
  auto tile_res = block_x();
  auto thread = thread_x<C::block>();
  if (thread.index() == 0) s_call = read_call_state(hdr);
  sync(thread);
  const CallState call = s_call;
  uint32_t x[C::rounds][4];
  load_tile<C, kVec>(in, n, tile_res.index(), tile_res.count(), x);
  scan_tile<C, kVec, kExcl>(out, n, tile_res.index(), tile_res.count(), call, hdr, status, x, sl);
}

template <class C, bool kExcl>
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s) {
  const int64_t ntiles = (n + C::tile - 1) / C::tile;
  WsHeader* hdr = (WsHeader*)ws;
  uint64_t* status = (uint64_t*)((char*)ws + sizeof(WsHeader));
  const bool vec = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL((scan_i32_kernel<C, true, kExcl>), dim3((unsigned)ntiles), dim3(C::block),
                       0, s, in, out, n, hdr, status);
  else
    hipLaunchKernelGGL((scan_i32_kernel<C, false, kExcl>), dim3((unsigned)ntiles), dim3(C::block),
                       0, s, in, out, n, hdr, status);
  return hipGetLastError();
}

template <bool kExcl>
hipError_t scan_any(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s) {
  switch (tune::get(tune::kScanI32, tune::size_class(tune::kScanI32, n))) {
    case 1: return launch_scan<ScanCfg<256, 8, false>, kExcl>(in, out, n, ws, s);
    case 2: return launch_scan<ScanCfg<512, 8, true>, kExcl>(in, out, n, ws, s);
    case 3: return launch_scan<ScanCfg<256, 16, true>, kExcl>(in, out, n, ws, s);
    case 4: return launch_scan<ScanCfg<1024, 4, true>, kExcl>(in, out, n, ws, s);
    case 5: return launch_scan<ScanCfg<512, 4, true>, kExcl>(in, out, n, ws, s);
    case 6: return launch_scan<ScanCfg<256, 32, true>, kExcl>(in, out, n, ws, s);
    case 7: return launch_scan<ScanCfg<512, 16, true>, kExcl>(in, out, n, ws, s);
    case 8: return launch_scan<ScanCfg<1024, 8, true>, kExcl>(in, out, n, ws, s);
    case 9: return launch_scan<ScanCfg<512, 32, true>, kExcl>(in, out, n, ws, s);
    case 10: return launch_scan<ScanCfg<1024, 16, true>, kExcl>(in, out, n, ws, s);
    default: return launch_scan<ScanCfg<256, 8, true>, kExcl>(in, out, n, ws, s);
  }
}

constexpr const char* kNames[] = {"b256_r8_nt", "b256_r8", "b512_r8_nt", "b256_r16_nt",
                                   "b1024_r4_nt", "b512_r4_nt", "b256_r32_nt", "b512_r16_nt",
                                   "b1024_r8_nt", "b512_r32_nt", "b1024_r16_nt"};
constexpr int kDefaults[tune::kClasses] = {0, 0, 0, 0};
const bool kRegistered =
    (tune::register_op(tune::kScanI32, "scan_i32", 11, kNames, kDefaults), true);

}  // namespace

namespace launch {

size_t scan_i32_workspace(int64_t n) {
  const int64_t ntiles = (n + kMinTile - 1) / kMinTile;
  return sizeof(WsHeader) + sizeof(uint64_t) * (size_t)(ntiles > 0 ? ntiles : 1);
}

hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s,
                    bool exclusive) {
  if (n == 0) return hipSuccess;
  (void)kRegistered;
  return exclusive ? scan_any<true>(in, out, n, ws, s) : scan_any<false>(in, out, n, ws, s);
}

}  // namespace launch
}  // namespace desc
