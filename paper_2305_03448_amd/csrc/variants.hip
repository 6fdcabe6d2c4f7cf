// variants.hip -- the paper's own forms of the reduction and the scan of
// Sec. 5, next to the single-pass forms of reduce.hip and scan.hip:
//
//   block-wide reduction: every block sums its chunk of the input and writes
//     one exact int64 per chunk (no grid-wide combination).  Inside the block
//     the 256 lane sums meet in LDS in a tree: at each step the block is
//     split at k, the first k threads add element i + k into element i, and
//     the whole block synchronises after the split -- a barrier may not sit
//     inside a split half (Sec. 2, Sec. 3.1), and `sync` refuses to compile
//     there.
//
//   two-kernel scan (reduce, then scan): kernel 1 writes the sum of every
//     tile; kernel 2 gives each tile the sum of the tile sums before it (a
//     block-wide reduction over them) and scans the tile with that carry.
//     The data is read twice and written once (3n words against the single
//     pass's 2n); no block waits on another, so there is no look-back and no
//     workspace state.
//
// Both use the views of layouts.hpp for the tile layout; integer addition is
// associative, so results equal the sequential definitions bit for bit.
#include "common.hpp"
#include "launch.hpp"
#include "layouts.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

// ----------------------------------------------------------------- block-wide reduction
constexpr int kRBlock = 256;

// Chunk b is in[b * E, min(n, (b + 1) * E)); E is a multiple of 1024, so a
// chunk is whole rounds of [256 threads][4], read as int32x4 when the input
// is 16-byte aligned (vec) and the chunk is full.
template <bool kVec>
__global__ __launch_bounds__(kRBlock) void reduce_blocks_kernel(const int32_t* __restrict__ in,
                                                               int64_t n, int64_t E,
                                                               int64_t* __restrict__ out) {
  __shared__ int64_t part[kRBlock];
  auto block = block_x();
  auto thread = thread_x<kRBlock>();
  const idx_t b0 = block.index() * E;
  const idx_t len = (n - b0) < E ? (n - b0) : E;
  const idx_t rounds = E / (kRBlock * 4);
  int64_t acc = 0;
  if (kVec && len == E) {
    // the chunk as [rounds][256 threads] int32x4; thread t takes column t
    auto rows = array((const i32x4*)in, n / 4).snd(b0 / 4).fst(E / 4).template group<kRBlock>();
#pragma unroll 8
    for (idx_t r = 0; r < rounds; ++r) {
      const i32x4 q = __builtin_nontemporal_load(&rows.idx(r).select(thread).get());
      acc += (int64_t)q.x + (int64_t)q.y + (int64_t)q.z + (int64_t)q.w;
    }
  } else {
    auto chunk = array(in, 0).snd(b0);
    for (idx_t i = thread.index(); i < len; i += kRBlock) acc += chunk[i];
  }
  // tree over the 256 lane sums: split at k, first half adds the second
  auto p = array(part, kRBlock);
  p[thread.index()] = acc;
  sync(thread);
#pragma unroll
  for (int k = kRBlock / 2; k >= 1; k /= 2) {
    split(thread, k,
          [&](auto first) { p.fst(k).select(first).get() += p.snd(k).fst(k).select(first).get(); },
          [](auto) {});
    sync(thread);
  }
  if (thread.index() == 0) array(out, block.count())[block.index()] = p[0];
}

// ----------------------------------------------------------------- two-kernel scan
// A tile is 1024 threads x 16 rounds x 4 int32 (65536), laid out as the
// single-pass scan's tiles: [waves][rounds][lanes][4].
constexpr int kSBlock = 1024, kSRounds = 16, kSWaves = kSBlock / kWave;
constexpr int kSTile = kSBlock * kSRounds * 4;

template <bool kVec>
__device__ __forceinline__ void load_tile(const int32_t* in, int64_t n, idx_t tile,
                                          idx_t ntiles, uint32_t (&x)[kSRounds][4]) {
  auto wv = wave_of_block<kSBlock>();
  auto lane = lane_of_wave();
  if (kVec && (tile + 1) * kSTile <= n) {
    auto mine = layout::wave_striped<kSWaves, kSRounds>(
        array((const i32x4*)in, ntiles * (kSTile / 4)), tile, wv, lane);
#pragma unroll
    for (int r = 0; r < kSRounds; ++r) {
      const i32x4 q = __builtin_nontemporal_load(&mine[r]);
      x[r][0] = (uint32_t)q.x; x[r][1] = (uint32_t)q.y;
      x[r][2] = (uint32_t)q.z; x[r][3] = (uint32_t)q.w;
    }
  } else {
    auto mine = layout::wave_striped<kSWaves, kSRounds>(
        array(in, ntiles * kSTile).group<4>(), tile, wv, lane);
#pragma unroll
    for (int r = 0; r < kSRounds; ++r) {
      auto grp = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[r][k] = grp.pos(k) < n ? (uint32_t)grp[k] : 0u;
    }
  }
}

// Sum of one value per thread over the block (wrapping), valid in every thread.
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* lds) {
  auto thread = thread_x<kSBlock>();
  auto wv = wave_of_block<kSBlock>();
  const uint32_t w = wave::sum_u32(v);
  if (lane_of_wave().index() == 0) lds[wv.index()] = w;
  sync(thread);
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kSWaves; ++i) s += lds[i];
  sync(thread);
  return s;
}

// Kernel 1: the sum of every tile.
template <bool kVec>
__global__ __launch_bounds__(kSBlock) void tile_sums_kernel(const int32_t* __restrict__ in,
                                                            int64_t n,
                                                            uint32_t* __restrict__ sums) {
  __shared__ uint32_t lds[kSWaves];
  auto tile = block_x();
  uint32_t x[kSRounds][4];
  load_tile<kVec>(in, n, tile.index(), tile.count(), x);
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kSRounds; ++r) s += x[r][0] + x[r][1] + x[r][2] + x[r][3];
  s = block_sum_u32(s, lds);
  if (thread_x<kSBlock>().index() == 0) array(sums, tile.count())[tile.index()] = s;
}

// Kernel 2: carry = sum of the tile sums before this tile, then the tile's
// inclusive scan plus the carry.
template <bool kVec>
__global__ __launch_bounds__(kSBlock) void scan_carry_kernel(const int32_t* __restrict__ in,
                                                             int32_t* __restrict__ out, int64_t n,
                                                             const uint32_t* __restrict__ sums) {
  __shared__ uint32_t lds[kSWaves];
  auto tile = block_x();
  auto thread = thread_x<kSBlock>();
  auto wv = wave_of_block<kSBlock>();
  auto lane = lane_of_wave();
  const idx_t ntiles = tile.count(), t = tile.index();
  uint32_t x[kSRounds][4];
  load_tile<kVec>(in, n, t, ntiles, x);
  // the carry: tiles [0, t) summed by the whole block
  auto before = array(sums, ntiles).fst(t);
  uint32_t c = 0;
  for (idx_t j = thread.index(); j < t; j += kSBlock) c += before[j];
  const uint32_t carry = block_sum_u32(c, lds);
  // wave sums for the offsets between the waves of the tile
  uint32_t lsum = 0;
#pragma unroll
  for (int r = 0; r < kSRounds; ++r) lsum += x[r][0] + x[r][1] + x[r][2] + x[r][3];
  const uint32_t wsum = wave::sum_u32(lsum);
  if (lane.index() == 0) lds[wv.index()] = wsum;
  sync(thread);
  uint32_t wex = 0;
#pragma unroll
  for (int w = 0; w < kSWaves; ++w) wex += (w < wv.index()) ? lds[w] : 0u;
  uint32_t run = 0;
#pragma unroll
  for (int r = 0; r < kSRounds; ++r) {
    x[r][1] += x[r][0];
    x[r][2] += x[r][1];
    x[r][3] += x[r][2];
    const uint32_t tt = x[r][3];
    const uint32_t incl = wave::inclusive_add_u32(tt);
    const uint32_t ex = run + incl - tt;
#pragma unroll
    for (int k = 0; k < 4; ++k) x[r][k] += ex;
    run += wave::lane_read_u32(incl, kWave - 1);
  }
  const uint32_t add = carry + wex;
  if (kVec && (t + 1) * kSTile <= n) {
    auto mine = layout::wave_striped<kSWaves, kSRounds>(
        array((i32x4*)out, ntiles * (kSTile / 4)), t, wv, lane);
#pragma unroll
    for (int r = 0; r < kSRounds; ++r) {
      i32x4 q;
      q.x = (int32_t)(x[r][0] + add); q.y = (int32_t)(x[r][1] + add);
      q.z = (int32_t)(x[r][2] + add); q.w = (int32_t)(x[r][3] + add);
      __builtin_nontemporal_store(q, &mine[r]);
    }
  } else {
    auto mine = layout::wave_striped<kSWaves, kSRounds>(array(out, ntiles * kSTile).group<4>(),
                                                        t, wv, lane);
#pragma unroll
    for (int r = 0; r < kSRounds; ++r) {
      auto grp = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (grp.pos(k) < n) grp[k] = (int32_t)(x[r][k] + add);
    }
  }
}

}  // namespace

namespace launch {

hipError_t reduce_blocks_i32(const int32_t* in, int64_t n, int64_t E, int64_t* out,
                             hipStream_t s) {
  const int64_t blocks = (n + E - 1) / E;
  if (blocks == 0) return hipSuccess;
  if ((((uintptr_t)in) & 15) == 0)
    hipLaunchKernelGGL(reduce_blocks_kernel<true>, dim3((unsigned)blocks), dim3(kRBlock), 0, s,
                       in, n, E, out);
  else
    hipLaunchKernelGGL(reduce_blocks_kernel<false>, dim3((unsigned)blocks), dim3(kRBlock), 0, s,
                       in, n, E, out);
  return hipGetLastError();
}

size_t scan_two_pass_workspace(int64_t n) {
  const int64_t ntiles = (n + kSTile - 1) / kSTile;
  return 4 * (size_t)(ntiles > 0 ? ntiles : 1);
}

hipError_t scan_two_pass_i32(const int32_t* in, int32_t* out, int64_t n, void* ws,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t ntiles = (n + kSTile - 1) / kSTile;
  uint32_t* sums = (uint32_t*)ws;
  if ((((uintptr_t)in | (uintptr_t)out) & 15) == 0) {
    hipLaunchKernelGGL(tile_sums_kernel<true>, dim3((unsigned)ntiles), dim3(kSBlock), 0, s, in,
                       n, sums);
    hipLaunchKernelGGL(scan_carry_kernel<true>, dim3((unsigned)ntiles), dim3(kSBlock), 0, s, in,
                       out, n, sums);
  } else {
    hipLaunchKernelGGL(tile_sums_kernel<false>, dim3((unsigned)ntiles), dim3(kSBlock), 0, s, in,
                       n, sums);
    hipLaunchKernelGGL(scan_carry_kernel<false>, dim3((unsigned)ntiles), dim3(kSBlock), 0, s, in,
                       out, n, sums);
  }
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
