// reduce.hip -- exact sum of int32 values into an int64 (the "block-wide
// parallel reduction" benchmark of Sec. 5, read as the full sum).
//
// One launch.  The grid is at most kReduceMaxBlocks blocks; block b takes
// the 16-byte-vector tiles b, b + grid, b + 2*grid, ... ([tiles][UNROLL]
// [BLOCK] int32x4, so every load instruction of a wave reads 1 KiB of
// consecutive memory).  Each lane sums into an int64, the wave sums with
// shuffles, the block's waves meet in LDS, and thread 0 publishes the block
// sum.  The block that finishes last (counted in the workspace header) adds
// the published sums in a fixed order, writes the result and resets the
// counter, so the workspace is ready for the next call.
//
// Integer addition is associative, so the result is the exact sum whatever
// the order.  The head (up to 3 elements before the first 16-byte boundary)
// and the tail (fewer than one tile) are summed by the last block of the
// grid with scalar loads.
#include "common.hpp"
#include "launch.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 4;                        // int32x4 per lane per tile
constexpr int kTileVec = kBlock * kUnroll;        // int32x4 per tile
constexpr int kTile = kTileVec * 4;               // int32 per tile

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* lds) {
  constexpr int NW = kBlock / kWave;
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  v = wave::sum_i64(v);
  if (lane_of_wave().index() == 0) lds[wv.index()] = v;
  sync(thread);
  int64_t s = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += lds[w];
  return s;
}

// body: the 16-byte-aligned middle of the input as ntiles full tiles;
// edge: the remaining scalars (head and tail), summed by the last block.
__global__ __launch_bounds__(kBlock) void reduce_i32_kernel(
    const i32x4* __restrict__ body, int64_t ntiles, const int32_t* __restrict__ head,
    int64_t nhead, const int32_t* __restrict__ tail, int64_t ntail, int64_t* __restrict__ out,
    WsHeader* __restrict__ hdr, uint64_t* __restrict__ partials) {
  __shared__ int64_t lds[kBlock / kWave];
  __shared__ uint32_t s_last;
  auto block = block_x();
  auto thread = thread_x<kBlock>();

  // tiles -> rounds -> threads: [ntiles][kUnroll][kBlock]
  auto tiles = array(body, ntiles * kTileVec).group<kBlock>().group<kUnroll>();

  int64_t acc = 0;
  for (idx_t t = block.index(); t < ntiles; t += block.count()) {
    auto mine = tiles.idx(t).transpose().select(thread);   // [kUnroll]
    i32x4 q[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) q[u] = __builtin_nontemporal_load(&mine[u]);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      acc += (int64_t)q[u].x + (int64_t)q[u].y + (int64_t)q[u].z + (int64_t)q[u].w;
  }
  if (block.index() == block.count() - 1) {
    auto h = array(head, nhead);
    auto tl = array(tail, ntail);
    for (idx_t i = thread.index(); i < nhead; i += kBlock) acc += h[i];
    for (idx_t i = thread.index(); i < ntail; i += kBlock) acc += tl[i];
  }
  const int64_t s = block_sum(acc, lds);

  // Publish; the release orders the block sum before the count.
  if (thread.index() == 0) {
    store_status(&partials[block.index()], (uint64_t)s);
    const uint32_t prev =
        __hip_atomic_fetch_add(&hdr->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == (uint32_t)(block.count() - 1));
  }
  sync(thread);
  if (!s_last) return;

  // Last block: sum the published block sums.
  auto parts = array(partials, block.count());
  int64_t acc2 = 0;
  for (idx_t b = thread.index(); b < parts.extent(); b += kBlock)
    acc2 += (int64_t)load_status(&parts[b]);
  sync(thread);   // lds is reused
  const int64_t total = block_sum(acc2, lds);
  if (thread.index() == 0) {
    out[0] = total;
    store_u32(&hdr->done, 0u);
  }
}

}  // namespace

namespace launch {

size_t reduce_i32_workspace() { return sizeof(WsHeader) + sizeof(uint64_t) * kReduceMaxBlocks; }

hipError_t reduce_i32(const int32_t* in, int64_t n, int64_t* out, void* ws, hipStream_t s) {
  // Split the input at the first 16-byte boundary and after the last full tile.
  const uintptr_t addr = (uintptr_t)in;
  int64_t nhead = (int64_t)(((16 - (addr & 15)) & 15) / 4);
  if (nhead > n) nhead = n;
  const int64_t rest = n - nhead;
  const int64_t ntiles = rest / kTile;
  const int64_t ntail = rest - ntiles * kTile;
  int64_t grid = ntiles < kReduceMaxBlocks ? ntiles : kReduceMaxBlocks;
  if (grid < 1) grid = 1;
  WsHeader* hdr = (WsHeader*)ws;
  uint64_t* partials = (uint64_t*)((char*)ws + sizeof(WsHeader));
  hipLaunchKernelGGL(reduce_i32_kernel, dim3((unsigned)grid), dim3(kBlock), 0, s,
                     (const i32x4*)(in + nhead), ntiles, in, nhead, in + nhead + ntiles * kTile,
                     ntail, out, hdr, partials);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
