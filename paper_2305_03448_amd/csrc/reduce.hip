// reduce.hip -- exact sum of int32 values into an int64 (the "block-wide
// parallel reduction" benchmark of Sec. 5, read as the full sum).
//
// One launch.  Block b takes the 16-byte-vector tiles b, b + grid,
// b + 2*grid, ... ([tiles][UNROLL][BLOCK] int32x4, so every load instruction
// of a wave reads 1 KiB of consecutive memory).  Each lane sums into an
// int64, the wave sums with shuffles, the block's waves meet in LDS, and
// thread 0 publishes the block sum in the block's slot of the workspace as
// one 64-bit word {tag:13, value:51}, the tag naming the call's generation.
// The last block of the grid waits until every slot carries the current tag,
// adds the slots in a fixed order, clears each slot it has read (so no word
// of an earlier call is left to match a later call's tag), writes the result
// and advances the generation.  No block waits on a later one and no counter
// is shared, so there are no same-address atomics and no fences.
//
// The grid is sized so that no block sums more than 2^19 elements, which
// bounds a block sum by 2^50 in magnitude and fits the 51-bit field.
//
// Integer addition is associative, so the result is the exact sum whatever
// the order.  The head (up to 3 elements before the first 16-byte boundary)
// and the tail (fewer than one tile) are summed by the last block of the
// grid with scalar loads.
#include "common.hpp"
#include "launch.hpp"
#include "layouts.hpp"
#include "tuning.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

constexpr int kBlock = 256;
// A tile is [kU][kBlock] int32x4: kU 16-byte loads per lane, all in flight at
// once.  kU = 4 (4096 elements) is the streaming shape; kU = 16 (16384) gives
// a quarter of the blocks, for sizes where dispatch and the final gather, not
// the stream, set the time.
constexpr int kMinU = 4;
constexpr int kTile = kBlock * kMinU * 4;         // int32 per tile of the smallest shape

constexpr int kValueBits = 51;
constexpr uint64_t kValueMask = (1ull << kValueBits) - 1;
constexpr uint32_t kTagPeriod = 8191;             // tags 1..8191; 0 never valid

__device__ __forceinline__ uint64_t tag_of(uint32_t gen) { return 1u + gen % kTagPeriod; }
__device__ __forceinline__ uint64_t pack_sum(int64_t v, uint32_t gen) {
  return (tag_of(gen) << kValueBits) | ((uint64_t)v & kValueMask);
}
__device__ __forceinline__ int64_t unpack_sum(uint64_t w) {   // sign-extend 51 bits
  return (int64_t)(w << (64 - kValueBits)) >> (64 - kValueBits);
}

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
template <int kU>
__global__ __launch_bounds__(kBlock) void reduce_i32_kernel(
    const i32x4* __restrict__ body, int64_t ntiles, const int32_t* __restrict__ head,
    int64_t nhead, const int32_t* __restrict__ tail, int64_t ntail, int64_t* __restrict__ out,
    WsHeader* __restrict__ hdr, uint64_t* __restrict__ partials) {
  __shared__ int64_t lds[kBlock / kWave];
  __shared__ CallState s_call;
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  if (thread.index() == 0) s_call = read_call_state(hdr);

  auto vecs = array(body, ntiles * (kBlock * kU));   // [tiles][kU][kBlock] int32x4

  int64_t acc = 0;
  for (idx_t t = block.index(); t < ntiles; t += block.count()) {
    auto mine = layout::block_striped<kBlock, kU>(vecs, t, thread);   // [kU]
    i32x4 q[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) q[u] = __builtin_nontemporal_load(&mine[u]);
#pragma unroll
    for (int u = 0; u < kU; ++u)
      acc += (int64_t)q[u].x + (int64_t)q[u].y + (int64_t)q[u].z + (int64_t)q[u].w;
  }
  const bool last = block.index() == block.count() - 1;
  if (last) {
    auto h = array(head, nhead);
    auto tl = array(tail, ntail);
    for (idx_t i = thread.index(); i < nhead; i += kBlock) acc += h[i];
    for (idx_t i = thread.index(); i < ntail; i += kBlock) acc += tl[i];
  }
  const int64_t s = block_sum(acc, lds);   // (its barrier also publishes s_call)
  const uint32_t gen = s_call.gen;
  auto parts = array(partials, block.count());
  if (!last) {
    if (thread.index() == 0) store_status(&parts[block.index()], pack_sum(s, gen));
    return;
  }

  // Last block: wait for every slot of this generation, add it and clear it.
  const uint64_t want = tag_of(gen);
  const uint32_t maxp = s_call.polls;
  int64_t acc2 = thread.index() == 0 ? s : 0;
  for (idx_t b = thread.index(); b < parts.extent() - 1; b += kBlock) {
    uint64_t w = 0;
    for (uint32_t polls = 0;; ++polls) {
      if (polls == maxp) {     // a bounded wait gave up: report it, leave the slot
        set_error(hdr, kDevWaitLimit);
        w = 0;
        break;
      }
      w = load_status(&parts[b]);
      if ((w >> kValueBits) == want) {
        store_status(&parts[b], 0);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    acc2 += unpack_sum(w);
  }
  sync(thread);   // lds is reused
  const int64_t total = block_sum(acc2, lds);
  if (thread.index() == 0) {
    out[0] = total;
    store_u32(&hdr->gen, next_gen(gen));
  }
}

constexpr const char* kNames[] = {"b256_u4_nt", "b256_u16_nt"};
constexpr int kDefaults[tune::kClasses] = {0, 0, 0, 0};
const bool kRegistered =
    (tune::register_op(tune::kReduceI32, "reduce_i32", 2, kNames, kDefaults), true);

}  // namespace

namespace launch {

// Grid: one block per tile (of `tile` elements) up to kReduceMaxBlocks, more
// when needed to keep a block's share at most 2^19 elements.  The smallest
// tile gives the largest grid, which sizes the workspace.
static int64_t reduce_grid(int64_t n, int64_t tile = kTile) {
  const int64_t ntiles = n / tile;
  int64_t grid = ntiles < kReduceMaxBlocks ? ntiles : kReduceMaxBlocks;
  const int64_t need = (n + (1 << 19) - 1) >> 19;
  if (grid < need) grid = need;
  return grid < 1 ? 1 : grid;
}

size_t reduce_i32_workspace(int64_t n) {
  return sizeof(WsHeader) + sizeof(uint64_t) * (size_t)reduce_grid(n < 0 ? 0 : n);
}

template <int kU>
static hipError_t launch_reduce(const int32_t* in, int64_t n, int64_t* out, void* ws,
                                hipStream_t s) {
  constexpr int64_t tile = (int64_t)kBlock * kU * 4;
  // Split the input at the first 16-byte boundary and after the last full tile.
  const uintptr_t addr = (uintptr_t)in;
  int64_t nhead = (int64_t)(((16 - (addr & 15)) & 15) / 4);
  if (nhead > n) nhead = n;
  const int64_t rest = n - nhead;
  const int64_t ntiles = rest / tile;
  const int64_t ntail = rest - ntiles * tile;
  const int64_t grid = reduce_grid(n, tile);
  WsHeader* hdr = (WsHeader*)ws;
  uint64_t* partials = (uint64_t*)((char*)ws + sizeof(WsHeader));
  hipLaunchKernelGGL(reduce_i32_kernel<kU>, dim3((unsigned)grid), dim3(kBlock), 0, s,
                     (const i32x4*)(in + nhead), ntiles, in, nhead, in + nhead + ntiles * tile,
                     ntail, out, hdr, partials);
  return hipGetLastError();
}

hipError_t reduce_i32(const int32_t* in, int64_t n, int64_t* out, void* ws, hipStream_t s) {
  (void)kRegistered;
  if (tune::get(tune::kReduceI32, tune::size_class(tune::kReduceI32, n)) == 1)
    return launch_reduce<16>(in, n, out, ws, s);
  return launch_reduce<kMinU>(in, n, out, ws, s);
}

}  // namespace launch
}  // namespace desc
