// reduce_ops.hip -- two more reductions over the block-wide structure of the
// sum (Sec. 5, "block-wide parallel reduction"): the smallest and largest of
// int32 values, and the sum of FP32 values accumulated in FP64 in an order
// fixed by the element indices and n alone.
//
// Layout.  The input is cut into chunks of 4096 elements, each read as
// [4][256] groups of four consecutive elements ([chunks][u][lane] x 4, so a
// wave's load instruction covers 1 KiB of consecutive memory): lane j of a
// block takes elements 1024 u + 4 j + e of a chunk, u, e = 0..3.  The groups
// are read as dword-aligned 16-byte vectors, so any 4-byte-aligned input
// takes the same path and the same order.  Block b of the G blocks takes
// chunks b, b + G, b + 2G, ...; the last, partial chunk (if any) is read
// element by element by the block whose turn it is, in the same order.
//
// Order of the float sum (every addition an FP64 addition, rounded to
// nearest even; the conversion of each float to FP64 is exact):
//   1. lane j of block b adds its elements from 0.0, chunk by chunk in
//      ascending order, u then e ascending inside a chunk (elements at or
//      beyond n are skipped);
//   2. the block combines its 256 lane values in a fixed tree: inside each
//      64-lane wave, lane i adds lane i ^ 32, then i ^ 16, 8, 4, 2, 1 (the
//      two lanes of a pair compute the same sum, addition being
//      commutative), and the four wave values as (w0 + w1) + (w2 + w3);
//   3. the last block gathers the G block values: its lane t adds those of
//      blocks t, t + 256, ... in ascending order from 0.0, and the block
//      combines them with the tree of step 2.
// G = min(max(ceil(n / 4096), 1), 2048) depends on n only, so the result is
// a function of the input values and n: the same on every run, at every
// input address, and whatever runs concurrently.  Its error is at most
// d u sum |x_i| (u = 2^-53), d the longest chain of additions, at most
// 16 ceil(ceil(n / 4096) / G) + 8 + ceil(G / 256) + 8.
//
// Hand-over between blocks as in the integer sum: no shared counter, no
// fence.  A block publishes its value in its two-word slot of the workspace,
// each 64-bit word {tag:32, half of the value:32}, the tag naming the call's
// generation; the last block waits until both words of every slot carry the
// current tag, clears each slot it has read, and advances the generation
// when it is done.
#include "common.hpp"
#include "handover.hpp"
#include "launch.hpp"
#include "view.hpp"

namespace desc {
namespace {

constexpr int kBlock = 256;
constexpr int kGroups = 4;                       // 16-byte groups per lane per chunk
constexpr int kChunk = kBlock * kGroups * 4;     // 4096 elements
constexpr int64_t kMaxBlocks = 2048;
constexpr int kWaves = kBlock / kWave;

typedef uint32_t u32x4u __attribute__((ext_vector_type(4))) __attribute__((aligned(4)));

// FP64 sum of FP32 values, in the order stated above.
struct SumF32 {
  typedef double Acc;
  typedef double Out;
  __device__ static Acc identity() { return 0.0; }
  __device__ static Acc step(Acc a, uint32_t w) { return a + (double)__uint_as_float(w); }
  __device__ static Acc join(Acc a, Acc b) { return a + b; }
  __device__ static Acc shfl_xor(Acc a, int m) { return __shfl_xor(a, m, kWave); }
  __device__ static uint32_t half(Acc a, int k) {
    const uint64_t u = (uint64_t)__double_as_longlong(a);
    return (uint32_t)(k ? u >> 32 : u);
  }
  __device__ static Acc from_halves(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  }
  __device__ static void write(Out* out, Acc a) { out[0] = a; }
};

// Smallest and largest int32 value (exact in any order).
struct MinMaxI32 {
  struct Acc {
    int32_t lo, hi;
  };
  typedef int32_t Out;
  __device__ static Acc identity() { return {INT32_MAX, INT32_MIN}; }
  __device__ static Acc step(Acc a, uint32_t w) {
    const int32_t v = (int32_t)w;
    return {min(a.lo, v), max(a.hi, v)};
  }
  __device__ static Acc join(Acc a, Acc b) { return {min(a.lo, b.lo), max(a.hi, b.hi)}; }
  __device__ static Acc shfl_xor(Acc a, int m) {
    return {__shfl_xor(a.lo, m, kWave), __shfl_xor(a.hi, m, kWave)};
  }
  __device__ static uint32_t half(Acc a, int k) { return (uint32_t)(k ? a.hi : a.lo); }
  __device__ static Acc from_halves(uint32_t lo, uint32_t hi) {
    return {(int32_t)lo, (int32_t)hi};
  }
  __device__ static void write(Out* out, Acc a) {
    out[0] = a.lo;
    out[1] = a.hi;
  }
};

// Step 2 of the order: the fixed tree over the block's lanes.  `lds` holds
// one value per wave; the result is valid in every thread.
template <class Op>
__device__ __forceinline__ typename Op::Acc block_tree(typename Op::Acc v,
                                                      typename Op::Acc* lds) {
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = Op::join(v, Op::shfl_xor(v, m));
  if (lane_of_wave().index() == 0) lds[wv.index()] = v;
  sync(thread);
  static_assert(kWaves == 4, "the tree below pairs four waves");
  return Op::join(Op::join(lds[0], lds[1]), Op::join(lds[2], lds[3]));
}

template <class Op>
__global__ __launch_bounds__(kBlock) void reduce_op_kernel(const uint32_t* __restrict__ in,
                                                           int64_t n,
                                                           typename Op::Out* __restrict__ out,
                                                           WsHeader* __restrict__ hdr,
                                                           uint64_t* __restrict__ slots) {
  typedef typename Op::Acc Acc;
  __shared__ Acc lds[kWaves];
  __shared__ CallState s_call;
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  if (thread.index() == 0) s_call = read_call_state(hdr);

  const int64_t nfull = n / kChunk;
  // [chunks][kGroups][kBlock] groups of four elements; this lane's [kGroups]
  auto groups = array((const u32x4u*)in, nfull * (kChunk / 4))
                    .template group<kBlock>()
                    .template group<kGroups>();

  Acc acc = Op::identity();
  for (idx_t c = block.index(); c < nfull; c += block.count()) {
    auto mine = groups.idx(c).transpose().select(thread);   // [kGroups]
    u32x4u q[kGroups];
#pragma unroll
    for (int u = 0; u < kGroups; ++u) q[u] = __builtin_nontemporal_load(&mine[u]);
#pragma unroll
    for (int u = 0; u < kGroups; ++u) {
      acc = Op::step(acc, q[u].x);
      acc = Op::step(acc, q[u].y);
      acc = Op::step(acc, q[u].z);
      acc = Op::step(acc, q[u].w);
    }
  }
  if (nfull * kChunk < n && nfull % block.count() == block.index()) {
    // The partial chunk, last in this block's sequence, element by element.
    auto x = array(in, n);
    const int64_t base = nfull * kChunk + 4 * (int64_t)thread.index();
#pragma unroll
    for (int u = 0; u < kGroups; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = base + u * (4 * kBlock) + e;
        if (i < n) acc = Op::step(acc, x[i]);
      }
  }
  const Acc mine = block_tree<Op>(acc, lds);   // (its barrier also publishes s_call)
  const uint32_t gen = s_call.gen;
  const uint64_t tag = handover::tag_of(gen);
  auto slot = array(slots, 2 * block.count()).template group<2>();   // [G][2]
  const bool last = block.index() == block.count() - 1;
  if (!last) {
    if (thread.index() == 0)
      handover::publish(&slot.idx(block.index())[0], tag,
                        ((uint64_t)Op::half(mine, 1) << 32) | Op::half(mine, 0));
    return;
  }

  // Step 3: the last block gathers the block values, lane t those of blocks
  // t, t + 256, ..., and clears each slot it has read.
  Acc g = Op::identity();
  for (idx_t b = thread.index(); b < block.count(); b += kBlock) {
    Acc v = mine;
    if (b != block.index()) {
      uint64_t w = 0;
      if (handover::poll(&slot.idx(b)[0], tag, w, s_call.polls))
        handover::clear(&slot.idx(b)[0]);
      else
        set_error(hdr, kDevWaitLimit);
      v = Op::from_halves((uint32_t)w, (uint32_t)(w >> 32));
    }
    g = Op::join(g, v);
  }
  sync(thread);   // lds is reused
  const Acc total = block_tree<Op>(g, lds);
  if (thread.index() == 0) {
    Op::write(out, total);
    store_u32(&hdr->gen, next_gen(gen));
  }
}

int64_t op_grid(int64_t n) {
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  return chunks < 1 ? 1 : (chunks < kMaxBlocks ? chunks : kMaxBlocks);
}

template <class Op>
hipError_t launch_op(const uint32_t* in, int64_t n, typename Op::Out* out, void* ws,
                     hipStream_t s) {
  const int64_t grid = op_grid(n);
  WsHeader* hdr = (WsHeader*)ws;
  uint64_t* slots = (uint64_t*)((char*)ws + sizeof(WsHeader));
  hipLaunchKernelGGL(reduce_op_kernel<Op>, dim3((unsigned)grid), dim3(kBlock), 0, s, in, n, out,
                     hdr, slots);
  return hipGetLastError();
}

}  // namespace

namespace launch {

int64_t reduce_op_grid(int64_t n) { return op_grid(n < 0 ? 0 : n); }

size_t reduce_op_workspace(int64_t n) {
  return sizeof(WsHeader) + 2 * sizeof(uint64_t) * (size_t)op_grid(n < 0 ? 0 : n);
}

hipError_t minmax_i32(const int32_t* in, int64_t n, int32_t* out, void* ws, hipStream_t s) {
  return launch_op<MinMaxI32>((const uint32_t*)in, n, out, ws, s);
}

hipError_t sum_f32(const float* in, int64_t n, double* out, void* ws, hipStream_t s) {
  return launch_op<SumF32>((const uint32_t*)in, n, out, ws, s);
}

}  // namespace launch
}  // namespace desc
