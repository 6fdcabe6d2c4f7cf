// copy.hip -- a plain copy of 32-bit words: the achievable HBM ceiling that
// the bandwidth-bound kernels are compared with, and the kernel of known
// traffic that calibrates the FETCH_SIZE / WRITE_SIZE counters.
//
// Grid-stride over 16-byte vectors, each lane moving UNROLL vectors per
// iteration with every load issued before the first store.
#include "common.hpp"
#include "launch.hpp"
#include "tuning.hpp"
#include "view.hpp"

namespace desc {
namespace {

constexpr int kBlock = 256;

template <int kUnroll, bool kNt>
__global__ __launch_bounds__(kBlock) void copy32_kernel(const u32x4* __restrict__ in,
                                                        u32x4* __restrict__ out, int64_t nvec,
                                                        const uint32_t* __restrict__ tail_in,
                                                        uint32_t* __restrict__ tail_out,
                                                        int64_t ntail) {
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  constexpr int kChunk = kBlock * kUnroll;
  const int64_t nchunks = nvec / kChunk;
  auto src = array(in, nchunks * kChunk).group<kBlock>().group<kUnroll>();
  auto dst = array(out, nchunks * kChunk).group<kBlock>().group<kUnroll>();
  for (idx_t c = block.index(); c < nchunks; c += block.count()) {
    auto s = src.idx(c).transpose().select(thread);
    auto d = dst.idx(c).transpose().select(thread);
    u32x4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if constexpr (kNt) v[u] = __builtin_nontemporal_load(&s[u]);
      else v[u] = s[u];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if constexpr (kNt) __builtin_nontemporal_store(v[u], &d[u]);
      else d[u] = v[u];
    }
  }
  if (block.index() == block.count() - 1) {
    // the vectors after the last full chunk, then the scalar tail
    auto rs = array(in, nvec).snd(nchunks * kChunk);
    auto rd = array(out, nvec).snd(nchunks * kChunk);
    for (idx_t i = thread.index(); i < rs.extent(); i += kBlock) rd[i] = rs[i];
    auto ts = array(tail_in, ntail);
    auto td = array(tail_out, ntail);
    for (idx_t i = thread.index(); i < ntail; i += kBlock) td[i] = ts[i];
  }
}

template <int kUnroll, bool kNt>
hipError_t launch_copy(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  const bool vec = (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  const int64_t nvec = vec ? n / 4 : 0;
  const int64_t chunks = nvec / (kBlock * kUnroll);
  // Many blocks in flight: at 2^28 words a grid of 16384 copies at 6.2 TB/s
  // where 4096 blocks reach 6.0 (reads alone stream at 6.5-7.0 TB/s and
  // writes alone at 6.2-6.9, so a read + write stream stays below either).
  constexpr int64_t kMaxGrid = 16384;
  int64_t grid = chunks < kMaxGrid ? chunks : kMaxGrid;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((copy32_kernel<kUnroll, kNt>), dim3((unsigned)grid), dim3(kBlock), 0, s,
                     (const u32x4*)in, (u32x4*)out, nvec, in + 4 * nvec, out + 4 * nvec,
                     n - 4 * nvec);
  return hipGetLastError();
}

// Reversal, out[i] = in[n - 1 - i]: the copy read through the reverse view.
// With n a multiple of 4 and both arrays 16-byte aligned, the input is seen
// as 16-byte vectors in reverse order and each vector's four words are
// swapped end for end; otherwise word by word.
template <bool kVec>
__global__ __launch_bounds__(kBlock) void reverse32_kernel(const uint32_t* __restrict__ in,
                                                           uint32_t* __restrict__ out, int64_t n) {
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  if constexpr (kVec) {
    constexpr int kUnroll = 4, kChunk = kBlock * kUnroll;
    const int64_t nvec = n / 4, nchunks = nvec / kChunk;
    auto src = array((const u32x4*)in, nvec).reverse();
    auto dst = array((u32x4*)out, nvec);
    auto sc = src.fst(nchunks * kChunk).group<kBlock>().group<kUnroll>();
    auto dc = dst.fst(nchunks * kChunk).group<kBlock>().group<kUnroll>();
    for (idx_t c = block.index(); c < nchunks; c += block.count()) {
      auto s = sc.idx(c).transpose().select(thread);
      auto d = dc.idx(c).transpose().select(thread);
      u32x4 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(&s[u]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const u32x4 w = {v[u].w, v[u].z, v[u].y, v[u].x};
        __builtin_nontemporal_store(w, &d[u]);
      }
    }
    if (block.index() == block.count() - 1) {   // the vectors after the last full chunk
      auto rs = src.snd(nchunks * kChunk);
      auto rd = dst.snd(nchunks * kChunk);
      for (idx_t i = thread.index(); i < rs.extent(); i += kBlock) {
        const u32x4 v = rs[i];
        rd[i] = u32x4{v.w, v.z, v.y, v.x};
      }
    }
  } else {
    auto src = array(in, n).reverse();
    auto dst = array(out, n);
    for (idx_t i = block.index() * kBlock + thread.index(); i < n; i += block.count() * kBlock)
      dst[i] = src[i];
  }
}

constexpr const char* kNames[] = {"u4_nt", "u4", "u8_nt", "u8"};
constexpr int kDefaults[tune::kClasses] = {0, 0, 0, 0};
const bool kRegistered = (tune::register_op(tune::kCopy32, "copy_32", 4, kNames, kDefaults), true);

}  // namespace

namespace launch {

hipError_t copy_32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  (void)kRegistered;
  switch (tune::get(tune::kCopy32, tune::size_class(tune::kCopy32, n))) {
    case 1: return launch_copy<4, false>(in, out, n, s);
    case 2: return launch_copy<8, true>(in, out, n, s);
    case 3: return launch_copy<8, false>(in, out, n, s);
    default: return launch_copy<4, true>(in, out, n, s);
  }
}

hipError_t reverse_32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const bool vec = n % 4 == 0 && (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  const int64_t per_block = vec ? 4 * kBlock * 4 : kBlock;
  int64_t grid = (n + per_block - 1) / per_block;
  if (grid > 16384) grid = 16384;
  if (vec)
    hipLaunchKernelGGL(reverse32_kernel<true>, dim3((unsigned)grid), dim3(kBlock), 0, s, in, out,
                       n);
  else
    hipLaunchKernelGGL(reverse32_kernel<false>, dim3((unsigned)grid), dim3(kBlock), 0, s, in, out,
                       n);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
