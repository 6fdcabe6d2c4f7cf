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
  // where 4096 blocks reach 6.0 (reads alone stream at 6.7 TB/s, writes
  // alone at 4.5: the writes set the ceiling of a read + write stream).
  constexpr int64_t kMaxGrid = 16384;
  int64_t grid = chunks < kMaxGrid ? chunks : kMaxGrid;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((copy32_kernel<kUnroll, kNt>), dim3((unsigned)grid), dim3(kBlock), 0, s,
                     (const u32x4*)in, (u32x4*)out, nvec, in + 4 * nvec, out + 4 * nvec,
                     n - 4 * nvec);
  return hipGetLastError();
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

}  // namespace launch
}  // namespace desc
