// grouped.hip -- many independent FP32 GEMMs of uneven shapes in one
// persistent launch (the batched form of the Sec. 5 matrix multiplication).
//
// Problem g is C_g = A_g * B_g with its own M, N, K, leading dimensions and
// pointers, described in a device array.
//
//   plan kernel (one block): gives each problem a tile shape (128 x 128 when
//     both M and N are at least 256, else 64 x 64; or 64 x 64 throughout, by
//     the tuning table), orders the problems with
//     the large tiles first (so the long tiles start early and the short ones
//     fill in at the end), and writes the exclusive prefix of tile counts in
//     that order with the total to the workspace.
//   main kernel: a grid of as many blocks as fit on the device at once walks
//     the global tile sequence, runs of 64 consecutive tiles per XCD so that
//     a problem's tiles share one L2; a binary search over the prefix finds
//     the problem, and the FP32 matrix-core tile routine of the plain GEMM
//     computes the tile.  Tiles are independent, so the loop needs no
//     inter-block communication.
#include "common.hpp"
#include "gemm_f32.hpp"
#include "launch.hpp"
#include "tuning.hpp"
#include "view.hpp"

#include "../../include/desc.h"

namespace desc {
namespace {

constexpr int kBlock = 256;
using BigTile = GemmCfgF32<128, 128, 16>;
using SmallTile = GemmCfgF32<64, 64, 16>;

struct GroupedWs {
  int64_t* total;        // tiles over all problems
  int64_t* tile_start;   // [G + 1], in planned order
  int32_t* order;        // [G] problem index in planned order
  int32_t* big;          // [G] 1 if the problem uses the large tile (indexed by problem)
};

// A problem takes the large tile when both M and N are at least big_min.
__device__ __forceinline__ bool is_big(const desc_gemm_problem& p, int64_t big_min) {
  return p.M >= big_min && p.N >= big_min;
}

__device__ __forceinline__ int64_t tiles_of(const desc_gemm_problem& p, bool big) {
  if (p.M <= 0 || p.N <= 0 || p.K < 0) return 0;
  const int64_t t = big ? 128 : 64;
  return ((p.M + t - 1) / t) * ((p.N + t - 1) / t);
}

// Block-wide exclusive prefix of one int64 per thread; returns the total.
__device__ __forceinline__ int64_t block_excl(int64_t v, int64_t* excl, int64_t* lds) {
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  int64_t incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t t = __shfl_up(incl, d, kWave);
    if ((int)lane_of_wave().index() >= d) incl += t;
  }
  if (lane_of_wave().index() == kWave - 1) lds[wv.index()] = incl;
  sync(thread);
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    before += (w < wv.index()) ? lds[w] : 0;
    tot += lds[w];
  }
  sync(thread);
  *excl = before + incl - v;
  return tot;
}

__global__ __launch_bounds__(kBlock) void grouped_plan_kernel(const desc_gemm_problem* probs,
                                                              int64_t G, int64_t big_min,
                                                              int64_t* total,
                                                              int64_t* tile_start,
                                                              int32_t* order, int32_t* big) {
  __shared__ int64_t lds[kBlock / kWave];
  auto thread = thread_x<kBlock>();
  auto pr = array(probs, G);
  auto ord = array(order, G);
  auto bg = array(big, G);
  auto ts = array(tile_start, G + 1);
  // pass 1: stable partition, large-tile problems first
  int64_t nbig = 0;
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    const bool b = g < G && is_big(pr[g], big_min);
    if (g < G) bg[g] = b;
    int64_t ex;
    const int64_t tot = block_excl(b ? 1 : 0, &ex, lds);
    if (b) ord[nbig + ex] = (int32_t)g;
    nbig += tot;
  }
  int64_t nsmall = 0;
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    const bool s = g < G && !is_big(pr[g], big_min);
    int64_t ex;
    const int64_t tot = block_excl(s ? 1 : 0, &ex, lds);
    if (s) ord[nbig + nsmall + ex] = (int32_t)g;
    nsmall += tot;
  }
  sync(thread);
  // pass 2: tile prefix in planned order
  int64_t carry = 0;
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t i = base + thread.index();
    int64_t t = 0;
    if (i < G) {
      const int32_t g = ord[i];
      t = tiles_of(pr[g], bg[g] != 0);
    }
    int64_t ex;
    const int64_t tot = block_excl(t, &ex, lds);
    if (i < G) ts[i] = carry + ex;
    carry += tot;
  }
  if (thread.index() == 0) {
    ts[G] = carry;
    total[0] = carry;
  }
}

// kBig: whether any problem may use the large tile (the LDS is sized for the
// largest tile the launch can meet, which bounds how many blocks fit a CU).
template <bool kBig>
__global__ __launch_bounds__(kBlock) void grouped_gemm_kernel(const desc_gemm_problem* probs,
                                                              int64_t G, const int64_t* total,
                                                              const int64_t* tile_start,
                                                              const int32_t* order,
                                                              const int32_t* big) {
  __shared__ float lds[kBig ? gemm_f32::lds_floats<BigTile>() : gemm_f32::lds_floats<SmallTile>()];
  __shared__ int64_t s_slot;
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  auto ts = array(tile_start, G + 1);
  const int64_t T = total[0];
  // Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
  // The planned tile sequence is cut into runs of kRun consecutive tiles
  // (about one problem), run u going to XCD u % 8, so the tiles that share a
  // problem's operands run on one XCD; the XCD's blocks walk its runs in
  // order.  t(l) grows with l, so the walk ends at the first t >= T.
  constexpr idx_t kRun = 64, kXcd = 8;
  const bool by_xcd = block.count() % kXcd == 0;
  const idx_t x = by_xcd ? block.index() % kXcd : 0;
  const idx_t per = by_xcd ? block.count() / kXcd : block.count();
  for (idx_t l = by_xcd ? block.index() / kXcd : block.index();; l += per) {
    const idx_t t = by_xcd ? (kXcd * (l / kRun) + x) * kRun + l % kRun : l;
    if (t >= T) break;
    if (thread.index() == 0) {       // planned slot of tile t: last i with ts[i] <= t
      idx_t lo = 0, hi = G;
      while (hi - lo > 1) {
        const idx_t mid = (lo + hi) / 2;
        if (ts[mid] <= t) lo = mid; else hi = mid;
      }
      s_slot = lo;
    }
    sync(thread);
    const idx_t slot = s_slot;
    const int32_t g = array(order, G)[slot];
    const desc_gemm_problem p = array(probs, G)[g];
    const bool b = array(big, G)[g] != 0;
    const GemmProblemF32 q{p.A, p.lda, p.B, p.ldb, p.C, p.ldc, p.M, p.N, p.K};
    const idx_t local = t - ts[slot];
    const bool vec = gemm_f32::vec_ok(p.A, p.lda, p.B, p.ldb);
    if (kBig && b) {
      const idx_t tn = (p.N + 127) / 128;
      if (vec) gemm_f32::tile<BigTile, true>(q, local / tn, local % tn, lds);
      else gemm_f32::tile<BigTile, false>(q, local / tn, local % tn, lds);
    } else {
      const idx_t tn = (p.N + 63) / 64;
      if (vec) gemm_f32::tile<SmallTile, true>(q, local / tn, local % tn, lds);
      else gemm_f32::tile<SmallTile, false>(q, local / tn, local % tn, lds);
    }
    sync(thread);   // s_slot and lds are reused by the next tile
  }
}

GroupedWs carve(void* ws, int64_t G) {
  uint8_t* w = (uint8_t*)ws;
  GroupedWs r;
  size_t o = 64;
  r.total = (int64_t*)w;
  r.tile_start = (int64_t*)(w + o);
  o += ((G + 1) * 8 + 63) & ~(size_t)63;
  r.order = (int32_t*)(w + o);
  o += (G * 4 + 63) & ~(size_t)63;
  r.big = (int32_t*)(w + o);
  return r;
}

template <bool kBig>
int persistent_grid() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cached[dev] == 0) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, grouped_gemm_kernel<kBig>, kBlock,
                                                     0) != hipSuccess || per < 1)
      per = 1;
    cached[dev] = cus * per;
  }
  return cached[dev];
}

// Tile choice: 128 x 128 tiles for problems with M, N >= 256 and 64 x 64
// otherwise, or 64 x 64 tiles throughout (more, smaller tiles balance better
// over the CUs when the problems are small).
constexpr const char* kNames[] = {"tile128_or_64", "tile64"};
constexpr int kDefaults[tune::kClasses] = {1, 1, 1, 1};
constexpr int64_t kBigMin[] = {256, INT64_MAX};
const bool kRegistered =
    (tune::register_op(tune::kGemmGrouped, "gemm_grouped", 2, kNames, kDefaults), true);

}  // namespace

namespace launch {

size_t gemm_grouped_workspace(int64_t G) {
  return 64 + (((G + 1) * 8 + 63) & ~(size_t)63) + 2 * ((G * 4 + 63) & ~(size_t)63);
}

hipError_t gemm_grouped_f32(const desc_gemm_problem* problems, int64_t G, void* ws,
                            hipStream_t s) {
  (void)kRegistered;
  const GroupedWs w = carve(ws, G);
  // the size class is taken from the problem count
  const int cfg = tune::get(tune::kGemmGrouped, tune::size_class(tune::kGemmGrouped, G));
  hipLaunchKernelGGL(grouped_plan_kernel, dim3(1), dim3(kBlock), 0, s, problems, G,
                     kBigMin[cfg == 1 ? 1 : 0], w.total, w.tile_start, w.order, w.big);
  if (cfg == 1)
    hipLaunchKernelGGL(grouped_gemm_kernel<false>, dim3((unsigned)persistent_grid<false>()),
                       dim3(kBlock), 0, s, problems, G, w.total, w.tile_start, w.order, w.big);
  else
    hipLaunchKernelGGL(grouped_gemm_kernel<true>, dim3((unsigned)persistent_grid<true>()),
                       dim3(kBlock), 0, s, problems, G, w.total, w.tile_start, w.order, w.big);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
