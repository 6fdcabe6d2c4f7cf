// grouped.hip -- many independent GEMMs of uneven shapes in persistent
// launches (the batched form of the Sec. 5 matrix multiplication), in FP32
// or in the three-product split-BF16 mode.
//
// Problem g is C_g = A_g * B_g with its own M, N, K, leading dimensions and
// pointers, described in a device array.
//
//   plan kernel (one block): gives each problem a tile shape (128 x 128 when
//     both M and N are at least 256, else 64 x 64; or 64 x 64 throughout, by
//     the tuning table), orders the problems longest tiles first -- the
//     large tiles, then by K in buckets of 64 -- so that the long tiles start
//     early and the short ones fill in at the end, and writes the exclusive
//     prefix of tile counts in that order with the total to the workspace.
//   main kernel: a grid of as many blocks as fit on the device at once walks
//     the global tile sequence, runs of 64 consecutive tiles per XCD so that
//     a problem's tiles share one L2; a binary search over the prefix finds
//     the problem, and the FP32 matrix-core tile routine of the plain GEMM
//     computes the tile.  Tiles are independent, so the loop needs no
//     inter-block communication.
#include "common.hpp"
#include "gemm_f32.hpp"
#include "gemm_nt.hpp"
#include "launch.hpp"
#include "lowp.hpp"
#include "tuning.hpp"
#include "view.hpp"
#include "wave.hpp"

#include "../../include/desc.h"

namespace desc {
namespace {

constexpr int kBlock = 256;
using BigTile = GemmCfgF32<128, 128, 16>;
using SmallTile = GemmCfgF32<64, 64, 16>;
using SmallTileRm = gemm_f32::GemmCfgF32W<64, 64, 16, 2, 2, 2, true>;   // row-major A, two stages ahead, 16x16x4

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

// Last i in [0, G) with start[i] <= t, for a nondecreasing start with
// start[0] <= t < start[G]: a 64-way search by one whole wave.  Each round
// every lane reads one boundary and a ballot counts those <= t (a prefix of
// the lanes), so G = 512 takes two rounds of parallel loads instead of nine
// dependent ones.
__device__ __forceinline__ idx_t wave_owner(const int64_t* start, int64_t G, int64_t t) {
  auto st = array(start, G + 1);
  const idx_t lane = lane_of_wave().index();
  idx_t lo = 0, hi = G;
  while (hi - lo > 1) {
    const idx_t step = (hi - lo + kWave - 1) / kWave;
    const idx_t i = lo + lane * step;
    const bool le = i < hi && st[i] <= t;
    lo += ((idx_t)__popcll(__ballot(le)) - 1) * step;
    hi = lo + step < hi ? lo + step : hi;
  }
  return lo;
}

// Sort key of the planned order: 0 .. kKBuckets-1 for large-tile problems,
// kKBuckets .. 2 kKBuckets-1 for the others, K descending in buckets of 64.
constexpr int kKBuckets = 16;
__device__ __forceinline__ int plan_key(const desc_gemm_problem& p, bool big) {
  const int64_t kb = p.K <= 64 ? 0 : ((p.K - 1) / 64 < kKBuckets - 1 ? (p.K - 1) / 64
                                                                       : kKBuckets - 1);
  return (big ? 0 : kKBuckets) + (kKBuckets - 1 - (int)kb);
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
  // pass 1: order the problems longest tiles first (a tile's time grows with
  // its area and its K): large-tile problems, then small ones, each by K in
  // buckets of 64, largest first.  A counting sort with LDS counters; the
  // order within a bucket varies from run to run, which changes only which
  // block computes a tile, never its arithmetic.
  __shared__ int32_t s_pos[2 * kKBuckets];
  if (thread.index() < 2 * kKBuckets) s_pos[thread.index()] = 0;
  sync(thread);
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    if (g < G) {
      const bool b = is_big(pr[g], big_min);
      bg[g] = b;
      atomicAdd(&s_pos[plan_key(pr[g], b)], 1);
    }
  }
  sync(thread);
  if (thread.index() == 0) {
    int32_t at = 0;
    for (int k = 0; k < 2 * kKBuckets; ++k) {
      const int32_t c = s_pos[k];
      s_pos[k] = at;
      at += c;
    }
  }
  sync(thread);
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    if (g < G) ord[atomicAdd(&s_pos[plan_key(pr[g], is_big(pr[g], big_min))], 1)] = (int32_t)g;
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
// kRm: 64 x 64 tiles of the row-major-A tile form.
template <bool kBig, bool kRm = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kRm ? 3 : 1)))
void grouped_gemm_kernel(const desc_gemm_problem* probs,
                                                              int64_t G, const int64_t* total,
                                                              const int64_t* tile_start,
                                                              const int32_t* order,
                                                              const int32_t* big) {
  __shared__ __attribute__((aligned(16))) float
      lds[kRm ? SmallTileRm::lds_floats
              : (kBig ? gemm_f32::lds_floats<BigTile>() : gemm_f32::lds_floats<SmallTile>())];
  __shared__ int64_t s_slot;
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  auto ts = array(tile_start, G + 1);
  const int64_t T = total[0];
  // The XCD-aware walk (layout::tile_walk): runs of 64 consecutive planned
  // tiles (about one problem) stay on one XCD, each with its own L2, so the
  // tiles that share a problem's operands meet its cache.
  const layout::TileWalk walk = layout::tile_walk(block.index(), block.count());
  for (idx_t l = walk.first;; l += walk.per) {
    const idx_t t = walk.tile(l);
    if (t >= T) break;
    if (thread.index() < kWave) {    // planned slot of tile t: last i with ts[i] <= t
      const idx_t slot = wave_owner(tile_start, G, t);
      if (thread.index() == 0) s_slot = slot;
    }
    sync(thread);
    const idx_t slot = wave::uniform_i64(s_slot);
    const int32_t g = array(order, G)[slot];
    const desc_gemm_problem p = array(probs, G)[g];
    const bool b = array(big, G)[g] != 0;
    const GemmProblemF32 q{p.A, p.lda, p.B, p.ldb, p.C, p.ldc, p.M, p.N, p.K};
    const idx_t local = t - ts[slot];
    const bool vec = gemm_f32::vec_ok(p.A, p.lda, p.B, p.ldb);
    if constexpr (kRm) {
      const idx_t tn = (p.N + 63) / 64, tm_ = local / tn, tn_ = local % tn;
      if (vec && gemm_f32::interior_tile<SmallTileRm>(q, tm_, tn_))
        gemm_f32::tile_rowmajor<SmallTileRm, true, true>(q, tm_, tn_, lds);
      else if (vec && p.K % 4 == 0 && p.N % 4 == 0 && p.K > 0)
        gemm_f32::tile_rowmajor<SmallTileRm, true>(q, tm_, tn_, lds);
      else
        gemm_f32::tile_rowmajor<SmallTileRm, false>(q, tm_, tn_, lds);
    } else if (kBig && b) {
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
  r.total = (int64_t*)(w + 8);   // (bytes 0-7 left alone: byte 4 is the status word of other calls)
  r.tile_start = (int64_t*)(w + o);
  o += ((G + 1) * 8 + 63) & ~(size_t)63;
  r.order = (int32_t*)(w + o);
  o += (G * 4 + 63) & ~(size_t)63;
  r.big = (int32_t*)(w + o);
  return r;
}

template <bool kBig, bool kRm>
int persistent_grid() {
  static int cached[64] = {0};
  return launch::resident_grid(grouped_gemm_kernel<kBig, kRm>, cached, 1, kBlock);
}

// --------------------------------------------------------------------------
// Split-BF16 (three products) mode.  Every problem's operands are split into
// bf16 planes in the workspace, Ah, Al as [Ma][Kp] and Bh^T, Bl^T as
// [Na][Kp]: K rounded up to a multiple of 64 (at least 64, so K = 0 gives
// zero products through the same path), M and N rounded up to multiples of
// 128 so that either output tile size fits the planes whatever the
// configuration.
//   plan kernel (one block): per problem the NT tiles, the split work items
//     and the byte offset of its planes, as exclusive prefixes; if the planes
//     do not fit the workspace, the error word is set and nothing is planned.
//   split kernel (persistent): 64 x 64 items -- A tiles split in place, B
//     tiles split and transposed through LDS -- over M and N rounded up to
//     64 and the whole of Kp.  Columns k >= K are written as zeros (they
//     enter every product); rows past M, N up to the 128 rounding are not
//     written: they only reach output rows or columns that are never stored.
//   NT kernel (persistent): output tiles of the low-precision tile routine,
//     64 x 64 or 128 x 128 per problem as the configuration says, runs of 64
//     tiles per XCD as in the FP32 mode.
// --------------------------------------------------------------------------
constexpr int kPad = 64, kPadBig = 128;
using NtSmall = NtCfg<64, 64, 64, Bf16x3Mode, 2, 2, 2>;
using NtBig = NtCfg<128, 128, 64, Bf16x3Mode, 2, 2, 2>;
static_assert(NtSmall::threads == kBlock && NtBig::threads == kBlock, "one block shape");
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

constexpr int64_t kMaxDim = int64_t(1) << 40;         // larger M, N or K: refused
constexpr int64_t kMaxPlaneBytes = int64_t(1) << 44;  // larger planes of one problem: refused
__host__ __device__ inline int64_t round_up(int64_t v, int64_t p) { return (v + p - 1) / p * p; }

struct Bf16Dims {
  int64_t Ma, Na;   // plane rows: M, N rounded up to 128
  int64_t Ms, Ns;   // rows the split writes: M, N rounded up to 64
  int64_t Kp;       // K rounded up to 64, at least 64
  bool empty;       // M <= 0 or N <= 0: nothing to compute or store
  bool huge;        // a dimension or the planes beyond the limits above
};
__host__ __device__ inline Bf16Dims bf16_dims(int64_t M, int64_t N, int64_t K) {
  Bf16Dims d;
  d.empty = M <= 0 || N <= 0;
  d.huge = !d.empty && (M > kMaxDim || N > kMaxDim || K > kMaxDim);
  const bool none = d.empty || d.huge;
  d.Ma = none ? 0 : round_up(M, kPadBig);
  d.Na = none ? 0 : round_up(N, kPadBig);
  d.Ms = none ? 0 : round_up(M, kPad);
  d.Ns = none ? 0 : round_up(N, kPad);
  d.Kp = none ? 0 : (K <= kPad ? kPad : round_up(K, kPad));   // K <= 0: one zero step
  d.huge = d.huge || (!none && d.Ma + d.Na > kMaxPlaneBytes / (4 * d.Kp));
  if (d.huge) d.Ma = d.Na = d.Ms = d.Ns = d.Kp = 0;
  return d;
}
// Four planes, 256-byte aligned (none for a refused or empty problem).
__host__ __device__ inline int64_t bf16_plane_bytes(const Bf16Dims& d) {
  return round_up(4 * (d.Ma + d.Na) * d.Kp, 256);
}
// Configurations: 0-1 split into planes first, 2-3 split while staging
// (fused: no planes).  Output tiles of 64 x 64 (0, 2) or 128 x 128 (1, 3).
template <int kCfg>
constexpr bool kFused = kCfg >= 2;
template <int kCfg>
constexpr bool kSmallOnly = kCfg == 0 || kCfg == 2;   // 64 x 64 tiles
// the fused kernel's tile routine configuration
template <int kCfg>
using FusedNt = typename std::conditional<kSmallOnly<kCfg>, NtSmall, NtBig>::type;
template <int kCfg>
__device__ __forceinline__ int64_t tile_edge(int64_t, int64_t) {
  return kSmallOnly<kCfg> ? kPad : kPadBig;
}

struct Bf16Ws {
  int64_t* totals;       // [0] NT tiles, [1] split items, [2] fused tiles
  uint32_t* error;       // kDevPlanes when the planes do not fit, else 0 (every call)
  int64_t* nt_start;     // [G + 1]
  int64_t* split_start;  // [G + 1]
  int64_t* plane_off;    // [G]
  int64_t* fused_start;  // [G + 1], over the fused order's slots
  int32_t* fused_order;  // [G] problem of each slot, longest tiles first
  uint8_t* planes;
  int64_t planes_bytes;  // room for the planes
};
size_t bf16_head_bytes(int64_t G) {   // planes start 256-byte aligned
  return 256 + 4 * (((G + 1) * 8 + 255) & ~(size_t)255) + ((G * 4 + 255) & ~(size_t)255);
}
Bf16Ws bf16_carve(void* ws, size_t ws_bytes, int64_t G) {
  uint8_t* w = (uint8_t*)ws;
  const size_t arr = ((G + 1) * 8 + 255) & ~(size_t)255;
  Bf16Ws r;
  r.error = (uint32_t*)(w + 4);    // the device status word, where every workspace has it
  r.totals = (int64_t*)(w + 8);
  r.nt_start = (int64_t*)(w + 256);
  r.split_start = (int64_t*)(w + 256 + arr);
  r.plane_off = (int64_t*)(w + 256 + 2 * arr);
  r.fused_start = (int64_t*)(w + 256 + 3 * arr);
  r.fused_order = (int32_t*)(w + 256 + 4 * arr);
  r.planes = w + bf16_head_bytes(G);
  r.planes_bytes = (int64_t)ws_bytes - (int64_t)bf16_head_bytes(G);
  return r;
}

// In the fused configurations a problem is staged straight from its FP32
// operands when its strides allow (the split source's buffer ranges), and
// through planes otherwise; the other configurations use planes throughout.
__host__ __device__ inline bool fused_route(int cfg, int64_t lda, int64_t ldb) {
  return cfg >= 2 && lda <= gemm_nt::kSplitMaxLd && ldb <= gemm_nt::kSplitMaxLd;
}
template <int kCfg>
__device__ __forceinline__ bool fused_for(const desc_gemm_problem& p) {
  return fused_route(kCfg, p.lda, p.ldb);
}

template <int kCfg>
__global__ __launch_bounds__(kBlock) void bf16_plan_kernel(const desc_gemm_problem* probs,
                                                           int64_t G, Bf16Ws w) {
  __shared__ int64_t lds[kBlock / kWave];
  auto thread = thread_x<kBlock>();
  auto pr = array(probs, G);
  auto nts = array(w.nt_start, G + 1);
  auto sps = array(w.split_start, G + 1);
  auto pof = array(w.plane_off, G);
  auto fts = array(w.fused_start, G + 1);
  int64_t c_nt = 0, c_sp = 0, c_pl = 0, c_ft = 0, c_huge = 0;
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    int64_t nt = 0, sp = 0, pl = 0, ft = 0, huge = 0;
    if (g < G) {
      const desc_gemm_problem p = pr[g];
      const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
      if (!d.empty && !d.huge) {
        const int64_t e = tile_edge<kCfg>(p.M, p.N);
        const int64_t tiles = (round_up(p.M, e) / e) * (round_up(p.N, e) / e);
        if (fused_for<kCfg>(p)) {
          ft = tiles;
        } else {
          nt = tiles;
          sp = (d.Ms / kPad) * (d.Kp / kPad) + (d.Kp / kPad) * (d.Ns / kPad);
          pl = bf16_plane_bytes(d);
        }
      }
      huge = d.huge;
    }
    int64_t e_nt, e_sp, e_pl, e_ft, e_huge;
    const int64_t t_nt = block_excl(nt, &e_nt, lds);
    const int64_t t_sp = block_excl(sp, &e_sp, lds);
    const int64_t t_pl = block_excl(pl, &e_pl, lds);
    const int64_t t_ft = block_excl(ft, &e_ft, lds);
    c_huge += block_excl(huge, &e_huge, lds);
    if (g < G) {
      nts[g] = c_nt + e_nt;
      sps[g] = c_sp + e_sp;
      pof[g] = c_pl + e_pl;
    }
    c_nt += t_nt;
    c_sp += t_sp;
    c_ft += t_ft;
    // at most 256 * 2^44 bytes per round: held below 2^60, no overflow
    c_pl = c_pl + t_pl < (int64_t(1) << 60) ? c_pl + t_pl : (int64_t(1) << 60);
  }
  // The fused tiles in the order of the FP32 plan (longest tiles first: the
  // large edge, then K descending), by a counting sort on LDS counters; the
  // order within a bucket varies from run to run, which changes only which
  // block computes a tile.  Problems that take no fused tiles keep a slot
  // with an empty range.
  __shared__ int32_t s_pos[2 * kKBuckets];
  auto ford = array(w.fused_order, G);
  if (thread.index() < 2 * kKBuckets) s_pos[thread.index()] = 0;
  sync(thread);
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    if (g < G) {
      const desc_gemm_problem p = pr[g];
      atomicAdd(&s_pos[plan_key(p, tile_edge<kCfg>(p.M, p.N) == kPadBig)], 1);
    }
  }
  sync(thread);
  if (thread.index() == 0) {
    int32_t at = 0;
    for (int k = 0; k < 2 * kKBuckets; ++k) {
      const int32_t c = s_pos[k];
      s_pos[k] = at;
      at += c;
    }
  }
  sync(thread);
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    if (g < G) {
      const desc_gemm_problem p = pr[g];
      ford[atomicAdd(&s_pos[plan_key(p, tile_edge<kCfg>(p.M, p.N) == kPadBig)], 1)] = (int32_t)g;
    }
  }
  sync(thread);
  int64_t c_slot = 0;
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t i = base + thread.index();
    int64_t ft = 0;
    if (i < G) {
      const desc_gemm_problem p = pr[ford[i]];
      const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
      if (!d.empty && !d.huge && fused_for<kCfg>(p)) {
        const int64_t e = tile_edge<kCfg>(p.M, p.N);
        ft = (round_up(p.M, e) / e) * (round_up(p.N, e) / e);
      }
    }
    int64_t e_ft;
    const int64_t t_ft = block_excl(ft, &e_ft, lds);
    if (i < G) fts[i] = c_slot + e_ft;
    c_slot += t_ft;
  }
  if (thread.index() == 0) {
    const bool fits = c_huge == 0 && c_pl <= w.planes_bytes;
    nts[G] = c_nt;
    sps[G] = c_sp;
    fts[G] = c_ft;
    w.totals[0] = fits ? c_nt : 0;
    w.totals[1] = fits ? c_sp : 0;
    w.totals[2] = fits ? c_ft : 0;
    w.error[0] = fits ? 0u : kDevPlanes;
  }
}

// The bf16 planes of problem g.
struct Planes {
  uint16_t *ah, *al, *bh, *bl;
};
// Problem g's region of the planes area (plane_off[g] bytes in, 256-byte
// aligned) holds Ah, Al as [Ma][Kp] and Bh^T, Bl^T as [Na][Kp], one after
// the other: a view over the region, split at the plane boundaries.
__device__ __forceinline__ Planes planes_of(const Bf16Ws& w, idx_t g, const Bf16Dims& d) {
  const idx_t off = array(w.plane_off, g + 1)[g];
  auto area = array((uint16_t*)w.planes, w.planes_bytes / 2);
  auto mine = area.snd(off / 2);                       // this problem's region
  const idx_t a = d.Ma * d.Kp, b = d.Na * d.Kp;
  return {&mine.snd(0)[0], &mine.snd(a)[0], &mine.snd(2 * a)[0], &mine.snd(2 * a + b)[0]};
}

// Split item: a 64 x 64 tile of A (rows r0.., k0..) into Ah, Al, or a
// 64 x 64 tile of B (k0.., n0..) into Bh^T, Bl^T through LDS.  Positions
// past M, N or K are written as zeros.
__global__ __launch_bounds__(kBlock) void bf16_split_kernel(const desc_gemm_problem* probs,
                                                            int64_t G, Bf16Ws w) {
  __shared__ float tile_lds[64 * 65];
  __shared__ int64_t s_g;
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  auto tile = matrix(tile_lds, 64, 65);
  const int64_t T = w.totals[1];
  const int tx = (int)thread.index() % 16, ty = (int)thread.index() / 16;
  for (idx_t t = block.index(); t < T; t += block.count()) {
    if (thread.index() < kWave) {
      const idx_t g = wave_owner(w.split_start, G, t);
      if (thread.index() == 0) s_g = g;
    }
    sync(thread);
    const idx_t g = wave::uniform_i64(s_g);
    const desc_gemm_problem p = array(probs, G)[g];
    const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
    const Planes pl = planes_of(w, g, d);
    const idx_t local = t - array(w.split_start, G + 1)[g];
    const idx_t kt = d.Kp / kPad, a_items = (d.Ms / kPad) * kt;
    if (local < a_items) {
      const idx_t r0 = (local / kt) * kPad, k0 = (local % kt) * kPad;
      auto a = matrix(p.A, p.M, p.lda);
      auto h = matrix(pl.ah, d.Ma, d.Kp);
      auto l = matrix(pl.al, d.Ma, d.Kp);
      const bool vec = gemm_f32::vec_ok(p.A, p.lda, p.A, p.lda);
#pragma unroll
      for (int i = 0; i < 4; ++i) {            // rows ty + 16 i, k = 4 tx ..
        const idx_t r = r0 + ty + 16 * i, c = k0 + 4 * tx;
        f32x4 v;
        if (vec && r < p.M && c + 4 <= p.K) {
          v = *(const f32x4*)&a.at(r, c);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (r < p.M && c + j < p.K) ? a.at(r, c + j) : 0.f;
        }
        const lowp::Split4 sp = lowp::split_bf16x4(v[0], v[1], v[2], v[3]);
        *(u16x4*)&h.at(r, c) = sp.hi;
        *(u16x4*)&l.at(r, c) = sp.lo;
      }
    } else {
      const idx_t j0 = local - a_items, ntl = d.Ns / kPad;
      const idx_t k0 = (j0 / ntl) * kPad, n0 = (j0 % ntl) * kPad;
      auto b = matrix(p.B, p.K, p.ldb);
      auto h = matrix(pl.bh, d.Na, d.Kp);
      auto l = matrix(pl.bl, d.Na, d.Kp);
      const bool vec = gemm_f32::vec_ok(p.B, p.ldb, p.B, p.ldb);
#pragma unroll
      for (int i = 0; i < 4; ++i) {            // rows (k) ty + 16 i, columns (n) 4 tx ..
        const idx_t r = ty + 16 * i, c = 4 * tx;
        f32x4 v;
        if (vec && k0 + r < p.K && n0 + c + 4 <= p.N) {
          v = *(const f32x4*)&b.at(k0 + r, n0 + c);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            v[j] = (k0 + r < p.K && n0 + c + j < p.N) ? b.at(k0 + r, n0 + c + j) : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) tile.at(r, c + j) = v[j];
      }
      sync(thread);
#pragma unroll
      for (int i = 0; i < 4; ++i) {            // output rows (n) ty + 16 i, k = 4 tx ..
        const idx_t c = ty + 16 * i, r = 4 * tx;
        const lowp::Split4 sp = lowp::split_bf16x4(tile.at(r, c), tile.at(r + 1, c),
                                                   tile.at(r + 2, c), tile.at(r + 3, c));
        *(u16x4*)&h.at(n0 + c, k0 + r) = sp.hi;
        *(u16x4*)&l.at(n0 + c, k0 + r) = sp.lo;
      }
    }
    sync(thread);   // s_g and the LDS tile are reused by the next item
  }
}

// Occupancy targets: four blocks per CU (a wave in 128 registers) with the
// 64 x 64 tile alone, two (256 registers) when the 128 x 128 tile can run;
// the tile coordinates and the problem index are kept in scalar registers
// so that only the tile's own state takes vector ones.
template <int kCfg>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kSmallOnly<kCfg> ? 4 : 2))) void bf16_nt_kernel(const desc_gemm_problem* probs,
                                                         int64_t G, Bf16Ws w) {
  __shared__ __attribute__((aligned(16)))
  uint8_t lds[kSmallOnly<kCfg> ? NtSmall::lds_bytes : NtBig::lds_bytes];
  __shared__ int64_t s_g;
  auto block = block_x();
  auto thread = thread_x<kBlock>();
  const int64_t T = w.totals[0];
  const layout::TileWalk walk = layout::tile_walk(block.index(), block.count());
  for (idx_t l = walk.first;; l += walk.per) {
    const idx_t t = walk.tile(l);
    if (t >= T) break;
    if (thread.index() < kWave) {
      const idx_t g = wave_owner(w.nt_start, G, t);
      if (thread.index() == 0) s_g = g;
    }
    sync(thread);
    const idx_t g = wave::uniform_i64(s_g);
    const desc_gemm_problem p = array(probs, G)[g];
    const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
    const Planes pl = planes_of(w, g, d);
    const idx_t local = t - array(w.nt_start, G + 1)[g];
    const NtOperands ops{{(const uint8_t*)pl.ah, (const uint8_t*)pl.al},
                         {(const uint8_t*)pl.bh, (const uint8_t*)pl.bl},
                         d.Kp * 2, p.C, p.ldc, p.M, p.N, nullptr, nullptr};
    // the tile coordinates come out of a vector division: made scalar again
    if constexpr (kSmallOnly<kCfg>) {
      const idx_t tn = d.Ns / kPad;
      gemm_nt::tile<NtSmall>(ops, wave::uniform_i64(local / tn), wave::uniform_i64(local % tn),
                             lds);
    } else {
      const idx_t tn = round_up(p.N, kPadBig) / kPadBig;
      gemm_nt::tile<NtBig>(ops, wave::uniform_i64(local / tn), wave::uniform_i64(local % tn),
                           lds);
    }
    sync(thread);   // s_g and the LDS stages are reused by the next tile
  }
}

// The fused form: output tiles straight from the FP32 operands, split into
// hi and lo while they are staged into LDS.
template <int kCfg>
__global__ __launch_bounds__(FusedNt<kCfg>::threads)
__attribute__((amdgpu_waves_per_eu(kSmallOnly<kCfg> ? 3 : 2)))
void bf16_fused_kernel(const desc_gemm_problem* probs, int64_t G, Bf16Ws w) {
  static_assert(kFused<kCfg>, "fused configurations only");
  using Nt = FusedNt<kCfg>;
  constexpr int kThreads = Nt::threads;
  __shared__ __attribute__((aligned(16))) uint8_t lds[Nt::lds_bytes];
  __shared__ int64_t s_g;
  auto block = block_x();
  auto thread = thread_x<kThreads>();
  const int64_t T = w.totals[2];
  const layout::TileWalk walk = layout::tile_walk(block.index(), block.count());
  for (idx_t l = walk.first;; l += walk.per) {
    const idx_t t = walk.tile(l);
    if (t >= T) break;
    if (thread.index() < kWave) {   // the slot of tile t in the fused order
      const idx_t slot = wave_owner(w.fused_start, G, t);
      if (thread.index() == 0) s_g = slot;
    }
    sync(thread);
    const idx_t slot = wave::uniform_i64(s_g);
    const idx_t g = array(w.fused_order, G)[slot];
    const desc_gemm_problem p = array(probs, G)[g];
    const idx_t local = t - array(w.fused_start, G + 1)[slot];
    constexpr int64_t e = kSmallOnly<kCfg> ? kPad : kPadBig;
    const idx_t tn = round_up(p.N, e) / e;
    const idx_t tm = wave::uniform_i64(local / tn), tc = wave::uniform_i64(local % tn);
    if (p.K <= 0) {                 // nothing to load: the tile is zero
      auto c = matrix(p.C, p.M, p.ldc);
      for (idx_t i = thread.index(); i < e * e; i += kThreads) {
        const idx_t r = tm * e + i / e, col = tc * e + i % e;
        if (r < p.M && col < p.N) c.at(r, col) = 0.f;
      }
    } else {
      const gemm_nt::F32Operands f{p.A, p.lda, p.B, p.ldb, p.M, p.N, p.K};
      if (gemm_f32::vec_ok(p.A, p.lda, p.A, p.lda) && p.K % 4 == 0)
        gemm_nt::tile_split<Nt, true>(f, p.C, p.ldc, tm, tc, lds);
      else
        gemm_nt::tile_split<Nt, false>(f, p.C, p.ldc, tm, tc, lds);
    }
    sync(thread);   // s_g and the LDS stages are reused by the next tile
  }
}

template <int kCfg>
hipError_t launch_bf16x3(const desc_gemm_problem* problems, int64_t G, const Bf16Ws& w,
                         hipStream_t s) {
  static int split_grid[64] = {0}, nt_grid[64] = {0};
  hipLaunchKernelGGL(bf16_plan_kernel<kCfg>, dim3(1), dim3(kBlock), 0, s, problems, G, w);
  if constexpr (kFused<kCfg>) {
    static int fused_grid[64] = {0};
    constexpr int kThreads = FusedNt<kCfg>::threads;
    const int gf = launch::resident_grid(bf16_fused_kernel<kCfg>, fused_grid, 1, kThreads);
    hipLaunchKernelGGL(bf16_fused_kernel<kCfg>, dim3((unsigned)gf), dim3(kThreads), 0, s,
                       problems, G, w);
  }
  // planes: every problem in configurations 0-2, those with strides past the
  // split source's limit in the fused ones (the kernels exit at once if none)
  const int gs = launch::resident_grid(bf16_split_kernel, split_grid, 4, kBlock);
  const int gn = launch::resident_grid(bf16_nt_kernel<kCfg>, nt_grid, 2, kBlock);
  hipLaunchKernelGGL(bf16_split_kernel, dim3((unsigned)gs), dim3(kBlock), 0, s, problems, G, w);
  hipLaunchKernelGGL(bf16_nt_kernel<kCfg>, dim3((unsigned)gn), dim3(kBlock), 0, s, problems, G,
                     w);
  return hipGetLastError();
}

// FP32 tile choice: 128 x 128 tiles for problems with M, N >= 256 and 64 x 64
// otherwise, or 64 x 64 tiles throughout (more, smaller tiles balance better
// over the CUs when the problems are small), in the first or the row-major-A
// tile form.
constexpr const char* kNames[] = {"tile128_or_64", "tile64", "tile64_rm_d2"};
constexpr int kDefaults[tune::kClasses] = {1, 1, 1, 1};
constexpr int64_t kBigMin[] = {256, INT64_MAX, INT64_MAX};
const bool kRegistered =
    (tune::register_op(tune::kGemmGrouped, "gemm_grouped", 3, kNames, kDefaults), true);

constexpr const char* kNamesBf16[] = {"tile64", "tile128", "fused64", "fused128"};
constexpr int kDefaultsBf16[tune::kClasses] = {3, 3, 3, 3};
const bool kRegisteredBf16 =
    (tune::register_op(tune::kGemmGroupedBf16x3, "gemm_grouped_bf16x3", 4, kNamesBf16,
                       kDefaultsBf16), true);

}  // namespace

namespace launch {

size_t gemm_grouped_bf16x3_head(int64_t G) { return bf16_head_bytes(G); }

size_t gemm_grouped_bf16x3_workspace(const desc_gemm_problem* host, int64_t G) {
  const int cfg =
      tune::get(tune::kGemmGroupedBf16x3, tune::size_class(tune::kGemmGroupedBf16x3, G));
  size_t total = bf16_head_bytes(G);
  for (int64_t g = 0; g < G; ++g) {
    const desc_gemm_problem& p = host[g];
    const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
    if (d.huge) return SIZE_MAX;
    if (fused_route(cfg, p.lda, p.ldb)) continue;   // staged from FP32: no planes
    const size_t b = (size_t)bf16_plane_bytes(d);
    if (total + b < total) return SIZE_MAX;
    total += b;
  }
  return total;
}

size_t gemm_grouped_bf16x3_workspace_uniform(const desc_gemm_problem& p, int64_t G) {
  const int cfg =
      tune::get(tune::kGemmGroupedBf16x3, tune::size_class(tune::kGemmGroupedBf16x3, G));
  const size_t head = bf16_head_bytes(G);
  const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
  if (d.huge) return SIZE_MAX;
  if (G == 0 || fused_route(cfg, p.lda, p.ldb)) return head;
  const size_t b = (size_t)bf16_plane_bytes(d);
  if (b != 0 && (size_t)G > (SIZE_MAX - head) / b) return SIZE_MAX;
  return head + (size_t)G * b;
}

hipError_t gemm_grouped_bf16x3(const desc_gemm_problem* problems, int64_t G, void* ws,
                               size_t ws_bytes, hipStream_t s) {
  (void)kRegisteredBf16;
  const Bf16Ws w = bf16_carve(ws, ws_bytes, G);
  // the size class is taken from the problem count
  switch (tune::get(tune::kGemmGroupedBf16x3, tune::size_class(tune::kGemmGroupedBf16x3, G))) {
    case 1: return launch_bf16x3<1>(problems, G, w, s);
    case 2: return launch_bf16x3<2>(problems, G, w, s);
    case 3: return launch_bf16x3<3>(problems, G, w, s);
    default: return launch_bf16x3<0>(problems, G, w, s);
  }
}

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
                     kBigMin[cfg >= 0 && cfg < 3 ? cfg : 1], w.total, w.tile_start, w.order,
                     w.big);
  if (cfg == 2)
    hipLaunchKernelGGL((grouped_gemm_kernel<false, true>),
                       dim3((unsigned)persistent_grid<false, true>()), dim3(kBlock), 0, s,
                       problems, G, w.total, w.tile_start, w.order, w.big);
  else if (cfg == 1)
    hipLaunchKernelGGL((grouped_gemm_kernel<false, false>),
                       dim3((unsigned)persistent_grid<false, false>()), dim3(kBlock), 0, s,
                       problems, G, w.total, w.tile_start, w.order, w.big);
  else
    hipLaunchKernelGGL((grouped_gemm_kernel<true, false>),
                       dim3((unsigned)persistent_grid<true, false>()), dim3(kBlock), 0, s,
                       problems, G, w.total, w.tile_start, w.order, w.big);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
