// grouped.hip -- many independent GEMMs of uneven shapes in persistent
// launches (the batched form of the Sec. 5 matrix multiplication), in FP32
// or in the three-product split-BF16 mode.
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
#include "gemm_nt.hpp"
#include "launch.hpp"
#include "lowp.hpp"
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
// --------------------------------------------------------------------------
// Split-BF16 (three products) mode.  Every problem is padded to multiples of
// 64 in M, N and K (K at least 64, so K = 0 gives zero products through the
// same path), and its operands are split into bf16 planes in the workspace:
// Ah, Al as [Mp][Kp] and Bh^T, Bl^T as [Np][Kp].
//   plan kernel (one block): per problem the NT tiles, the split work items
//     and the byte offset of its planes, as exclusive prefixes; if the planes
//     do not fit the workspace, the error word is set and nothing is planned.
//   split kernel (persistent): 64 x 64 items -- A tiles split in place, B
//     tiles split and transposed through LDS.
//   NT kernel (persistent): 64 x 64 output tiles of the low-precision tile
//     routine, runs of 64 tiles per XCD as in the FP32 mode.
// --------------------------------------------------------------------------
constexpr int kPad = 64;
using NtTile = NtCfg<64, 64, 64, Bf16x3Mode, 2, 2, 2>;
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

constexpr int64_t kMaxDim = int64_t(1) << 40;         // larger M, N or K: refused
constexpr int64_t kMaxPlaneBytes = int64_t(1) << 44;  // larger planes of one problem: refused
struct Bf16Dims {
  int64_t Mp, Np, Kp;
  bool empty;   // M <= 0 or N <= 0: nothing to compute or store
  bool huge;    // a dimension or the planes beyond the limits above
};
__host__ __device__ inline Bf16Dims bf16_dims(int64_t M, int64_t N, int64_t K) {
  Bf16Dims d;
  d.empty = M <= 0 || N <= 0;
  d.huge = !d.empty && (M > kMaxDim || N > kMaxDim || K > kMaxDim);
  const bool none = d.empty || d.huge;
  d.Mp = none ? 0 : (M + kPad - 1) / kPad * kPad;
  d.Np = none ? 0 : (N + kPad - 1) / kPad * kPad;
  d.Kp = none ? 0 : (K <= kPad ? kPad : (K + kPad - 1) / kPad * kPad);   // K <= 0: one zero step
  d.huge = d.huge || (!none && d.Mp + d.Np > kMaxPlaneBytes / (4 * d.Kp));
  if (d.huge) d.Mp = d.Np = d.Kp = 0;
  return d;
}
// Four planes, 256-byte aligned (none for a refused problem).
__host__ __device__ inline int64_t bf16_plane_bytes(const Bf16Dims& d) {
  return (4 * (d.Mp + d.Np) * d.Kp + 255) / 256 * 256;
}

struct Bf16Ws {
  int64_t* totals;       // [0] NT tiles, [1] split items
  uint32_t* error;       // set when the planes do not fit
  int64_t* nt_start;     // [G + 1]
  int64_t* split_start;  // [G + 1]
  int64_t* plane_off;    // [G]
  uint8_t* planes;
  int64_t planes_bytes;  // room for the planes
};
size_t bf16_head_bytes(int64_t G) {
  return 256 + 3 * (((G + 1) * 8 + 255) & ~(size_t)255);   // planes start 256-byte aligned
}
Bf16Ws bf16_carve(void* ws, size_t ws_bytes, int64_t G) {
  uint8_t* w = (uint8_t*)ws;
  const size_t arr = ((G + 1) * 8 + 255) & ~(size_t)255;
  Bf16Ws r;
  r.totals = (int64_t*)w;
  r.error = (uint32_t*)(w + 16);
  r.nt_start = (int64_t*)(w + 256);
  r.split_start = (int64_t*)(w + 256 + arr);
  r.plane_off = (int64_t*)(w + 256 + 2 * arr);
  r.planes = w + bf16_head_bytes(G);
  r.planes_bytes = (int64_t)ws_bytes - (int64_t)bf16_head_bytes(G);
  return r;
}

__global__ __launch_bounds__(kBlock) void bf16_plan_kernel(const desc_gemm_problem* probs,
                                                           int64_t G, Bf16Ws w) {
  __shared__ int64_t lds[kBlock / kWave];
  auto thread = thread_x<kBlock>();
  auto pr = array(probs, G);
  auto nts = array(w.nt_start, G + 1);
  auto sps = array(w.split_start, G + 1);
  auto pof = array(w.plane_off, G);
  int64_t c_nt = 0, c_sp = 0, c_pl = 0, c_huge = 0;
  for (idx_t base = 0; base < G; base += kBlock) {
    const idx_t g = base + thread.index();
    int64_t nt = 0, sp = 0, pl = 0, huge = 0;
    if (g < G) {
      const Bf16Dims d = bf16_dims(pr[g].M, pr[g].N, pr[g].K);
      nt = (d.Mp / kPad) * (d.Np / kPad);
      sp = (d.Mp / kPad) * (d.Kp / kPad) + (d.Kp / kPad) * (d.Np / kPad);
      pl = bf16_plane_bytes(d);
      huge = d.huge;
    }
    int64_t e_nt, e_sp, e_pl, e_huge;
    const int64_t t_nt = block_excl(nt, &e_nt, lds);
    const int64_t t_sp = block_excl(sp, &e_sp, lds);
    const int64_t t_pl = block_excl(pl, &e_pl, lds);
    c_huge += block_excl(huge, &e_huge, lds);
    if (g < G) {
      nts[g] = c_nt + e_nt;
      sps[g] = c_sp + e_sp;
      pof[g] = c_pl + e_pl;
    }
    c_nt += t_nt;
    c_sp += t_sp;
    // at most 256 * 2^44 bytes per round: held below 2^60, no overflow
    c_pl = c_pl + t_pl < (int64_t(1) << 60) ? c_pl + t_pl : (int64_t(1) << 60);
  }
  if (thread.index() == 0) {
    const bool fits = c_huge == 0 && c_pl <= w.planes_bytes;
    nts[G] = c_nt;
    sps[G] = c_sp;
    w.totals[0] = fits ? c_nt : 0;
    w.totals[1] = fits ? c_sp : 0;
    w.error[0] = fits ? 0u : 1u;
  }
}

// Last i with start[i] <= t (the problem holding item t).
__device__ __forceinline__ idx_t owner(const int64_t* start, int64_t G, int64_t t) {
  auto st = array(start, G + 1);
  idx_t lo = 0, hi = G;
  while (hi - lo > 1) {
    const idx_t mid = (lo + hi) / 2;
    if (st[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// The bf16 planes of problem g.
struct Planes {
  uint16_t *ah, *al, *bh, *bl;
};
__device__ __forceinline__ Planes planes_of(const Bf16Ws& w, idx_t g, const Bf16Dims& d) {
  uint16_t* p = (uint16_t*)(w.planes + array(w.plane_off, g + 1)[g]);
  return {p, p + d.Mp * d.Kp, p + 2 * d.Mp * d.Kp, p + 2 * d.Mp * d.Kp + d.Np * d.Kp};
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
    if (thread.index() == 0) s_g = owner(w.split_start, G, t);
    sync(thread);
    const idx_t g = s_g;
    const desc_gemm_problem p = array(probs, G)[g];
    const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
    const Planes pl = planes_of(w, g, d);
    const idx_t local = t - array(w.split_start, G + 1)[g];
    const idx_t kt = d.Kp / kPad, a_items = (d.Mp / kPad) * kt;
    if (local < a_items) {
      const idx_t r0 = (local / kt) * kPad, k0 = (local % kt) * kPad;
      auto a = matrix(p.A, p.M, p.lda);
      auto h = matrix(pl.ah, d.Mp, d.Kp);
      auto l = matrix(pl.al, d.Mp, d.Kp);
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
        u16x4 vh, vl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const lowp::Split sp = lowp::split_bf16(v[j]);
          vh[j] = sp.hi;
          vl[j] = sp.lo;
        }
        *(u16x4*)&h.at(r, c) = vh;
        *(u16x4*)&l.at(r, c) = vl;
      }
    } else {
      const idx_t j0 = local - a_items, ntl = d.Np / kPad;
      const idx_t k0 = (j0 / ntl) * kPad, n0 = (j0 % ntl) * kPad;
      auto b = matrix(p.B, p.K, p.ldb);
      auto h = matrix(pl.bh, d.Np, d.Kp);
      auto l = matrix(pl.bl, d.Np, d.Kp);
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
        u16x4 vh, vl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const lowp::Split sp = lowp::split_bf16(tile.at(r + j, c));
          vh[j] = sp.hi;
          vl[j] = sp.lo;
        }
        *(u16x4*)&h.at(n0 + c, k0 + r) = vh;
        *(u16x4*)&l.at(n0 + c, k0 + r) = vl;
      }
    }
    sync(thread);   // s_g and the LDS tile are reused by the next item
  }
}

__global__ __launch_bounds__(NtTile::threads) void bf16_nt_kernel(const desc_gemm_problem* probs,
                                                                  int64_t G, Bf16Ws w) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[NtTile::lds_bytes];
  __shared__ int64_t s_g;
  auto block = block_x();
  auto thread = thread_x<NtTile::threads>();
  const int64_t T = w.totals[0];
  constexpr idx_t kRun = 64, kXcd = 8;
  const bool by_xcd = block.count() % kXcd == 0;
  const idx_t x = by_xcd ? block.index() % kXcd : 0;
  const idx_t per = by_xcd ? block.count() / kXcd : block.count();
  for (idx_t l = by_xcd ? block.index() / kXcd : block.index();; l += per) {
    const idx_t t = by_xcd ? (kXcd * (l / kRun) + x) * kRun + l % kRun : l;
    if (t >= T) break;
    if (thread.index() == 0) s_g = owner(w.nt_start, G, t);
    sync(thread);
    const idx_t g = s_g;
    const desc_gemm_problem p = array(probs, G)[g];
    const Bf16Dims d = bf16_dims(p.M, p.N, p.K);
    const Planes pl = planes_of(w, g, d);
    const idx_t local = t - array(w.nt_start, G + 1)[g], tn = d.Np / kPad;
    NtOperands ops{{(const uint8_t*)pl.ah, (const uint8_t*)pl.al},
                   {(const uint8_t*)pl.bh, (const uint8_t*)pl.bl},
                   d.Kp * 2, p.C, p.ldc, p.M, p.N, nullptr, nullptr};
    gemm_nt::tile<NtTile>(ops, local / tn, local % tn, lds);
    sync(thread);   // s_g and the LDS stages are reused by the next tile
  }
}

template <class K>
int resident_grid(K kernel, int threads, int fallback_per_cu) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess ||
      per < 1)
    per = fallback_per_cu;
  return cus * per;
}

constexpr const char* kNames[] = {"tile128_or_64", "tile64"};
constexpr int kDefaults[tune::kClasses] = {1, 1, 1, 1};
constexpr int64_t kBigMin[] = {256, INT64_MAX};
const bool kRegistered =
    (tune::register_op(tune::kGemmGrouped, "gemm_grouped", 2, kNames, kDefaults), true);

}  // namespace

namespace launch {

size_t gemm_grouped_bf16x3_head(int64_t G) { return bf16_head_bytes(G); }

size_t gemm_grouped_bf16x3_planes(int64_t M, int64_t N, int64_t K) {
  const Bf16Dims d = bf16_dims(M, N, K);
  return d.huge ? SIZE_MAX : (size_t)bf16_plane_bytes(d);
}

hipError_t gemm_grouped_bf16x3(const desc_gemm_problem* problems, int64_t G, void* ws,
                               size_t ws_bytes, hipStream_t s) {
  const Bf16Ws w = bf16_carve(ws, ws_bytes, G);
  static int grid_split = 0, grid_nt = 0;
  if (grid_split == 0) grid_split = resident_grid(bf16_split_kernel, kBlock, 4);
  if (grid_nt == 0) grid_nt = resident_grid(bf16_nt_kernel, NtTile::threads, 2);
  hipLaunchKernelGGL(bf16_plan_kernel, dim3(1), dim3(kBlock), 0, s, problems, G, w);
  hipLaunchKernelGGL(bf16_split_kernel, dim3((unsigned)grid_split), dim3(kBlock), 0, s, problems,
                     G, w);
  hipLaunchKernelGGL(bf16_nt_kernel, dim3((unsigned)grid_nt), dim3(NtTile::threads), 0, s,
                     problems, G, w);
  return hipGetLastError();
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
