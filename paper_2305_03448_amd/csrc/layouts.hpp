// layouts.hpp -- the views through which the kernels distribute data over
// blocks, waves and lanes.  Kept apart from the kernels so that the host-side
// enumeration tests check exactly the maps the kernels use.
#pragma once
#include "view.hpp"

namespace desc {
namespace layout {

// Wave-striped tiles: a rank-1 view of 4-element groups (int32x4, or a
// [n/4][4] scalar view) seen as [tiles][waves][rounds][64 lanes]; the
// result is the [rounds] groups of one lane of one wave of one tile.  Each
// wave owns a contiguous sub-tile and each round of a wave covers 64
// consecutive groups, so a wave's 16-byte accesses are one contiguous 1 KiB.
template <int kWaves, int kRounds, class V, class W, class L>
DESC_HD auto wave_striped(const V& groups, idx_t tile, const W& wave, const L& lane) {
  return groups.template group<64>()
      .template group<kRounds>()
      .template group<kWaves>()
      .idx(tile)
      .select(wave)
      .transpose()
      .select(lane);
}

// Block-striped tiles: [tiles][rounds][threads]; the [rounds] elements of one
// thread of tile t (round u of thread x is element u * threads + x).
template <int kThreads, int kRounds, class V, class T>
DESC_HD auto block_striped(const V& elems, idx_t tile, const T& thread) {
  return elems.template group<kThreads>().template group<kRounds>().idx(tile).transpose().select(
      thread);
}

// Tiled transposition.  `m` is a [rows][cols / kV] view of 16-byte groups of
// kV elements (kV = 4 for 32-bit words); tile (by, bx) is T x T elements,
// read by a [T / kItems][T / kV] block of threads, thread (y, x) taking rows
// y, y + T/kItems, ... of the tile (group_by_tile, then group_by_row).
template <int T, int kItems, int kV = 4, class V, class BY, class BX, class TY, class TX>
DESC_HD auto tile_rows(const V& m, const BY& by, const BX& bx, const TY& ty, const TX& tx) {
  return group_by_row<T, kItems>(group_by_tile<T, T / kV>(m).select(by).select(bx))
      .select(ty)
      .select(tx);
}

// The same thread's slots of the T x T LDS tile ([T][T] elements):
// [kItems][kV], row y + (T/kItems) i, elements kV x .. kV x + kV - 1.
template <int T, int kItems, int kV = 4, class V, class TY, class TX>
DESC_HD auto lds_rows(const V& tile, const TY& ty, const TX& tx) {
  return group_by_row<T, kItems>(tile.template group<kV, 1>()).select(ty).select(tx);
}

// The LDS tile read column-wise for the write-out: [kItems][kV], element
// (i, k) = tile[kV x + k][y + (T/kItems) i].
template <int T, int kItems, int kV = 4, class V, class TY, class TX>
DESC_HD auto lds_cols(const V& tile, const TY& ty, const TX& tx) {
  return group_by_row<T, kItems>(tile.transpose().template group<kV, 1>()).select(ty).select(tx);
}

// Fused split staging (the split-BF16 tile routine reading FP32 operands
// through buffer windows): a wave stages 16 rows x 8 kChunks values of k of
// A, lane l taking row l / kChunks of the wave's rows and the octet (8
// consecutive k) from 8 (l % kChunks); and an octet of B (8 rows of k) x 64
// columns, lane l taking column l.
template <int kChunks>
DESC_HD int split_a_row(int lane) { return lane / kChunks; }
template <int kChunks>
DESC_HD int split_a_k(int lane) { return 8 * (lane % kChunks); }
DESC_HD int split_b_col(int lane) { return lane; }

// FP32 GEMM, row-major tile form (gemm_f32.hpp tile_rowmajor): the LDS
// buffers of one stage are A as [BM][BK + 4] words and B as [BK][BN + 4].
// Stage store: group q (thread t's i-th, q = t + T i) of four words goes to
// row q / (BK/4), word 4 (q % (BK/4)) of A's buffer, and to row q / (BN/4),
// word 4 (q % (BN/4)) of B's.  Fragment reads: lane (half, c32) of wave
// (wm, wn) reads, at step group k4, A's row wm WTM + 32 i + c32 from word
// half BK/2 + k4 (four words) and B's row half BK/2 + k4 + kk, word
// wn WTN + 32 j + c32; the matrix instruction's two k slots take the two
// halves of the stage.
template <int kWidth>
DESC_HD int gemm_store_row(int q) { return q / (kWidth / 4); }
template <int kWidth>
DESC_HD int gemm_store_word(int q) { return 4 * (q % (kWidth / 4)); }
template <int kWTM>
DESC_HD int gemm_a_frag_row(int wm, int i, int c32) { return wm * kWTM + 32 * i + c32; }
template <int kBK>
DESC_HD int gemm_frag_k(int half, int k4) { return half * (kBK / 2) + k4; }
template <int kWTN>
DESC_HD int gemm_b_frag_word(int wn, int j, int c32) { return wn * kWTN + 32 * j + c32; }
// The same tile form with 16 x 16 x 4 instructions: the four k slots take
// the four quarters of the stage (lane l: row or column l % 16 of its
// fragment, k = (BK / 4) (l / 16) + kk at step kk), so a lane's A values of
// a stage are again one 16-byte read.
template <int kWTM>
DESC_HD int gemm16_a_frag_row(int wm, int i, int c16) { return wm * kWTM + 16 * i + c16; }
template <int kBK>
DESC_HD int gemm16_frag_k(int quarter) { return quarter * (kBK / 4); }
template <int kWTN>
DESC_HD int gemm16_b_frag_word(int wn, int j, int c16) { return wn * kWTN + 16 * j + c16; }

// Segmented forms (segmented.hip): segment s of length L_s gives
// ceil(L_s / U) units of at most U consecutive elements; unit_start is the
// exclusive prefix of the unit counts over the segments (S + 1 entries).
// Unit u belongs to the last segment s with unit_start[s] <= u, is unit
// j = u - unit_start[s] of it, and covers [off[s] + j U, min(off[s + 1],
// off[s] + (j + 1) U)); offsets are read clamped to [0, n].
DESC_HD int64_t seg_clamp(int64_t v, int64_t n) { return v < 0 ? 0 : (v > n ? n : v); }
DESC_HD int64_t seg_units(int64_t len, int64_t unit) {
  return len > 0 ? (len + unit - 1) / unit : 0;
}
template <class V>
DESC_HD idx_t seg_of_unit(const V& unit_start, int64_t S, int64_t u) {
  idx_t lo = 0, hi = S;   // answer in [lo, hi)
  while (hi - lo > 1) {
    const idx_t mid = (lo + hi) / 2;
    if (unit_start[mid] <= u) lo = mid; else hi = mid;
  }
  return lo;
}
struct SegUnit {
  idx_t seg, j, begin, len;   // segment, unit index inside it, first position, length
  bool single;                // the segment has one unit only
};
template <class VO, class VU>
DESC_HD SegUnit seg_unit(const VO& off, const VU& unit_start, int64_t n, int64_t S, int64_t unit,
                         int64_t u) {
  const idx_t s = seg_of_unit(unit_start, S, u);
  const idx_t j = u - unit_start[s];
  const idx_t b = seg_clamp(off[s], n) + j * unit;
  const idx_t e = seg_clamp(off[s + 1], n);
  return SegUnit{s, j, b, (e - b) < unit ? (e - b) : unit, (unit_start[s + 1] - unit_start[s]) == 1};
}

// Decoupled look-back over the earlier units of a segment: at window w a
// whole wave inspects the status words of units u - 1 - 64 w - lane, the
// lanes with 64 w + lane < j taking part (unit u is unit j of its segment),
// so the windows walk the segment's earlier units from the nearest back to
// its first and never leave the segment.
DESC_HD idx_t lookback_unit(idx_t u, idx_t window, int lane) { return u - 1 - 64 * window - lane; }
DESC_HD bool lookback_in_segment(idx_t j, idx_t window, int lane) { return 64 * window + lane < j; }

// Persistent tile walk (grouped.hip): block b of B walks steps l = l0,
// l0 + per, ... and step l takes tile t(l); the walk ends at the first
// t(l) >= T, t growing with l.  When B is a multiple of the 8 XCDs (blocks
// are dispatched round-robin over them, block b running on XCD b mod 8), the
// tile sequence is cut into runs of 64 consecutive tiles, run r going to XCD
// r mod 8: l0 = b / 8, per = B / 8, t(l) = (8 (l / 64) + b mod 8) 64 + l mod 64.
// Otherwise l0 = b, per = B, t(l) = l.
struct TileWalk {
  idx_t first, per, xcd;
  bool by_xcd;
  DESC_HD idx_t tile(idx_t l) const {
    return by_xcd ? (8 * (l / 64) + xcd) * 64 + l % 64 : l;
  }
};
DESC_HD TileWalk tile_walk(idx_t block, idx_t blocks) {
  const bool by_xcd = blocks % 8 == 0;
  return by_xcd ? TileWalk{block / 8, blocks / 8, block % 8, true}
                : TileWalk{block, blocks, 0, false};
}

// The float scan's hand-over (scan_f32.hip): tiles in groups of K; tile
// t = g K + p publishes its aggregate in slot t of the aggregates; its lane
// l < p waits for slot g K + l, and its lane 0 (g > 0) for slot g - 1 of the
// group prefixes, which the last tile of group g - 1 publishes (the group's
// tile p = K - 1, or the last tile of all).  A tile waits only for tiles
// with smaller indices.  The call's region is the T aggregate slots, then
// the group prefixes, two 64-bit words a slot.
template <int K>
DESC_HD idx_t handover_peer(idx_t tile, int lane) { return tile / K * K + lane; }
template <int K>
DESC_HD bool handover_publishes_group(idx_t tile, idx_t tiles) {
  return tile % K == K - 1 || tile == tiles - 1;
}
template <int K>
DESC_HD idx_t handover_words(idx_t tiles) { return 2 * tiles + 2 * ((tiles + K - 1) / K); }

}  // namespace layout
}  // namespace desc
