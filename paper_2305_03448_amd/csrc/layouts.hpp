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

}  // namespace layout
}  // namespace desc
