// transpose.hip -- out-of-place transpose of a row-major rows x cols matrix
// of 32-bit words (the "matrix transposition" benchmark of Sec. 5 and the
// running example of Sec. 1).
//
// The structure is the paper's: every block owns one tile, its threads copy
// the tile from the input into an LDS buffer, the block synchronises, and
// the threads copy the tile back out transposed, so both the global reads
// and the global writes run along rows.  On CDNA the tile is 64 x 64 words
// and a block is 256 threads seen as a [16][16] block (Listing 2 uses a
// 32 x 32 tile and [8][32] threads):
//
//   read  : thread (y, x) copies rows y, y+16, y+32, y+48 of the tile, 16
//           bytes per row (group_by_tile::<64,16> over int32x4 columns, then
//           group_by_row::<64,4>);
//   write : the same thread writes rows y, y+16, ... of the transposed tile,
//           each four consecutive words being one 16-byte store, and reads
//           them from column y+16i, rows 4x..4x+3 of the LDS tile.
//
// The LDS tile has a row pitch of 65 words, so that both the row-wise
// writes and the column-wise reads of a wave fall into distinct banks.
// Tiles on the ragged right or bottom edge (and unaligned matrices) go
// through a guarded element-by-element copy with the same tile and barrier.
// The kernel moves bit patterns only: NaN payloads, signed zeros and
// subnormals pass unchanged.
#include "common.hpp"
#include "launch.hpp"
#include "view.hpp"

namespace desc {
namespace {

constexpr int kT = 64;            // tile edge (words)
constexpr int kPitch = kT + 1;    // LDS row pitch (words)
constexpr int kBlock = 256;
constexpr int kTY = 16, kTX = 16; // threads as [16][16]

template <bool kVec>
__global__ __launch_bounds__(kBlock) void transpose32_kernel(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out,
                                                             int64_t rows, int64_t cols) {
  __shared__ uint32_t lds[kT * kPitch];
  auto bx = block_x();   // column tile of the input
  auto by = block_y();   // row tile of the input
  auto thread = thread_x<kBlock>();
  const Block bz{(idx_t)blockIdx.z, (idx_t)gridDim.z};   // matrix of the batch

  // The LDS tile as [64][65] words with the padding column split off.
  auto tile = matrix(lds, kT, kPitch).fst<1>(kT);            // [64][64]

  const bool full = kVec && (by.index() + 1) * kT <= rows && (bx.index() + 1) * kT <= cols;
  if (full) {
    auto t2 = thread_yx<kTY, kTX>();
    // input tile (by, bx), as [64 rows][16 groups of 4 words]
    auto a = group_by_tile<kT, kT / 4>(
                 matrices((const u32x4*)in, bz.count(), rows, cols / 4).select(bz))
                 .select(by).select(bx);
    auto a_mine = group_by_row<kT, 4>(a).select(t2.y).select(t2.x);           // [4]
    auto l_mine = group_by_row<kT, 4>(tile.group<4, 1>()).select(t2.y).select(t2.x);  // [4][4]
    u32x4 v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = __builtin_nontemporal_load(&a_mine[i]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      auto l = l_mine.idx(i);
      l[0] = v[i].x; l[1] = v[i].y; l[2] = v[i].z; l[3] = v[i].w;
    }
    sync(thread);
    // output tile (bx, by) of the cols x rows result
    auto b = group_by_tile<kT, kT / 4>(
                 matrices((u32x4*)out, bz.count(), cols, rows / 4).select(bz))
                 .select(bx).select(by);
    auto b_mine = group_by_row<kT, 4>(b).select(t2.y).select(t2.x);            // [4]
    // the LDS tile read column-wise: element (c, x, k) = tile[4x + k][c]
    auto lt = group_by_row<kT, 4>(tile.transpose().group<4, 1>()).select(t2.y).select(t2.x);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      auto l = lt.idx(i);
      u32x4 w;
      w.x = l[0]; w.y = l[1]; w.z = l[2]; w.w = l[3];
      __builtin_nontemporal_store(w, &b_mine[i]);
    }
  } else {
    // Ragged edge: element e of the tile is (e / 64, e % 64); guard both sides.
    auto a = matrices(in, bz.count(), rows, cols).select(bz);
    auto b = matrices(out, bz.count(), cols, rows).select(bz);
    const idx_t r0 = by.index() * kT, c0 = bx.index() * kT;
    for (idx_t e = thread.index(); e < kT * kT; e += kBlock) {
      const idx_t r = e / kT, c = e % kT;
      if (r0 + r < rows && c0 + c < cols) tile.at(r, c) = a.at(r0 + r, c0 + c);
    }
    sync(thread);
    for (idx_t e = thread.index(); e < kT * kT; e += kBlock) {
      const idx_t c = e / kT, r = e % kT;
      if (r0 + r < rows && c0 + c < cols) b.at(c0 + c, r0 + r) = tile.at(r, c);
    }
  }
}

}  // namespace

namespace launch {

hipError_t transpose_32(const uint32_t* in, uint32_t* out, int64_t batch, int64_t rows,
                        int64_t cols, hipStream_t s) {
  if (batch == 0 || rows == 0 || cols == 0) return hipSuccess;
  const dim3 grid((unsigned)((cols + kT - 1) / kT), (unsigned)((rows + kT - 1) / kT),
                  (unsigned)batch);
  const bool vec = rows % 4 == 0 && cols % 4 == 0 && (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(transpose32_kernel<true>, grid, dim3(kBlock), 0, s, in, out, rows, cols);
  else
    hipLaunchKernelGGL(transpose32_kernel<false>, grid, dim3(kBlock), 0, s, in, out, rows, cols);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
