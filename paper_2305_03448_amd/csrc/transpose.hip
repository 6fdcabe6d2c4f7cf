// transpose.hip -- out-of-place transpose of a row-major rows x cols matrix
// of 32-bit words (the "matrix transposition" benchmark of Sec. 5 and the
// running example of Sec. 1).
//
// The structure is the paper's: every block owns one tile, its threads copy
// the tile from the input into an LDS buffer, the block synchronises, and
// the threads copy the tile back out transposed, so both the global reads
// and the global writes run along rows.  On CDNA a tile is T x T words
// (T = 32, 64 or 128; Listing 2 uses 32) and a block is 256 threads seen as
// a [256/(T/4)][T/4] block, every thread moving 16 bytes per row:
//
//   read  : thread (y, x) copies rows y, y+TY, y+2TY, ... of the tile, words
//           4x..4x+3 of each (group_by_tile::<T,T/4> over int32x4 columns,
//           then group_by_row::<T,T/TY>);
//   write : the same thread writes rows y, y+TY, ... of the transposed tile,
//           each four consecutive words being one 16-byte store, and reads
//           them from column y+TY*i, rows 4x..4x+3 of the LDS tile.
//
// The LDS tile has a row pitch of T+1 words, so that the column-wise reads
// of a wave spread over the banks.
// Blocks take the column tiles of their row of tiles in diagonal order
// (block (x, y) takes tile (x + y mod the tiles per row, y)): with the plain
// order the blocks in flight together write output rows a power-of-two
// stride apart, which measured 10-13 % slower on MI355X.
// Tiles on the ragged right or bottom edge (and unaligned matrices) go
// through a guarded element-by-element copy with the same tile and barrier.
// The kernel moves bit patterns only: NaN payloads, signed zeros and
// subnormals pass unchanged.
#include "common.hpp"
#include "launch.hpp"
#include "layouts.hpp"
#include "tuning.hpp"
#include "view.hpp"

namespace desc {
namespace {

constexpr int kBlock = 256;

template <int kT, bool kNt, int kThreads>
struct TransposeShape {
  static constexpr int block = kThreads;     // threads per block
  static constexpr int t = kT;               // tile edge (words)
  static constexpr int pitch = kT + 1;       // LDS row pitch (words)
  static constexpr int tx = kT / 4;          // threads along a row (16 bytes each)
  static constexpr int ty = kThreads / tx;   // threads along a column
  static constexpr int items = kT / ty;      // rows per thread
  static constexpr bool nt = kNt;
  static_assert(ty * items == kT, "tile rows must divide among the thread rows");
};
// 256 threads per block, and 512 (twice the waves per tile, half the rows
// per thread).
template <int kT, bool kNt>
struct TransposeCfg : TransposeShape<kT, kNt, kBlock> {};
template <int kT, bool kNt>
struct TransposeCfg512 : TransposeShape<kT, kNt, 512> {};

template <bool kNt, class T>
__device__ __forceinline__ T load16(const T* p) {
  if constexpr (kNt) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool kNt, class T>
__device__ __forceinline__ void store16(T v, T* p) {
  if constexpr (kNt) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <class C, bool kVec>
__global__ __launch_bounds__(C::block) void transpose32_kernel(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out,
                                                             int64_t rows, int64_t cols) {
  constexpr int T = C::t, TY = C::ty, TX = C::tx, IT = C::items;
  __shared__ uint32_t lds[T * C::pitch];
  // Column tile of the input in diagonal order: row tile by starts at column
  // tile by, so that the blocks in flight together write output rows spread
  // over the matrix rather than rows a power-of-two stride apart.
  const Block bx{((idx_t)blockIdx.x + (idx_t)blockIdx.y) % (idx_t)gridDim.x, (idx_t)gridDim.x};
  auto by = block_y();   // row tile of the input
  auto thread = thread_x<C::block>();
  const Block bz{(idx_t)blockIdx.z, (idx_t)gridDim.z};   // matrix of the batch

  // The LDS tile as [T][T+1] words with the padding column split off.
  auto tile = matrix(lds, T, C::pitch).template fst<1>(T);            // [T][T]

  const bool full = kVec && (by.index() + 1) * T <= rows && (bx.index() + 1) * T <= cols;
  if (full) {
    auto t2 = thread_yx<TY, TX>();
    // input tile (by, bx), as [T rows][T/4 groups of 4 words]
    auto a_mine = layout::tile_rows<T, IT>(
        matrices((const u32x4*)in, bz.count(), rows, cols / 4).select(bz), by, bx, t2.y, t2.x);
    auto l_mine = layout::lds_rows<T, IT>(tile, t2.y, t2.x);                              // [IT][4]
    u32x4 v[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) v[i] = load16<C::nt>(&a_mine[i]);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      auto l = l_mine.idx(i);
      l[0] = v[i].x; l[1] = v[i].y; l[2] = v[i].z; l[3] = v[i].w;
    }
    sync(thread);
    // output tile (bx, by) of the cols x rows result
    auto b_mine = layout::tile_rows<T, IT>(
        matrices((u32x4*)out, bz.count(), cols, rows / 4).select(bz), bx, by, t2.y, t2.x);
    // the LDS tile read column-wise: element (i, k) = tile[4x + k][y + TY i]
    auto lt = layout::lds_cols<T, IT>(tile, t2.y, t2.x);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      auto l = lt.idx(i);
      u32x4 w;
      w.x = l[0]; w.y = l[1]; w.z = l[2]; w.w = l[3];
      store16<C::nt>(w, &b_mine[i]);
    }
  } else {
    // Ragged edge: element e of the tile is (e / T, e % T); guard both sides.
    auto a = matrices(in, bz.count(), rows, cols).select(bz);
    auto b = matrices(out, bz.count(), cols, rows).select(bz);
    const idx_t r0 = by.index() * T, c0 = bx.index() * T;
    for (idx_t e = thread.index(); e < T * T; e += C::block) {
      const idx_t r = e / T, c = e % T;
      if (r0 + r < rows && c0 + c < cols) tile.at(r, c) = a.at(r0 + r, c0 + c);
    }
    sync(thread);
    for (idx_t e = thread.index(); e < T * T; e += C::block) {
      const idx_t c = e / T, r = e % T;
      if (r0 + r < rows && c0 + c < cols) b.at(c0 + c, r0 + r) = tile.at(r, c);
    }
  }
}

template <class C>
hipError_t launch_transpose(const uint32_t* in, uint32_t* out, int64_t batch, int64_t rows,
                            int64_t cols, hipStream_t s) {
  constexpr int T = C::t;
  const dim3 grid((unsigned)((cols + T - 1) / T), (unsigned)((rows + T - 1) / T),
                  (unsigned)batch);
  const bool vec = rows % 4 == 0 && cols % 4 == 0 && (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL((transpose32_kernel<C, true>), grid, dim3(C::block), 0, s, in, out, rows,
                       cols);
  else
    hipLaunchKernelGGL((transpose32_kernel<C, false>), grid, dim3(C::block), 0, s, in, out, rows,
                       cols);
  return hipGetLastError();
}

// ----------------------------------------------------------------- other element sizes
// The same kernel for elements of 1, 2 or 8 bytes (the paper's own example
// moves doubles): a 16-byte group holds kV = 16 / sizeof(E) elements and a
// tile is T x T elements read by a [256 / (T/kV)][T/kV] block.  A column
// read of the LDS tile must spread over the banks: bytes pad the rows by 4
// bytes; 2- and 8-byte elements keep unpadded rows and XOR-swizzle the
// column index with the row (a whole-element pad cannot separate the 64
// rows one wave reads): doubles by c ^ ((r / 2) % 32), which gives the 32
// rows a half-wave reads 32 different 8-byte bank pairs, and 2-byte elements
// by c ^ 4 ((r / 8) % 16), which gives the 16 rows of a wave different
// dword columns while keeping element pairs in one dword.
template <class E, int kT>
struct TransposeCfgE {
  static constexpr int v = 16 / (int)sizeof(E);            // elements per 16-byte group
  static constexpr int t = kT;
  static constexpr int pad = sizeof(E) == 1 ? 4 : 0;
  static constexpr int pitch = kT + pad;
  static constexpr int tx = kT / v;
  static constexpr int ty = kBlock / tx;
  static constexpr int items = kT / ty;
  static_assert(tx * ty == kBlock && ty * items == kT, "tile rows must divide among the threads");
};

template <class C, class E, bool kVec>
__global__ __launch_bounds__(kBlock) void transpose_elem_kernel(const E* __restrict__ in,
                                                                E* __restrict__ out, int64_t rows,
                                                                int64_t cols) {
  constexpr int T = C::t, TY = C::ty, TX = C::tx, IT = C::items, V = C::v;
  typedef E vec_t __attribute__((ext_vector_type(V)));
  __shared__ __attribute__((aligned(16))) E lds[T * C::pitch];
  // Diagonal tile order: row tile by starts at column tile by, so that the
  // blocks in flight together write output rows spread over the matrix
  // rather than rows a power-of-two stride apart.
  const Block bx{((idx_t)blockIdx.x + (idx_t)blockIdx.y) % (idx_t)gridDim.x, (idx_t)gridDim.x};
  auto by = block_y();
  auto thread = thread_x<kBlock>();
  const Block bz{(idx_t)blockIdx.z, (idx_t)gridDim.z};
  auto tile = [&] {
    if constexpr (sizeof(E) == 8)
      return matrix(lds, T, T).template xor_swizzle_by<2, 32, 1>();     // [T][T]
    else if constexpr (sizeof(E) == 2)
      return matrix(lds, T, T).template xor_swizzle_by<8, 16, 4>();
    else
      return matrix(lds, T, C::pitch).template fst<1>(T);
  }();

  const bool full = kVec && (by.index() + 1) * T <= rows && (bx.index() + 1) * T <= cols;
  if (full) {
    auto t2 = thread_yx<TY, TX>();
    auto a_mine = layout::tile_rows<T, IT, V>(
        matrices((const vec_t*)in, bz.count(), rows, cols / V).select(bz), by, bx, t2.y, t2.x);
    auto l_mine = layout::lds_rows<T, IT, V>(tile, t2.y, t2.x);                        // [IT][V]
    vec_t g[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) g[i] = __builtin_nontemporal_load(&a_mine[i]);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      auto l = l_mine.idx(i);
#pragma unroll
      for (int k = 0; k < V; ++k) l[k] = g[i][k];
    }
    sync(thread);
    auto b_mine = layout::tile_rows<T, IT, V>(
        matrices((vec_t*)out, bz.count(), cols, rows / V).select(bz), bx, by, t2.y, t2.x);
    auto lt = layout::lds_cols<T, IT, V>(tile, t2.y, t2.x);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      auto l = lt.idx(i);
      vec_t w;
#pragma unroll
      for (int k = 0; k < V; ++k) w[k] = l[k];
      __builtin_nontemporal_store(w, &b_mine[i]);
    }
  } else {
    auto a = matrices(in, bz.count(), rows, cols).select(bz);
    auto b = matrices(out, bz.count(), cols, rows).select(bz);
    const idx_t r0 = by.index() * T, c0 = bx.index() * T;
    for (idx_t e = thread.index(); e < T * T; e += kBlock) {
      const idx_t r = e / T, c = e % T;
      if (r0 + r < rows && c0 + c < cols) tile.at(r, c) = a.at(r0 + r, c0 + c);
    }
    sync(thread);
    for (idx_t e = thread.index(); e < T * T; e += kBlock) {
      const idx_t c = e / T, r = e % T;
      if (r0 + r < rows && c0 + c < cols) b.at(c0 + c, r0 + r) = tile.at(r, c);
    }
  }
}

template <class E, int kT>
hipError_t launch_transpose_elem(const void* in, void* out, int64_t batch, int64_t rows,
                                 int64_t cols, hipStream_t s) {
  using C = TransposeCfgE<E, kT>;
  const dim3 grid((unsigned)((cols + kT - 1) / kT), (unsigned)((rows + kT - 1) / kT),
                  (unsigned)batch);
  const bool vec = rows % C::v == 0 && cols % C::v == 0 &&
                   (((uintptr_t)in | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL((transpose_elem_kernel<C, E, true>), grid, dim3(kBlock), 0, s,
                       (const E*)in, (E*)out, rows, cols);
  else
    hipLaunchKernelGGL((transpose_elem_kernel<C, E, false>), grid, dim3(kBlock), 0, s,
                       (const E*)in, (E*)out, rows, cols);
  return hipGetLastError();
}

constexpr const char* kNames[] = {"t64_nt", "t64", "t32_nt", "t32", "t128_nt", "t128",
                                   "t128_nt_b512", "t128_b512"};
constexpr int kDefaults[tune::kClasses] = {0, 0, 0, 0};
const bool kRegistered =
    (tune::register_op(tune::kTranspose32, "transpose_32", 8, kNames, kDefaults), true);

}  // namespace

namespace launch {

// Rows are tiled by at most 128 words, so a grid of 65535 row tiles covers
// any row count this bound admits.
int64_t transpose_max_rows() { return (int64_t)65535 * 32; }

hipError_t transpose_32(const uint32_t* in, uint32_t* out, int64_t batch, int64_t rows,
                        int64_t cols, hipStream_t s) {
  if (batch == 0 || rows == 0 || cols == 0) return hipSuccess;
  (void)kRegistered;
  const int64_t size = batch * rows * cols;
  switch (tune::get(tune::kTranspose32, tune::size_class(tune::kTranspose32, size))) {
    case 1: return launch_transpose<TransposeCfg<64, false>>(in, out, batch, rows, cols, s);
    case 2: return launch_transpose<TransposeCfg<32, true>>(in, out, batch, rows, cols, s);
    case 3: return launch_transpose<TransposeCfg<32, false>>(in, out, batch, rows, cols, s);
    case 4: return launch_transpose<TransposeCfg<128, true>>(in, out, batch, rows, cols, s);
    case 5: return launch_transpose<TransposeCfg<128, false>>(in, out, batch, rows, cols, s);
    case 6: return launch_transpose<TransposeCfg512<128, true>>(in, out, batch, rows, cols, s);
    case 7: return launch_transpose<TransposeCfg512<128, false>>(in, out, batch, rows, cols, s);
    default: return launch_transpose<TransposeCfg<64, true>>(in, out, batch, rows, cols, s);
  }
}

// Tiles of 128 elements for 1- and 2-byte elements, 64 for doubles (eight
// 16-byte groups per thread either way).
int64_t transpose_elem_max_rows(int64_t elem_bytes) {
  return (int64_t)65535 * (elem_bytes == 8 ? 64 : 128);
}

hipError_t transpose_elem(const void* in, void* out, int64_t elem_bytes, int64_t batch,
                          int64_t rows, int64_t cols, hipStream_t s) {
  if (batch == 0 || rows == 0 || cols == 0) return hipSuccess;
  switch (elem_bytes) {
    case 1: return launch_transpose_elem<uint8_t, 128>(in, out, batch, rows, cols, s);
    case 2: return launch_transpose_elem<uint16_t, 128>(in, out, batch, rows, cols, s);
    case 4:
      return transpose_32((const uint32_t*)in, (uint32_t*)out, batch, rows, cols, s);
    default: return launch_transpose_elem<uint64_t, 64>(in, out, batch, rows, cols, s);
  }
}

}  // namespace launch
}  // namespace desc
