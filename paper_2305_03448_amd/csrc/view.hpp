// view.hpp -- execution resources and memory views as compile-time index maps.
//
// This is the layer that stands in for the paper's execution resources
// (Sec. 3.1: grid / block / thread, `sched`, `split`) and memory views
// (Sec. 3.2: `split`, `group`, `transpose`, `reverse`, `map`, and the select
// place expression `p[[e]]`).  Kernels reach memory only through a View; the
// single place where an index becomes an address is View::ref().  An index
// given to a view is rewritten by the view that was applied last first and
// then by each earlier one in turn, down to a row-major offset into the
// underlying array -- the order the paper's code generator uses (Sec. 5).
//
// Every map is a template, so the composition folds into plain integer
// arithmetic at compile time; group sizes are compile-time constants (the
// paper's nats) while array extents may be runtime values.
//
// Execution resources carry their own index and the number of siblings at
// that level.  `select` checks that the selected dimension has exactly as
// many elements as the resource has siblings (statically when both are
// compile-time constants), which is what makes the selection disjoint by
// construction: sibling i owns element i and nothing else.  `sync` is only
// defined for an unsplit block; calling it on a resource produced by `split`
// does not compile (Sec. 2/3: a barrier inside a divergent branch).
//
// The header compiles as plain C++17 on the host as well, so the index maps
// can be enumerated and checked without a GPU.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define DESC_HD __host__ __device__ __forceinline__
#else
#include <cassert>
#define DESC_HD inline
#endif

namespace desc {

using idx_t = int64_t;

// ---------------------------------------------------------------------------
// Index tuples
// ---------------------------------------------------------------------------
template <int R>
struct Idx {
  idx_t v[R > 0 ? R : 1];
  DESC_HD idx_t& operator[](int d) { return v[d]; }
  DESC_HD idx_t operator[](int d) const { return v[d]; }
};

// ---------------------------------------------------------------------------
// Index maps.  Each map has a rank R, extents ext(d) for d < R, and
// `to_parent` rewriting an Idx<R> into its parent's index; the root map
// (Dense) turns the index into a row-major element offset.
// ---------------------------------------------------------------------------

// Root: a contiguous row-major array with R dimensions, innermost last.
template <int R>
struct Dense {
  static constexpr int rank = R;
  idx_t e[R];
  DESC_HD idx_t ext(int d) const { return e[d]; }
  DESC_HD idx_t offset(const Idx<R>& i) const {
    idx_t o = i[0];
    for (int d = 1; d < R; ++d) o = o * e[d] + i[d];
    return o;
  }
};

// group<K> at depth D: dimension D of extent n becomes [n/K][K].
template <class P, idx_t K, int D>
struct GroupMap {
  static constexpr int rank = P::rank + 1;
  static_assert(K > 0, "group size must be positive");
  P p;
  DESC_HD idx_t ext(int d) const {
    return d < D ? p.ext(d) : d == D ? p.ext(D) / K : d == D + 1 ? K : p.ext(d - 1);
  }
  DESC_HD Idx<P::rank> to_parent(const Idx<rank>& i) const {
    Idx<P::rank> j;
    for (int d = 0; d < D; ++d) j[d] = i[d];
    j[D] = i[D] * K + i[D + 1];
    for (int d = D + 1; d < P::rank; ++d) j[d] = i[d + 1];
    return j;
  }
};

// transpose at depth D: swaps dimensions D and D+1.
template <class P, int D>
struct TransposeMap {
  static constexpr int rank = P::rank;
  static_assert(D + 1 < P::rank, "transpose needs two dimensions");
  P p;
  DESC_HD idx_t ext(int d) const { return d == D ? p.ext(D + 1) : d == D + 1 ? p.ext(D) : p.ext(d); }
  DESC_HD Idx<rank> to_parent(const Idx<rank>& i) const {
    Idx<rank> j = i;
    j[D] = i[D + 1];
    j[D + 1] = i[D];
    return j;
  }
};

// reverse at depth D: index k of dimension D reads n-1-k.
template <class P, int D>
struct ReverseMap {
  static constexpr int rank = P::rank;
  P p;
  DESC_HD idx_t ext(int d) const { return p.ext(d); }
  DESC_HD Idx<rank> to_parent(const Idx<rank>& i) const {
    Idx<rank> j = i;
    j[D] = p.ext(D) - 1 - i[D];
    return j;
  }
};

// split at depth D: dimension D is cut at `pos`; the first part keeps
// [0, pos), the second part [pos, n) shifted to start at 0.
template <class P, int D>
struct SplitMap {
  static constexpr int rank = P::rank;
  P p;
  idx_t pos;
  bool second;
  DESC_HD idx_t ext(int d) const {
    return d == D ? (second ? p.ext(D) - pos : pos) : p.ext(d);
  }
  DESC_HD Idx<rank> to_parent(const Idx<rank>& i) const {
    Idx<rank> j = i;
    if (second) j[D] = i[D] + pos;
    return j;
  }
};

// xor_swizzle at depth D: in a [rows][chunks] pair of dimensions, chunk c of
// row r is stored at chunk c ^ (((r / kDiv) % kMod) * kMul) of that row -- a
// permutation within every row (for a power-of-two row length above
// (kMod - 1) * kMul), so the view is a bijection onto the same storage.  Used
// to spread the LDS accesses of consecutive rows over banks.
template <class P, int D, idx_t kDiv, idx_t kMod, idx_t kMul = 1>
struct XorMap {
  static constexpr int rank = P::rank;
  static_assert(D + 1 < P::rank, "xor_swizzle needs two dimensions");
  P p;
  DESC_HD idx_t ext(int d) const { return p.ext(d); }
  // Positions are never negative, so the row term is taken in unsigned
  // arithmetic: with power-of-two kDiv and kMod it is then a shift and a
  // mask, and rows that differ by a multiple of kDiv * kMod visibly share it
  // (the compiler can then reuse one address for all of them).
  DESC_HD Idx<rank> to_parent(const Idx<rank>& i) const {
    Idx<rank> j = i;
    const uint64_t r = (uint64_t)i[D];
    j[D + 1] = i[D + 1] ^ (idx_t)(((r / (uint64_t)kDiv) % (uint64_t)kMod) * (uint64_t)kMul);
    return j;
  }
};

// select: dimension 0 is fixed to one index (the selecting resource's).
template <class P>
struct SelectMap {
  static constexpr int rank = P::rank - 1;
  static_assert(P::rank >= 1, "select needs an array");
  P p;
  idx_t sel;
  DESC_HD idx_t ext(int d) const { return p.ext(d + 1); }
  DESC_HD Idx<P::rank> to_parent(const Idx<rank>& i) const {
    Idx<P::rank> j;
    j[0] = sel;
    for (int d = 0; d < rank; ++d) j[d + 1] = i[d];
    return j;
  }
};

// Applying a chain of maps, last applied first, down to the dense offset.
template <int R>
DESC_HD idx_t resolve(const Dense<R>& m, const Idx<R>& i) { return m.offset(i); }
template <class M>
DESC_HD idx_t resolve(const M& m, const Idx<M::rank>& i) { return resolve(m.p, m.to_parent(i)); }

// ---------------------------------------------------------------------------
// Execution resources.
// ---------------------------------------------------------------------------
// A resource knows its own position among its siblings and how many siblings
// there are.  `N` is the sibling count when it is a compile-time constant
// (0 = known only at run time).  `Splittable` is false for the halves that
// `split` produces; those may not synchronise.
enum class Level { Grid, Block, Wave, Thread };

template <Level L, idx_t N = 0, bool Whole = true>
struct Res {
  static constexpr Level level = L;
  static constexpr idx_t static_count = N;
  static constexpr bool whole = Whole;
  idx_t id;       // position among siblings
  idx_t n;        // number of siblings
  DESC_HD idx_t index() const { return id; }
  DESC_HD idx_t count() const { return N ? N : n; }
};

template <idx_t NT> using Thread = Res<Level::Thread, NT>;     // a thread of a block of NT
template <idx_t NW> using Wave = Res<Level::Wave, NW>;         // a wave of a block of NW waves
using Block = Res<Level::Block, 0>;                            // a block of a 1-D grid
template <idx_t NT> using Lane = Res<Level::Thread, NT>;       // a lane of a wave of NT lanes

#if defined(__HIPCC__)
// Binding of `sched` to the hardware indices: the grid's blocks along x / y
// and the threads of a block (Sec. 5: sched becomes a scope plus an index).
__device__ __forceinline__ Block block_x() { return Block{(idx_t)blockIdx.x, (idx_t)gridDim.x}; }
__device__ __forceinline__ Block block_y() { return Block{(idx_t)blockIdx.y, (idx_t)gridDim.y}; }
template <idx_t NT>
__device__ __forceinline__ Thread<NT> thread_x() { return Thread<NT>{(idx_t)threadIdx.x, NT}; }
// Our extension below the block: waves of 64 lanes.
template <idx_t NT>
__device__ __forceinline__ Wave<NT / 64> wave_of_block() {
  return Wave<NT / 64>{(idx_t)(threadIdx.x / 64), NT / 64};
}
__device__ __forceinline__ Lane<64> lane_of_wave() { return Lane<64>{(idx_t)(threadIdx.x % 64), 64}; }
// The threads of a 1-D block of NY*NX threads seen as a [NY][NX] block:
// sched(Y,X) gives the row resource first and the column resource second.
template <idx_t NY, idx_t NX>
struct Thread2 {
  Res<Level::Thread, NY> y;
  Res<Level::Thread, NX> x;
};
template <idx_t NY, idx_t NX>
__device__ __forceinline__ Thread2<NY, NX> thread_yx() {
  const idx_t t = threadIdx.x;
  return Thread2<NY, NX>{{t / NX, NY}, {t % NX, NX}};
}

// A block-wide barrier.  Only a whole (unsplit) block may wait on it.
template <idx_t NT, bool Whole>
__device__ __forceinline__ void sync(const Res<Level::Thread, NT, Whole>&) {
  static_assert(Whole, "sync inside a split execution resource would diverge");
  __syncthreads();
}
#endif

// sched: run `body` for the given resource (the resource already names the
// calling sub-resource; this keeps the nesting visible in kernel bodies).
template <class R, class F>
DESC_HD void sched(const R& r, F&& body) { body(r); }

// split a resource at `pos` into two independent groups; the halves are not
// whole and cannot `sync`.
template <class R, class F1, class F2>
DESC_HD void split(const R& r, idx_t pos, F1&& fst, F2&& snd) {
  using Half = Res<R::level, 0, false>;
  if (r.index() < pos) fst(Half{r.index(), pos});
  else snd(Half{r.index() - pos, r.count() - pos});
}

// ---------------------------------------------------------------------------
// Views.
// ---------------------------------------------------------------------------
template <class T, class M>
struct View {
  static constexpr int rank = M::rank;
  T* base;
  M m;

  DESC_HD idx_t extent(int d = 0) const { return m.ext(d); }

  // The one place an index becomes an address.
  DESC_HD T& ref(const Idx<rank>& i) const { return base[resolve(m, i)]; }

  // Position in the underlying array that an index resolves to (used to
  // guard the ragged tail of a view whose nominal extent is rounded up).
  DESC_HD idx_t pos(idx_t i) const {
    static_assert(rank == 1, "pos of a rank-1 view");
    Idx<1> j;
    j[0] = i;
    return resolve(m, j);
  }

  // Element access on a rank-1 view.
  DESC_HD T& operator[](idx_t i) const {
    static_assert(rank == 1, "index a rank-1 view; select outer dimensions first");
    Idx<1> j;
    j[0] = i;
    return ref(j);
  }
  // The single element of a rank-0 view (every dimension selected).
  DESC_HD T& get() const {
    static_assert(rank == 0, "get() needs every dimension selected");
    Idx<0> j;
    return ref(j);
  }
  template <class... I>
  DESC_HD T& at(I... is) const {
    static_assert(sizeof...(I) == rank, "one index per dimension");
    Idx<rank> j{{(idx_t)is...}};
    return ref(j);
  }

  template <idx_t K, int D = 0>
  DESC_HD View<T, GroupMap<M, K, D>> group() const { return {base, {m}}; }
  template <int D = 0>
  DESC_HD View<T, TransposeMap<M, D>> transpose() const { return {base, {m}}; }
  template <int D = 0>
  DESC_HD View<T, ReverseMap<M, D>> reverse() const { return {base, {m}}; }
  template <idx_t kDiv, idx_t kMod, int D = 0>
  DESC_HD View<T, XorMap<M, D, kDiv, kMod>> xor_swizzle() const { return {base, {m}}; }
  template <idx_t kDiv, idx_t kMod, idx_t kMul, int D = 0>
  DESC_HD View<T, XorMap<M, D, kDiv, kMod, kMul>> xor_swizzle_by() const { return {base, {m}}; }
  template <int D = 0>
  DESC_HD View<T, SplitMap<M, D>> fst(idx_t pos) const { return {base, {m, pos, false}}; }
  template <int D = 0>
  DESC_HD View<T, SplitMap<M, D>> snd(idx_t pos) const { return {base, {m, pos, true}}; }

  // Plain index into the outermost dimension (a sequential loop variable).
  DESC_HD View<T, SelectMap<M>> idx(idx_t i) const { return {base, {m, i}}; }

  // p[[e]]: each sibling of `r` takes the element of dimension 0 at its own
  // position.  The dimension must have exactly as many elements as there are
  // siblings.
  template <Level L, idx_t N, bool W>
  DESC_HD View<T, SelectMap<M>> select(const Res<L, N, W>& r) const {
#if !defined(__HIP_DEVICE_COMPILE__)
    assert(m.ext(0) == r.count() && "select: extent must equal the number of sub-resources");
#endif
    return {base, {m, r.index()}};
  }
};

// Composite views built from the basic ones (Sec. 3.2).
//
// group_by_row<R, N> over a [R][C] tile read by a [R/N][C] block of threads:
// thread (y, x) owns the N elements at rows y, y + R/N, y + 2R/N, ... of
// column x.  Written as group::<R/N> followed by moving the group index
// innermost (transpose, then map(transpose)).
template <idx_t R, idx_t N, class T, class M>
DESC_HD auto group_by_row(const View<T, M>& v) {
  static_assert(R % N == 0, "rows must divide into N groups");
  return v.template group<R / N>().template transpose<0>().template transpose<1>();
}

// group_by_tile<H, W> over a [R][C] matrix: [R/H][C/W][H][W] tiles.
template <idx_t H, idx_t W, class T, class M>
DESC_HD auto group_by_tile(const View<T, M>& v) {
  return v.template group<H, 0>()          // [R/H][H][C]
      .template group<W, 2>()              // [R/H][H][C/W][W]
      .template transpose<1>();            // [R/H][C/W][H][W]
}

// A window of a row-major matrix read through a hardware buffer range.  The
// window starts at one element of the matrix (the range's base) and covers
// `rows` x `cols` valid elements at row stride `ld` (elements of kBytes
// bytes); the range is bytes() long, ending at the last valid element.  The
// index map gives the byte offset of (r, c) as row(r) + col(c): inside the
// range for a valid element; at least kOutside (past any range) for a column
// c >= cols; and for a row r >= rows past bytes() by itself (when
// cols <= ld), so a buffer load of an invalid element returns zero without a
// row test.  The two parts let a kernel compute a lane's column part once
// and add the row parts of its loads.  Offsets are 32-bit: the caller keeps
// every row(r) it uses below 2^30 (then kOutside + row(r) < 2^32 too).
constexpr uint32_t kOutside = 0x80000000u;   // an offset past any range a window uses
template <int kBytes>
struct BufferWindow {
  uint32_t ld;                // row stride, elements
  int32_t rows, cols;         // valid rows and columns (<= 0: an empty window)
  DESC_HD uint32_t bytes() const {
    return rows > 0 && cols > 0 ? ((uint32_t)(rows - 1) * ld + (uint32_t)cols) * kBytes : 0u;
  }
  DESC_HD uint32_t row(int32_t r) const { return (uint32_t)r * ld * kBytes; }
  DESC_HD uint32_t col(int32_t c) const { return c < cols ? (uint32_t)c * kBytes : kOutside; }
  DESC_HD uint32_t offset(int32_t r, int32_t c) const { return row(r) + col(c); }
  // The column part of a column the caller knows to be valid (c < cols),
  // without the test.
  DESC_HD uint32_t col_valid(int32_t c) const { return (uint32_t)c * kBytes; }
};

// An array of n elements of type T at p (rank 1) or a rows x cols matrix.
template <class T>
DESC_HD View<T, Dense<1>> array(T* p, idx_t n) { return {p, {{n}}}; }
template <class T>
DESC_HD View<T, Dense<2>> matrix(T* p, idx_t rows, idx_t cols) { return {p, {{rows, cols}}}; }
// A batch of `count` rows x cols matrices stored one after the other.
template <class T>
DESC_HD View<T, Dense<3>> matrices(T* p, idx_t count, idx_t rows, idx_t cols) {
  return {p, {{count, rows, cols}}};
}

}  // namespace desc
