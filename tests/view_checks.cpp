// Host-side enumeration of the index maps of the view layer (Sec. 3.2 of the
// paper) and of the maps the kernels use: every (resource, item) pair is
// resolved to an index, and the resulting access sets are checked for
// disjointness (no two sub-resources touch one element), coverage, and the
// closed forms the paper's examples fix.  Prints one line per check;
// exits non-zero if any fails.
//
// Built by tests/test_views.py with: g++ -std=c++17 -O1 -I <csrc> view_checks.cpp
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <string>
#include <type_traits>
#include <vector>

#include "access_check.hpp"
#include "layouts.hpp"

using namespace desc;

// 16-byte group of four words (the host stand-in of the kernels' int32x4)
struct u32x4 {
  unsigned v[4];
};

static int g_fail = 0;
static void check(bool ok, const char* name, const std::string& detail = "") {
  std::printf("%s %s%s%s\n", ok ? "OK" : "FAIL", name, detail.empty() ? "" : ": ",
              detail.c_str());
  if (!ok) g_fail = 1;
}

// Records which sub-resource touches which index and reports collisions.
struct Access {
  std::vector<long> owner;
  long collisions = 0, touched = 0;
  explicit Access(long n) : owner(n, -1) {}
  void add(long idx, long who) {
    if (idx < 0 || idx >= (long)owner.size()) { ++collisions; return; }
    if (owner[idx] >= 0 && owner[idx] != who) ++collisions;
    if (owner[idx] < 0) ++touched;
    owner[idx] = who;
  }
  bool bijection() const { return collisions == 0 && touched == (long)owner.size(); }
};

template <Level L>
static Res<L, 0> R(long id, long n) { return Res<L, 0>{id, n}; }

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "select_mismatch") == 0) {
    // a select whose extent differs from the number of sub-resources
    std::vector<int> a(100);
    auto v = array(a.data(), 100).group<10>();
    auto t = R<Level::Thread>(0, 7);
    (void)v.select(t);          // asserts
    return 0;
  }

  // --- Listing 1 of the paper: the racy index and its correction --------------
  {
    std::set<long> all;
    bool per_j = true;
    for (int j = 0; j < 32; j += 8) {
      std::set<long> s;
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 32; ++x) {
          s.insert(y + j * 32 + x);     // threadIdx.y + j*32 + threadIdx.x, as printed
          all.insert(y + j * 32 + x);
        }
      per_j &= s.size() == 39;
    }
    check(per_j && all.size() == 156, "listing1_racy_index_collides",
          std::to_string(all.size()) + " distinct slots for 1024 writes");
    Access acc(1024);
    for (int j = 0; j < 32; j += 8)
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 32; ++x) acc.add((y + j) * 32 + x, (y * 32 + x) * 4 + j / 8);
    check(acc.bijection(), "listing1_corrected_index_is_bijection");
  }

  // --- group_by_row<32,4> equals the corrected Listing 1 index ---------------
  {
    std::vector<int> tmp(32 * 32);
    auto t = matrix(tmp.data(), 32, 32);
    bool same = true;
    Access acc(1024);
    for (int y = 0; y < 8; ++y)
      for (int x = 0; x < 32; ++x)
        for (int i = 0; i < 4; ++i) {
          auto v = group_by_row<32, 4>(t).select(R<Level::Thread>(y, 8)).select(
              R<Level::Thread>(x, 32));
          const long idx = &v[i] - tmp.data();
          same &= idx == (y + 8 * i) * 32 + x;
          acc.add(idx, y * 32 + x);
        }
    check(same && acc.bijection(), "group_by_row_32_4_is_listing1_corrected");
  }

  // --- array.group::<8>.transpose selected by 8 threads (Sec. 3.2 figure) ------
  {
    std::vector<int> a(32);
    bool ok = true;
    for (int t = 0; t < 8; ++t) {
      auto v = array(a.data(), 32).group<8>().transpose().select(R<Level::Thread>(t, 8));
      for (int i = 0; i < 4; ++i) ok &= (&v[i] - a.data()) == t + 8 * i;
    }
    check(ok, "group8_transpose_thread_t_gets_t_t8_t16_t24");
  }

  // --- Listing 2: the transposition through views, end to end on 2048^2 --------
  // Phase 1 copies the input tile into tmp, phase 2 copies tmp out; with the
  // element transpose on the tmp read the output is the transposed matrix,
  // with the printed listing (tmp read through the same view it was written
  // through) it is not.
  for (int fixed = 1; fixed >= 0; --fixed) {
    const int n = 2048;
    std::vector<int> in(n * n), out(n * n, -1);
    for (int i = 0; i < n * n; ++i) in[i] = i;
    std::vector<int> tmp(32 * 32);
    auto inp = matrix(in.data(), n, n);
    auto outp = matrix(out.data(), n, n);
    auto tmpv = matrix(tmp.data(), 32, 32);
    Access writes(n * n);
    for (int by = 0; by < 64; ++by)
      for (int bx = 0; bx < 64; ++bx) {
        auto bY = R<Level::Block>(by, 64), bX = R<Level::Block>(bx, 64);
        for (int ty = 0; ty < 8; ++ty)
          for (int tx = 0; tx < 32; ++tx) {
            auto tY = R<Level::Thread>(ty, 8), tX = R<Level::Thread>(tx, 32);
            auto src = group_by_row<32, 4>(group_by_tile<32, 32>(inp).transpose().select(bY).select(bX))
                           .select(tY).select(tX);
            auto dst = group_by_row<32, 4>(tmpv).select(tY).select(tX);
            for (int i = 0; i < 4; ++i) dst[i] = src[i];
          }
        for (int ty = 0; ty < 8; ++ty)
          for (int tx = 0; tx < 32; ++tx) {
            auto tY = R<Level::Thread>(ty, 8), tX = R<Level::Thread>(tx, 32);
            auto dst = group_by_row<32, 4>(group_by_tile<32, 32>(outp).select(bY).select(bX))
                           .select(tY).select(tX);
            for (int i = 0; i < 4; ++i) {
              if (fixed) {
                auto src = group_by_row<32, 4>(tmpv.transpose()).select(tY).select(tX);
                dst[i] = src[i];
              } else {
                auto src = group_by_row<32, 4>(tmpv).select(tY).select(tX);
                dst[i] = src[i];
              }
              writes.add(&dst[i] - out.data(), (((by * 64 + bx) * 8 + ty) * 32 + tx));
            }
          }
      }
    bool is_t = true;
    for (int r = 0; r < n && is_t; ++r)
      for (int c = 0; c < n; ++c)
        if (out[c * n + r] != in[r * n + c]) { is_t = false; break; }
    if (fixed)
      check(is_t && writes.bijection(), "listing2_with_tmp_transpose_is_transposition");
    else
      check(!is_t && writes.bijection(), "listing2_as_printed_moves_tiles_only");
  }

  // --- Narrowing (Sec. 3.3): grid X<32> of X<32> over [f32; 1024] --------------
  {
    std::vector<float> arr(1024);
    Access good(1024), bad(1024);
    for (int b = 0; b < 32; ++b)
      for (int t = 0; t < 32; ++t) {
        auto v = array(arr.data(), 1024).group<32>().select(R<Level::Block>(b, 32)).select(
            R<Level::Thread>(t, 32));
        good.add(&v.get() - arr.data(), b * 32 + t);
        // selecting by thread only: every block's thread t reaches group t
        auto w = array(arr.data(), 1024).group<32>().select(R<Level::Thread>(t, 32));
        for (int i = 0; i < 32; ++i) bad.add(&w[i] - arr.data(), b * 32 + t);
      }
    check(good.bijection(), "narrowing_group32_block_thread_is_bijection");
    check(bad.collisions > 0, "narrowing_without_block_selection_conflicts",
          std::to_string(bad.collisions) + " conflicting accesses");
  }

  // --- rev_per_block: write arr[[thread]], read arr.reverse[[thread]] ---------
  {
    const int n = 64;
    std::vector<int> arr(n);
    long conflicts = 0;
    for (int t = 0; t < n; ++t) {
      auto w = array(arr.data(), n).select(R<Level::Thread>(t, n));
      auto r = array(arr.data(), n).reverse().select(R<Level::Thread>(t, n));
      const long wi = &w.get() - arr.data(), ri = &r.get() - arr.data();
      if (wi != ri) ++conflicts;   // another thread writes what this one reads
    }
    check(conflicts == n, "reverse_per_block_read_write_conflict");
  }

  // --- execution resources: split(Y) at 1 of 2 blocks (Sec. 3.1 example) ------
  {
    int fst = 0, snd = 0;
    bool ok = true;
    for (int y = 0; y < 2; ++y)
      split(R<Level::Block>(y, 2), 1,
            [&](auto h) { ++fst; ok &= h.count() == 1 && h.index() == 0 && !decltype(h)::whole; },
            [&](auto h) { ++snd; ok &= h.count() == 1 && h.index() == 0; });
    check(ok && fst == 1 && snd == 1, "split_Y_at_1_gives_two_single_block_groups");
  }

  // --- the kernels' own maps ----------------------------------------------------
  {
    // scan / segmented: wave-striped tiles of int32x4 groups and of scalars
    const int W = 4, Rr = 8, tiles = 3, per = W * Rr * 64;
    std::vector<int> groups(tiles * per);
    Access g(tiles * per), e(tiles * per * 4);
    bool contiguous = true;
    for (int t = 0; t < tiles; ++t)
      for (int w = 0; w < W; ++w)
        for (int l = 0; l < 64; ++l) {
          auto v = layout::wave_striped<W, Rr>(array(groups.data(), tiles * per), t,
                                               R<Level::Wave>(w, W), R<Level::Thread>(l, 64));
          std::vector<int> sc(tiles * per * 4);
          auto s = layout::wave_striped<W, Rr>(array(sc.data(), tiles * per * 4).group<4>(), t,
                                               R<Level::Wave>(w, W), R<Level::Thread>(l, 64));
          for (int r = 0; r < Rr; ++r) {
            const long idx = &v[r] - groups.data();
            g.add(idx, (t * W + w) * 64 + l);
            contiguous &= idx == (long)t * per + w * Rr * 64 + r * 64 + l;
            for (int k = 0; k < 4; ++k) e.add(s.idx(r).pos(k), (t * W + w) * 64 + l);
          }
        }
    check(g.bijection() && contiguous, "scan_wave_striped_groups_bijection_and_coalesced");
    check(e.bijection(), "scan_wave_striped_elements_bijection");

    // reduce: block-striped tiles
    const int B = 256, U = 4, T2 = 5;
    std::vector<int> v(T2 * U * B);
    Access rb(T2 * U * B);
    for (int t = 0; t < T2; ++t)
      for (int x = 0; x < B; ++x) {
        auto m = layout::block_striped<B, U>(array(v.data(), T2 * U * B), t,
                                             R<Level::Thread>(x, B));
        for (int u = 0; u < U; ++u) rb.add(&m[u] - v.data(), t * B + x);
      }
    check(rb.bijection(), "reduce_block_striped_bijection");
  }

  // low-precision GEMM LDS stage: [rows][chunks] of 16 bytes, XOR-swizzled;
  // a bijection per row, and both access patterns of 16 lanes (the staging
  // writes along a row, the fragment reads down 16 rows) hit 16 distinct
  // 16-byte bank groups of a 256-byte bank period.
  auto swizzle_case = [&](auto Bc) {
    constexpr int BKB = decltype(Bc)::value, CPR = BKB / 16, RPB = 256 / BKB;
    const int rows = 64;
    std::vector<u32x4> lds(rows * CPR);
    auto v = matrix(lds.data(), rows, CPR).xor_swizzle<RPB, CPR>();
    Access all(rows * CPR);
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < CPR; ++c) all.add(&v.at(r, c) - lds.data(), r * CPR + c);
    bool reads_ok = true, writes_ok = true;
    for (int r0 = 0; r0 < rows; r0 += 16)
      for (int c = 0; c < CPR; ++c) {
        std::set<long> g;
        for (int r = r0; r < r0 + 16; ++r) g.insert((&v.at(r, c) - lds.data()) % 16);
        reads_ok &= g.size() == 16;
      }
    for (int q0 = 0; q0 < rows * CPR; q0 += 16) {
      std::set<long> g;
      for (int q = q0; q < q0 + 16; ++q) g.insert((&v.at(q / CPR, q % CPR) - lds.data()) % 16);
      writes_ok &= g.size() == 16;
    }
    // the pipelined FP8 reads step from a lane's first fragment to the next
    // by whole 32-row blocks: the swizzle must repeat every 32 rows
    bool period_ok = true;
    for (int r = 0; r + 32 < rows; ++r)
      for (int c = 0; c < CPR; ++c) period_ok &= &v.at(r + 32, c) == &v.at(r, c) + 32 * CPR;
    const std::string name = "gemm_lds_xor_swizzle_bkb" + std::to_string(BKB);
    check(all.bijection() && reads_ok && writes_ok && period_ok, name.c_str());
  };
  swizzle_case(std::integral_constant<int, 32>{});
  swizzle_case(std::integral_constant<int, 64>{});
  swizzle_case(std::integral_constant<int, 128>{});

  // transposition kernel: tiles T = 32, 64, 128 on a 2T x 3T matrix
  auto transpose_case = [&](auto Tc) {
    constexpr int T = decltype(Tc)::value;
    constexpr int TX = T / 4, TY = 256 / TX, IT = T / TY;
    const int rows = 2 * T, cols = 3 * T;
    std::vector<unsigned> in(rows * cols), out(rows * cols, 0xffffffffu), lds(T * (T + 1));
    for (int i = 0; i < rows * cols; ++i) in[i] = i;
    Access rd(rows * cols), wr(rows * cols), lw(T * T);
    for (int by = 0; by < rows / T; ++by)
      for (int bx = 0; bx < cols / T; ++bx) {
        auto bY = R<Level::Block>(by, rows / T), bX = R<Level::Block>(bx, cols / T);
        auto tile = matrix(lds.data(), T, T + 1).fst<1>(T);
        auto inm = matrix((u32x4*)in.data(), rows, cols / 4);
        auto outm = matrix((u32x4*)out.data(), cols, rows / 4);
        Access lw1(T * (T + 1));
        for (int y = 0; y < TY; ++y)
          for (int x = 0; x < TX; ++x) {
            auto tY = R<Level::Thread>(y, TY), tX = R<Level::Thread>(x, TX);
            auto a = layout::tile_rows<T, IT>(inm, bY, bX, tY, tX);
            auto l = layout::lds_rows<T, IT>(tile, tY, tX);
            for (int i = 0; i < IT; ++i)
              for (int k = 0; k < 4; ++k) {
                const unsigned* src = (const unsigned*)&a[i] + k;
                rd.add(src - in.data(), (by * 8 + bx) * 256 + y * TX + x);
                l.idx(i)[k] = *src;
                lw1.add(&l.idx(i)[k] - lds.data(), y * TX + x);
              }
          }
        lw.collisions += lw1.collisions;
        for (int y = 0; y < TY; ++y)
          for (int x = 0; x < TX; ++x) {
            auto tY = R<Level::Thread>(y, TY), tX = R<Level::Thread>(x, TX);
            auto b = layout::tile_rows<T, IT>(outm, bX, bY, tY, tX);
            auto l = layout::lds_cols<T, IT>(tile, tY, tX);
            for (int i = 0; i < IT; ++i)
              for (int k = 0; k < 4; ++k) {
                unsigned* dst = (unsigned*)&b[i] + k;
                *dst = l.idx(i)[k];
                wr.add(dst - out.data(), (by * 8 + bx) * 256 + y * TX + x);
              }
          }
      }
    bool is_t = true;
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c) is_t &= out[c * rows + r] == in[r * cols + c];
    const std::string name = "transpose_kernel_maps_T" + std::to_string(T);
    check(is_t && rd.bijection() && wr.bijection() && lw.collisions == 0, name.c_str());
  };
  transpose_case(std::integral_constant<int, 32>{});
  transpose_case(std::integral_constant<int, 64>{});
  transpose_case(std::integral_constant<int, 128>{});

  // the LDS swizzles of the 2- and 8-byte transposes: a bijection on the
  // tile, and the column reads of the write-out spread over the banks
  // (doubles: the 32 rows 2x + k of a half-wave land on 32 different 8-byte
  // bank pairs; 2-byte elements: the 16 rows 8x + k of a wave on 16
  // different dwords mod 64 banks, element pairs sharing a dword)
  {
    const int T = 64;
    std::vector<unsigned long long> lds(T * T);
    auto v = matrix(lds.data(), T, T).xor_swizzle_by<2, 32, 1>();
    Access all(T * T);
    for (int r = 0; r < T; ++r)
      for (int c = 0; c < T; ++c) all.add(&v.at(r, c) - lds.data(), r * T + c);
    bool spread = true;
    for (int k = 0; k < 2; ++k)
      for (int c = 0; c < T; ++c) {
        std::set<long> banks;
        for (int x = 0; x < 32; ++x) banks.insert(((&v.at(2 * x + k, c) - lds.data()) * 2) % 64);
        spread &= banks.size() == 32;
      }
    check(all.bijection() && spread, "transpose_f64_lds_swizzle");
  }
  {
    const int T = 128;
    std::vector<unsigned short> lds(T * T);
    auto v = matrix(lds.data(), T, T).xor_swizzle_by<8, 16, 4>();
    Access all(T * T);
    for (int r = 0; r < T; ++r)
      for (int c = 0; c < T; ++c) all.add(&v.at(r, c) - lds.data(), r * T + c);
    bool spread = true, pairs = true;
    for (int k = 0; k < 8; ++k)
      for (int c = 0; c < T; ++c) {
        std::set<long> dwords;
        for (int x = 0; x < 16; ++x) dwords.insert(((&v.at(8 * x + k, c) - lds.data()) / 2) % 64);
        spread &= dwords.size() == 16;
      }
    for (int r = 0; r < T; ++r)
      for (int c = 0; c < T; c += 2)
        pairs &= (&v.at(r, c) - lds.data()) / 2 == (&v.at(r, c + 1) - lds.data()) / 2;
    check(all.bijection() && spread && pairs, "transpose_u16_lds_swizzle");
  }

  // --- access checking over the kernels' own maps (access_check.hpp) ----------
  // Listing 1 as printed: the 256 threads of a 32 x 8 block write tmp through
  // the racy index in one interval; the corrected index writes disjointly.
  {
    std::vector<float> tmp(1024);
    access_check::Checker racy, fixed;
    for (int j = 0; j < 32; j += 8)
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 32; ++x) {
          racy.write(0, y * 32 + x, &tmp[y + j * 32 + x]);
          fixed.write(0, y * 32 + x, &tmp[(y + j) * 32 + x]);
        }
    check(!racy.conflicts().empty() && fixed.conflicts().empty(),
          "access_check_listing1_racy_conflicts_corrected_clean",
          std::to_string(racy.conflicts().size()) + " conflicts");
  }
  // rev_per_block (Sec. 2): each thread writes arr[[thread]] and reads
  // arr.rev[[thread]], which another thread writes: a conflict unless a
  // barrier separates the write from the read.
  {
    const int n = 64;
    std::vector<int> arr(n);
    access_check::Checker no_sync, with_sync;
    for (int t = 0; t < n; ++t)
      for (auto* c : {&no_sync, &with_sync})
        c->write(0, t, &array(arr.data(), n).select(R<Level::Thread>(t, n)).get());
    with_sync.sync(0);
    for (int t = 0; t < n; ++t)
      for (auto* c : {&no_sync, &with_sync})
        c->read(0, t, &array(arr.data(), n).reverse().select(R<Level::Thread>(t, n)).get());
    check(no_sync.conflicts().size() == (size_t)n && with_sync.conflicts().empty(),
          "access_check_rev_per_block_needs_barrier");
  }
  // The transposition kernel: global reads and LDS writes, a barrier, LDS
  // reads and global writes; each block has its own LDS tile.  Clean as
  // written; without the barrier the LDS reads race the writes of other
  // threads of the block.
  auto transpose_access = [&](auto Tc, bool barrier) {
    constexpr int T = decltype(Tc)::value;
    constexpr int TX = T / 4, TY = 256 / TX, IT = T / TY;
    const int rows = 2 * T, cols = 2 * T, nb = 4;
    std::vector<unsigned> in(rows * cols), out(rows * cols);
    std::vector<std::vector<unsigned>> lds(nb, std::vector<unsigned>(T * (T + 1)));
    access_check::Checker c;
    for (int by = 0; by < 2; ++by)
      for (int bx = 0; bx < 2; ++bx) {
        const long blk = by * 2 + bx;
        auto bY = R<Level::Block>(by, 2), bX = R<Level::Block>(bx, 2);
        auto tile = matrix(lds[blk].data(), T, T + 1).template fst<1>(T);
        auto inm = matrix((u32x4*)in.data(), rows, cols / 4);
        auto outm = matrix((u32x4*)out.data(), cols, rows / 4);
        for (int y = 0; y < TY; ++y)
          for (int x = 0; x < TX; ++x) {
            auto tY = R<Level::Thread>(y, TY), tX = R<Level::Thread>(x, TX);
            auto a = layout::tile_rows<T, IT>(inm, bY, bX, tY, tX);
            auto l = layout::lds_rows<T, IT>(tile, tY, tX);
            const long who = blk * 256 + y * TX + x;
            for (int i = 0; i < IT; ++i) {
              c.read(blk, who, &a[i]);
              for (int k = 0; k < 4; ++k) c.write(blk, who, &l.idx(i)[k]);
            }
          }
        if (barrier) c.sync(blk);
        for (int y = 0; y < TY; ++y)
          for (int x = 0; x < TX; ++x) {
            auto tY = R<Level::Thread>(y, TY), tX = R<Level::Thread>(x, TX);
            auto b = layout::tile_rows<T, IT>(outm, bX, bY, tY, tX);
            auto l = layout::lds_cols<T, IT>(tile, tY, tX);
            const long who = blk * 256 + y * TX + x;
            for (int i = 0; i < IT; ++i) {
              for (int k = 0; k < 4; ++k) c.read(blk, who, &l.idx(i)[k]);
              c.write(blk, who, &b[i]);
            }
          }
      }
    return c.conflicts().size();
  };
  {
    const size_t c32 = transpose_access(std::integral_constant<int, 32>{}, true);
    const size_t c64 = transpose_access(std::integral_constant<int, 64>{}, true);
    const size_t c128 = transpose_access(std::integral_constant<int, 128>{}, true);
    const size_t r64 = transpose_access(std::integral_constant<int, 64>{}, false);
    check(c32 == 0 && c64 == 0 && c128 == 0, "access_check_transpose_kernel_clean");
    check(r64 > 0, "access_check_transpose_without_barrier_races",
          std::to_string(r64) + " conflicts");
  }
  // The block-wide reduction's tree (variants.hip): at each step the block is
  // split at k, the first k threads read p[i] and p[i + k] and write p[i], and
  // the whole block synchronises.  Clean with the barriers, racy without.
  auto tree_access = [&](bool barriers) {
    std::vector<long> part(256);
    access_check::Checker c;
    auto p = array(part.data(), 256);
    for (int t = 0; t < 256; ++t) c.write(0, t, &p[t]);
    c.sync(0);
    for (int k = 128; k >= 1; k /= 2) {
      for (int t = 0; t < 256; ++t)
        split(R<Level::Thread>(t, 256), k,
              [&](auto first) {
                c.read(0, t, &p.fst(k).select(first).get());
                c.read(0, t, &p.snd(k).fst(k).select(first).get());
                c.write(0, t, &p.fst(k).select(first).get());
              },
              [](auto) {});
      if (barriers) c.sync(0);
    }
    return c.conflicts().size();
  };
  check(tree_access(true) == 0, "access_check_reduce_tree_clean");
  check(tree_access(false) > 0, "access_check_reduce_tree_without_barriers_races");
  // The scan's tile stores: every (tile, wave, lane) writes its own 4-element
  // groups, across all blocks, with no barrier needed.
  {
    const int W = 4, Rr = 4, tiles = 3, per = W * Rr * 64;
    std::vector<int> out(tiles * per * 4);
    access_check::Checker c;
    for (int t = 0; t < tiles; ++t)
      for (int w = 0; w < W; ++w)
        for (int l = 0; l < 64; ++l) {
          auto s = layout::wave_striped<W, Rr>(array(out.data(), tiles * per * 4).group<4>(), t,
                                               R<Level::Wave>(w, W), R<Level::Thread>(l, 64));
          for (int r = 0; r < Rr; ++r)
            for (int k = 0; k < 4; ++k) c.write(t, (t * W + w) * 64 + l, &s.idx(r)[k]);
        }
    check(c.conflicts().empty() && c.accesses() == out.size(), "access_check_scan_stores_clean");
  }

  // --- min/max and float-sum chunk layout: [chunks][4][256] groups of four --------
  // Lane j of a block takes groups 256 u + j of a chunk (elements 1024 u + 4 j ..),
  // u = 0..3; over the grid-strided chunks of G blocks every group is read once.
  {
    const int G = 3, chunks = 7, lanes = 256;
    std::vector<int> a(chunks * 1024);    // groups
    Access acc(chunks * 1024);
    bool order = true;
    for (int b = 0; b < G; ++b)
      for (int c = b; c < chunks; c += G)
        for (int j = 0; j < lanes; ++j) {
          auto v = array(a.data(), chunks * 1024).group<256>().group<4>().idx(c).transpose().select(
              R<Level::Thread>(j, lanes));
          for (int u = 0; u < 4; ++u) {
            const long g = &v[u] - a.data();
            order &= g == c * 1024L + 256 * u + j;
            acc.add(g, b * lanes + j);
          }
        }
    check(order && acc.bijection(), "reduce_ops_chunk_groups_bijection");
  }

  // --- transpose tiles in diagonal order: block (x, y) -> tile ((x + y) mod X, y) ---
  {
    bool ok = true;
    for (const auto& gxy : std::vector<std::pair<int, int>>{{64, 128}, {64, 64}, {5, 3}, {1, 9}}) {
      Access acc(gxy.first * gxy.second);
      for (int y = 0; y < gxy.second; ++y)
        for (int x = 0; x < gxy.first; ++x) acc.add(((x + y) % gxy.first) + gxy.first * y, x + gxy.first * y);
      ok &= acc.bijection();
    }
    check(ok, "transpose_diagonal_tile_order_bijection");
  }

  // --- fused split staging: the buffer windows of A and B ---
  // For every shape edge a wave can meet, each of the wave's positions is
  // staged exactly once, a load returns data (offset inside the range) for
  // exactly the valid positions, and then from the element's own address.
  {
    bool ok = true;
    long checked = 0;
    const int CPR = 4, KS = 8 * CPR;
    for (int rows = 0; rows <= 17; ++rows)             // valid rows of A's window (16 staged)
      for (int cols : {1, 3, 4, 5, 8, 17, 31, 32})     // valid k of the stage
        for (long ld : {32L, 33L, 100L, 1L << 24}) {
          if (cols > ld) continue;
          const BufferWindow<4> w{(uint32_t)ld, rows > 16 ? 16 : rows, cols};
          Access acc(16 * KS);
          for (int lane = 0; lane < 64; ++lane)
            for (int j = 0; j < 8; ++j) {
              const int r = layout::split_a_row<CPR>(lane), c = layout::split_a_k<CPR>(lane) + j;
              acc.add(r * KS + c, lane);
              const uint32_t off = w.row(r) + w.col(c);
              const bool valid = r < w.rows && c < w.cols;
              ok &= (off < w.bytes()) == valid;
              if (valid) ok &= off == (uint32_t)((r * ld + c) * 4);
              ++checked;
            }
          ok &= acc.bijection();
        }
    for (int rows = 0; rows <= 8; ++rows)              // valid k of B's octet
      for (int cols = -3; cols <= 64; cols += 1)       // valid columns of the wave (<= 0: none)
        for (long ld : {64L, 65L, 1000L, 1L << 24}) {
          const BufferWindow<4> w{(uint32_t)ld, rows, cols};
          Access acc(8 * 64);
          for (int lane = 0; lane < 64; ++lane)
            for (int j = 0; j < 8; ++j) {
              const int c = layout::split_b_col(lane);
              acc.add(j * 64 + c, lane);
              const uint32_t off = w.row(j) + w.col(c);
              const bool valid = j < w.rows && c < w.cols;
              ok &= (off < w.bytes()) == valid;
              if (valid) ok &= off == (uint32_t)((j * ld + c) * 4);
              ++checked;
            }
          ok &= acc.bijection();
        }
    check(ok, "split_staging_buffer_windows", std::to_string(checked) + " positions");
  }

  // --- FP32 GEMM, row-major tile: the LDS double buffer under the two-stages-ahead
  // schedule (gemm_f32.hpp tile_rowmajor), 256 x 128 x 16 with 2 x 2 waves.  Every
  // stage's fragment reads find words written by an earlier phase, and no read meets
  // a write of the same buffer between the same two barriers; dropping any one of
  // the loop's barriers makes the next phase's stores race its reads.
  {
    constexpr int BM = 256, BN = 128, BK = 16, WM = 2, WN = 2, T = 64 * WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / 32, FN = WTN / 32;
    constexpr int PA = BK + 4, PB = BN + 4, AV = BM * BK / 4 / T, BV = BK * BN / 4 / T;
    auto replay = [&](int nk, int drop_barrier, long* uninit) {
      std::vector<float> lds(2 * BM * PA + 2 * BK * PB);
      std::vector<char> written(lds.size(), 0);
      auto a_lds = matrices(lds.data(), 2, BM, PA);
      auto b_lds = matrices(lds.data() + 2 * BM * PA, 2, BK, PB);
      access_check::Checker c;
      int barrier_no = 0;
      auto sync_ = [&]() { if (barrier_no++ != drop_barrier) c.sync(0); };
      auto store = [&](int buf) {
        for (int t = 0; t < T; ++t) {
          for (int i = 0; i < AV; ++i) {
            const int q = t + T * i;
            for (int e = 0; e < 4; ++e) {
              float* w = &a_lds.idx(buf).at(layout::gemm_store_row<BK>(q), layout::gemm_store_word<BK>(q) + e);
              c.write(0, t, w); written[w - lds.data()] = 1;
            }
          }
          for (int i = 0; i < BV; ++i) {
            const int q = t + T * i;
            for (int e = 0; e < 4; ++e) {
              float* w = &b_lds.idx(buf).at(layout::gemm_store_row<BN>(q), layout::gemm_store_word<BN>(q) + e);
              c.write(0, t, w); written[w - lds.data()] = 1;
            }
          }
        }
      };
      auto compute = [&](int buf) {
        for (int t = 0; t < T; ++t) {
          const int w = t / 64, l = t % 64, half = l / 32, c32 = l % 32, wm = w / WN, wn = w % WN;
          for (int k4 = 0; k4 < BK / 2; k4 += 4) {
            for (int i = 0; i < FM; ++i)
              for (int e = 0; e < 4; ++e) {
                float* r = &a_lds.idx(buf).at(layout::gemm_a_frag_row<WTM>(wm, i, c32),
                                              layout::gemm_frag_k<BK>(half, k4) + e);
                c.read(0, t, r); *uninit += !written[r - lds.data()];
              }
            for (int kk = 0; kk < 4; ++kk)
              for (int j = 0; j < FN; ++j) {
                float* r = &b_lds.idx(buf).at(layout::gemm_frag_k<BK>(half, k4) + kk,
                                              layout::gemm_b_frag_word<WTN>(wn, j, c32));
                c.read(0, t, r); *uninit += !written[r - lds.data()];
              }
          }
        }
      };
      // the schedule of tile_rowmajor with kDepth = 2
      store(0);
      sync_();
      int kt = 0;
      for (; kt + 3 < nk; kt += 2) {
        compute(0); store(1); sync_();
        compute(1); store(0); sync_();
      }
      if (kt < nk) { compute(0); if (kt + 1 < nk) store(1); sync_(); }
      if (kt + 1 < nk) { compute(1); if (kt + 2 < nk) store(0); sync_(); }
      if (kt + 2 < nk) { compute(0); sync_(); }
      return std::make_pair(c.conflicts(64).size(), barrier_no);
    };
    bool ok = true;
    long uninit = 0;
    int barriers = 0;
    for (int nk : {1, 2, 3, 4, 5, 6, 7}) {
      auto r = replay(nk, -1, &uninit);
      ok &= r.first == 0;
      barriers = r.second;
    }
    check(ok && uninit == 0, "access_check_gemm_double_buffer_clean");
    bool all_racy = true;
    for (int drop = 0; drop < barriers - 1; ++drop) {
      long u = 0;
      all_racy &= replay(7, drop, &u).first > 0;
    }
    check(all_racy, "access_check_gemm_double_buffer_without_a_barrier_races");
  }
  // --- the same with the shipped 16 x 16 x 4 form (gemm_f32.hpp tile_rowmajor, k16):
  // 128 x 128 x 16, 2 x 2 waves of 64 x 64, the four k quarters on the instruction's
  // four k slots.  Every
  // stage's fragment reads find words written by an earlier phase, and no read meets
  // a write of the same buffer between the same two barriers; dropping any one of
  // the loop's barriers makes the next phase's stores race its reads.
  {
    constexpr int BM = 128, BN = 128, BK = 16, WM = 2, WN = 2, T = 64 * WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / 16, FN = WTN / 16;
    constexpr int PA = BK + 4, PB = BN + 4, AV = BM * BK / 4 / T, BV = BK * BN / 4 / T;
    auto replay = [&](int nk, int drop_barrier, long* uninit) {
      std::vector<float> lds(2 * BM * PA + 2 * BK * PB);
      std::vector<char> written(lds.size(), 0);
      auto a_lds = matrices(lds.data(), 2, BM, PA);
      auto b_lds = matrices(lds.data() + 2 * BM * PA, 2, BK, PB);
      access_check::Checker c;
      int barrier_no = 0;
      auto sync_ = [&]() { if (barrier_no++ != drop_barrier) c.sync(0); };
      auto store = [&](int buf) {
        for (int t = 0; t < T; ++t) {
          for (int i = 0; i < AV; ++i) {
            const int q = t + T * i;
            for (int e = 0; e < 4; ++e) {
              float* w = &a_lds.idx(buf).at(layout::gemm_store_row<BK>(q), layout::gemm_store_word<BK>(q) + e);
              c.write(0, t, w); written[w - lds.data()] = 1;
            }
          }
          for (int i = 0; i < BV; ++i) {
            const int q = t + T * i;
            for (int e = 0; e < 4; ++e) {
              float* w = &b_lds.idx(buf).at(layout::gemm_store_row<BN>(q), layout::gemm_store_word<BN>(q) + e);
              c.write(0, t, w); written[w - lds.data()] = 1;
            }
          }
        }
      };
      auto compute = [&](int buf) {
        for (int t = 0; t < T; ++t) {
          const int w = t / 64, l = t % 64, quarter = l / 16, c16 = l % 16, wm = w / WN, wn = w % WN;
          for (int i = 0; i < FM; ++i)
            for (int e = 0; e < 4; ++e) {
              float* r = &a_lds.idx(buf).at(layout::gemm16_a_frag_row<WTM>(wm, i, c16),
                                            layout::gemm16_frag_k<BK>(quarter) + e);
              c.read(0, t, r); *uninit += !written[r - lds.data()];
            }
          for (int kk = 0; kk < 4; ++kk)
            for (int j = 0; j < FN; ++j) {
              float* r = &b_lds.idx(buf).at(layout::gemm16_frag_k<BK>(quarter) + kk,
                                            layout::gemm16_b_frag_word<WTN>(wn, j, c16));
              c.read(0, t, r); *uninit += !written[r - lds.data()];
            }
        }
      };
      // the schedule of tile_rowmajor with kDepth = 2
      store(0);
      sync_();
      int kt = 0;
      for (; kt + 3 < nk; kt += 2) {
        compute(0); store(1); sync_();
        compute(1); store(0); sync_();
      }
      if (kt < nk) { compute(0); if (kt + 1 < nk) store(1); sync_(); }
      if (kt + 1 < nk) { compute(1); if (kt + 2 < nk) store(0); sync_(); }
      if (kt + 2 < nk) { compute(0); sync_(); }
      return std::make_pair(c.conflicts(64).size(), barrier_no);
    };
    bool ok = true;
    long uninit = 0;
    int barriers = 0;
    for (int nk : {1, 2, 3, 4, 5, 6, 7}) {
      auto r = replay(nk, -1, &uninit);
      ok &= r.first == 0;
      barriers = r.second;
    }
    check(ok && uninit == 0, "access_check_gemm16_double_buffer_clean");
    bool all_racy = true;
    for (int drop = 0; drop < barriers - 1; ++drop) {
      long u = 0;
      all_racy &= replay(7, drop, &u).first > 0;
    }
    check(all_racy, "access_check_gemm16_double_buffer_without_a_barrier_races");
  }

  // --- segmented forms (segmented.hip): the unit map, the look-back windows and the
  // stores, with a unit of 2 waves x 2 rounds x 256 = 1024 elements (the kernels'
  // maps are templated on the unit).  Segments: empty, one element, unit edges, a
  // segment of 67 units (two look-back windows), at an offset inside the array.
  {
    constexpr int W = 2, Rr = 2, U = W * Rr * 256, TPB = W * 64;
    const std::vector<long> lens = {0, 1, 1023, 1024, 1025, 0, 3000, 67 * U - 5, 0, 2048, 7};
    const long S = (long)lens.size(), off0 = 5;
    std::vector<int64_t> off(S + 1);
    off[0] = off0;
    for (long s2 = 0; s2 < S; ++s2) off[s2 + 1] = off[s2] + lens[s2];
    const long n = off[S] + 13;
    // the plan: unit counts and their exclusive prefix (plan_kernel)
    std::vector<int64_t> us(S + 1, 0);
    for (long s2 = 0; s2 < S; ++s2)
      us[s2 + 1] = us[s2] + layout::seg_units(layout::seg_clamp(off[s2 + 1], n) -
                                                  layout::seg_clamp(off[s2], n), U);
    const long units = us[S];
    std::vector<int> in(n), out(n);
    std::vector<uint64_t> status(units);
    std::vector<int64_t> red(S);
    auto offv = array(off.data(), S + 1);
    auto usv = array(us.data(), S + 1);
    // scan: the plan clears the status words; then each unit stores its flag
    // word(s), walks its look-back windows, loads and stores its elements
    access_check::Checker c;
    for (long u = 0; u < units; ++u) c.write(0, u % 1024, &status[u]);
    c.kernel_boundary();
    Access cover(n);
    bool windows_ok = true, map_ok = true;
    for (long u = 0; u < units; ++u) {
      const layout::SegUnit su = layout::seg_unit(offv, usv, n, S, U, u);
      map_ok &= su.seg >= 0 && su.seg < S && su.j >= 0 && su.len > 0 && su.len <= U &&
                su.begin >= off[su.seg] && su.begin + su.len <= off[su.seg + 1];
      const long lane0 = u * TPB;
      c.atomic(u, lane0, &status[u], true);                 // aggregate, or the prefix at j = 0
      std::set<long> seen;
      for (long w = 0; 64 * w < su.j; ++w)                  // every window (no prefix found early)
        for (int l = 0; l < 64; ++l)
          if (layout::lookback_in_segment(su.j, w, l)) {
            const long v = layout::lookback_unit(u, w, l);
            windows_ok &= v >= us[su.seg] && v < u && seen.insert(v).second;
            if (v >= 0 && v < units) c.atomic(u, lane0 + l, &status[v], false);
          }
      windows_ok &= (long)seen.size() == su.j;
      if (su.j > 0) c.atomic(u, lane0, &status[u], true);   // the inclusive prefix
      for (int wv = 0; wv < W; ++wv)
        for (int l = 0; l < 64; ++l) {
          auto mine = layout::wave_striped<W, Rr>(array(out.data() + su.begin, U).group<4>(), 0,
                                                  R<Level::Wave>(wv, W), R<Level::Thread>(l, 64));
          auto mine_in = layout::wave_striped<W, Rr>(array(in.data() + su.begin, U).group<4>(), 0,
                                                     R<Level::Wave>(wv, W), R<Level::Thread>(l, 64));
          for (int r = 0; r < Rr; ++r)
            for (int k = 0; k < 4; ++k) {
              auto g = mine.idx(r);
              if (g.pos(k) >= su.len) continue;
              c.read(u, lane0 + wv * 64 + l, &mine_in.idx(r)[k]);
              c.write(u, lane0 + wv * 64 + l, &g[k]);
              cover.add(&g[k] - out.data(), u);
            }
        }
    }
    // every position of every segment is stored exactly once, nothing else
    long outside = 0, in_seg = 0;
    for (long i = 0; i < n; ++i) {
      const bool inside = i >= off[0] && i < off[S];
      in_seg += inside;
      outside += !inside && cover.owner[i] >= 0;
      map_ok &= !inside || cover.owner[i] >= 0;
    }
    check(map_ok && outside == 0 && cover.collisions == 0 && cover.touched == in_seg,
          "segmented_units_cover_every_segment_once",
          std::to_string(units) + " units, " + std::to_string(in_seg) + " positions");
    check(windows_ok, "segmented_lookback_windows_stay_in_segment");
    check(c.conflicts(64).empty(), "access_check_segmented_scan_clean",
          std::to_string(c.accesses()) + " accesses");
    // reduce: the plan zeroes the outputs of segments without exactly one
    // unit; a single-unit segment's block stores its sum, the others add
    // atomically.  Every output is then written (a store, or zero and adds);
    // plain stores from several units of one segment would race.
    auto reduce_access = [&](bool plain_everywhere, long* unset) {
      access_check::Checker r;
      std::vector<char> zeroed(S, 0), stored(S, 0);
      for (long s2 = 0; s2 < S; ++s2)
        if (us[s2 + 1] - us[s2] != 1) { r.write(0, s2 / 4, &red[s2]); zeroed[s2] = 1; }
      r.kernel_boundary();
      for (long u = 0; u < units; ++u) {
        const layout::SegUnit su = layout::seg_unit(offv, usv, n, S, U, u);
        if (su.single || plain_everywhere) { r.write(u, u * TPB, &red[su.seg]); stored[su.seg] = 1; }
        else r.atomic(u, u * TPB, &red[su.seg], true);
      }
      *unset = 0;
      for (long s2 = 0; s2 < S; ++s2) *unset += !(zeroed[s2] || stored[s2]);
      return r.conflicts(64).size();
    };
    long unset = 0, unset2 = 0;
    const size_t rc = reduce_access(false, &unset);
    const size_t rr = reduce_access(true, &unset2);
    check(rc == 0 && unset == 0, "access_check_segmented_reduce_clean");
    check(rr > 0, "access_check_segmented_reduce_plain_stores_race", std::to_string(rr) + " conflicts");
    // The persistent reduce: block b of G walks the contiguous units
    // [T b / G, T (b + 1) / G); a segment that starts and ends in the range
    // is stored by the block; the range's last segment, if it continues, is
    // published as the block's tail (every block writes its tail word); the
    // range's first segment, if it started earlier and ends here, is stored
    // by this block from the tails of earlier blocks back to the one where
    // it starts.  Every output is written exactly once, the ranges cover the
    // units once, and a block reads only tails of blocks of smaller index
    // whose ranges lie in the segment.
    auto persistent_reduce = [&](long G, bool, long* writes_bad) {
      access_check::Checker r;
      std::vector<uint64_t> tails(2 * G);
      std::vector<int> written(S, 0), covered(units, 0);
      const long TH = 64;
      auto first_unit = [&](long k) { return (long)((int64_t)units * k / G); };
      for (long b = 0; b < G; ++b)
        for (long s2 = b * TH; s2 < S; s2 += G * TH)
          for (long t = 0; t < TH && s2 + t < S; ++t)
            if (us[s2 + t] == us[s2 + t + 1]) { r.write(b, b * TH + t, &red[s2 + t]); ++written[s2 + t]; }
      *writes_bad = 0;
      for (long b = 0; b < G; ++b) {
        const long u0 = first_unit(b), u1 = first_unit(b + 1);
        long head_seg = -1;
        for (long u = u0; u < u1; ++u) {
          ++covered[u];
          const layout::SegUnit su = layout::seg_unit(offv, usv, n, S, U, u);
          if (u + 1 == us[su.seg + 1] || u + 1 == u1) {
            if (us[su.seg + 1] > u1) continue;                      // tail: published below
            if (us[su.seg] < u0) { head_seg = su.seg; continue; }
            r.write(b, b * TH, &red[su.seg]);
            ++written[su.seg];
          }
        }
        for (int h = 0; h < 2; ++h) r.atomic(b, b * TH, &tails[2 * b + h], true);
        if (head_seg >= 0) {
          for (long k = b - 1; k >= 0; --k) {
            if (first_unit(k) == first_unit(k + 1)) continue;
            // block k's range lies in the segment (its last unit does)
            *writes_bad += first_unit(k + 1) - 1 < us[head_seg];
            for (int h = 0; h < 2; ++h) r.atomic(b, b * TH, &tails[2 * k + h], false);
            if (first_unit(k) <= us[head_seg]) break;
          }
          r.write(b, b * TH, &red[head_seg]);
          ++written[head_seg];
        }
      }
      for (long s2 = 0; s2 < S; ++s2) *writes_bad += written[s2] != 1;
      for (long u = 0; u < units; ++u) *writes_bad += covered[u] != 1;
      return r.conflicts(64).size();
    };
    bool pr_ok = true;
    for (long G : {1L, 2L, 3L, 8L, 77L, 100L, 1000L}) {
      long bad = 0;
      pr_ok &= persistent_reduce(G, false, &bad) == 0 && bad == 0;
    }
    check(pr_ok, "access_check_segmented_persistent_reduce_clean");
  }

  // --- the grouped GEMM's persistent tile walk (grouped.hip): every tile of the
  // planned sequence is taken by exactly one block, runs of 64 stay on one XCD, and
  // the tiles' output regions partition every problem's C.  Within a block, thread 0
  // publishes the tile's slot in LDS and all threads read it after a barrier; the
  // barrier that ends each tile orders those reads before the next tile's store.
  {
    struct P { long M, N; };
    const std::vector<P> probs = {{130, 70}, {64, 64}, {1, 1}, {0, 5}, {200, 129}, {640, 64}, {65, 700}};
    const long G = (long)probs.size(), E = 64, TH = 256;
    std::vector<int64_t> ts(G + 1, 0);
    for (long g = 0; g < G; ++g)
      ts[g + 1] = ts[g] + ((probs[g].M + E - 1) / E) * ((probs[g].N + E - 1) / E);
    const long T = ts[G];
    std::vector<std::vector<float>> C(G);
    for (long g = 0; g < G; ++g) C[g].assign(std::max(0L, probs[g].M * probs[g].N), 0.f);
    auto walk_access = [&](long B, bool end_barrier, bool* ok) {
      access_check::Checker c;
      std::vector<long> taken(T, -1);
      std::vector<int64_t> s_slot(B);
      for (long b = 0; b < B; ++b) {
        const layout::TileWalk wk = layout::tile_walk(b, B);
        long prev = -1;
        for (long l = wk.first;; l += wk.per) {
          const long t = wk.tile(l);
          if (t >= T) break;
          *ok &= t > prev && taken[t] < 0;
          if (wk.by_xcd) *ok &= (t / 64) % 8 == b % 8;
          prev = t;
          taken[t] = b;
          c.write(b, b * TH, &s_slot[b]);
          c.sync(b);
          const long slot = layout::seg_of_unit(array(ts.data(), G + 1), G, t);
          *ok &= ts[slot] <= t && t < ts[slot + 1];
          const P& p = probs[slot];
          const long tn = (p.N + E - 1) / E, local = t - ts[slot];
          const long tm = local / tn, tc = local % tn;
          auto cm = matrix(C[slot].data(), p.M, p.N);
          for (long th = 0; th < TH; ++th) {
            c.read(b, b * TH + th, &s_slot[b]);
            for (long i = th; i < E * E; i += TH) {
              const long r = tm * E + i / E, col = tc * E + i % E;
              if (r < p.M && col < p.N) c.write(b, b * TH + th, &cm.at(r, col));
            }
          }
          if (end_barrier) c.sync(b);
        }
      }
      for (long t = 0; t < T; ++t) *ok &= taken[t] >= 0;
      return c;
    };
    bool ok = true, clean = true, racy = true;
    long writes = 0;
    for (long B : {1L, 3L, 7L, 8L, 16L, 24L, 64L}) {
      auto c = walk_access(B, true, &ok);
      clean &= c.conflicts(64).empty();
      writes += c.accesses();
      bool ok2 = true;
      racy &= !walk_access(B, false, &ok2).conflicts(64).empty() || T <= B;
    }
    // every element of every C written (the tiles cover it; the checker saw no
    // second writer of any element)
    long total = 0;
    for (long g = 0; g < G; ++g) total += std::max(0L, probs[g].M * probs[g].N);
    check(ok, "grouped_tile_walk_takes_every_tile_once", std::to_string(T) + " tiles");
    check(clean, "access_check_grouped_walk_clean", std::to_string(total) + " outputs per grid");
    check(racy, "access_check_grouped_walk_without_the_end_barrier_races");
  }

  // --- the float scan's hand-over (scan_f32.hip): every slot a tile waits for is
  // published once in the call, by a tile with a smaller index (so the waits end
  // when earlier tiles run); publications and polls are atomics, and the last tile's
  // clear of [used, hw) touches none of the call's words.  Over calls of changing
  // size, every word past the call's region is zero when the call ends, so no word
  // outlives the call after the one that wrote it.
  {
    constexpr int K = 4;                         // a small group, so that calls span many
    bool waits_ok = true, clean = true, stale_ok = true;
    std::vector<long> gen_of(2 * 300 + 2 * 80, 0);   // generation of each word's tag (0: zero)
    uint64_t hw = 0;
    long gen = 0;
    for (long T : {200L, 65L, 1L, 130L, 4L, 5L, 257L, 3L}) {
      ++gen;
      const long groups = (T + K - 1) / K;
      std::vector<long> agg_pub(T, -1), grp_pub(groups, -1);
      std::vector<uint64_t> words(gen_of.size());
      auto ag = array(words.data(), 2 * T).group<2>();
      auto gq = array(words.data() + 2 * T, 2 * groups).group<2>();
      access_check::Checker c;
      // publications (lane 0 of wave 0 of each tile)
      for (long t = 0; t < T; ++t) {
        for (int h = 0; h < 2; ++h) c.atomic(t, t * 64, &ag.idx(t)[h], true);
        agg_pub[t] = t;
        if (layout::handover_publishes_group<K>(t, T)) {
          const long g = t / K;
          waits_ok &= grp_pub[g] < 0;
          grp_pub[g] = t;
          for (int h = 0; h < 2; ++h) c.atomic(t, t * 64, &gq.idx(g)[h], true);
        }
      }
      // polls: every awaited slot has one publisher with a smaller index
      for (long t = 0; t < T; ++t) {
        const long g = t / K, pos = t % K;
        for (int l = 0; l < pos; ++l) {
          const long peer = layout::handover_peer<K>(t, l);
          waits_ok &= peer >= 0 && peer < t && agg_pub[peer] == peer;
          for (int h = 0; h < 2; ++h) c.atomic(t, t * 64 + l, &ag.idx(peer)[h], false);
        }
        if (g > 0) {
          waits_ok &= grp_pub[g - 1] >= 0 && grp_pub[g - 1] < t;
          for (int h = 0; h < 2; ++h) c.atomic(t, t * 64, &gq.idx(g - 1)[h], false);
        }
      }
      // the last tile clears [used, hw) with plain stores and raises hw to used
      const uint64_t used = (uint64_t)layout::handover_words<K>(T);
      waits_ok &= (uint64_t)(&gq.idx(groups - 1)[1] - words.data()) + 1 == used;
      for (uint64_t i = used; i < hw; ++i) c.write(T - 1, (T - 1) * 64 + (long)(i % 64), &words[i]);
      clean &= c.conflicts(16).empty();
      for (uint64_t i = 0; i < used; ++i) gen_of[i] = gen;
      for (uint64_t i = used; i < hw; ++i) gen_of[i] = 0;
      hw = used;
      for (size_t i = 0; i < gen_of.size(); ++i) stale_ok &= gen_of[i] == (i < used ? gen : 0);
    }
    check(waits_ok, "float_scan_handover_waits_on_earlier_tiles_only");
    check(clean, "access_check_float_scan_handover_clean");
    check(stale_ok, "float_scan_handover_leaves_no_older_word");
  }

  return g_fail;
}
