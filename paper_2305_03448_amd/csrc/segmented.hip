// segmented.hip -- reduce and inclusive scan restarted at every segment
// (the batched form of the Sec. 5 reduction and scan): segment s covers
// positions [offsets[s], offsets[s+1]) of one int32 array.
//
// Work is cut into units: segment s of length L_s gives ceil(L_s / UNIT)
// units of at most UNIT consecutive elements (an empty segment gives none);
// UNIT is 8K to 64K elements, picked per size class by the tuning table.
// A unit finds its segment by binary search over the exclusive prefix of the
// unit counts, loads its elements with dword-aligned 16-byte loads (segments
// start anywhere), and
//   reduce: sums them in int64; a segment of one unit stores its sum, the
//           units of a longer one combine theirs (below);
//   scan:   publishes the unit aggregate, looks back over the earlier units
//           of the same segment only (the look-back of the plain scan,
//           stopped at the segment's first unit), and writes its part of the
//           segment's scan.
//
// Reduce, up to kSegLds segments (the batched workloads: thousands of
// uneven segments): one persistent launch.  Every block computes the unit
// prefix into its LDS (S + 1 int32) and then walks its own contiguous range
// of units in order, keeping running sums per segment, so it streams through
// contiguous memory and synchronises only where a segment ends.  A segment
// split between ranges is finished by the block holding its end, from the
// tail sums the earlier blocks publish (tagged with the call's generation,
// handover.hpp) when their ranges are done; those blocks have smaller
// indices and were dispatched first.  The last block waits for every tail,
// then clears the words the previous call left past this call's and
// advances the generation, as the plain scan does, so no word older than
// the previous call can match a later tag.
//
// Scan (and the reduce above kSegLds segments, and the batched forms): a
// one-block plan kernel writes the unit prefix to the workspace (zeroing
// the reduce outputs of segments without exactly one unit, which the units
// then add to atomically; clearing the scan status words), and a main
// kernel runs one block per unit (launched for the bound S + n / UNIT units;
// blocks past the total return at once, and units are handed out in block
// order, so a unit waits only on units whose blocks are already running).
//
// Integer addition is associative, so results are exact and independent of
// the order.
#include "common.hpp"
#include "handover.hpp"
#include "launch.hpp"
#include "layouts.hpp"
#include "tuning.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace {

// A unit is kBlock threads x kRounds rounds x 4 int32.
template <int kBlock_, int kRounds_>
struct UnitCfg {
  static constexpr int block = kBlock_;
  static constexpr int rounds = kRounds_;
  static constexpr int waves = kBlock_ / kWave;
  static constexpr int unit = waves * kWave * 4 * kRounds_;   // int32 per unit
};
constexpr int kMinUnit = 8192;   // smallest unit of the configurations below
constexpr uint64_t kFlagAggregate = 1, kFlagPrefix = 2;
constexpr int64_t kSegLds = 8192;   // segments whose unit prefix a block keeps in LDS

struct SegWs {
  int64_t* total;        // number of units (two-launch form)
  int64_t* unit_start;   // S + 1 entries (two-launch form)
  uint64_t* status;      // one word per unit (scan)
  uint64_t* words;       // two tail words per block (persistent reduce)
};

template <class C>
__device__ __forceinline__ int64_t units_of(int64_t len) { return layout::seg_units(len, C::unit); }

// Offsets are read clamped to [0, n]: offsets that break the documented
// precondition (non-decreasing, within the array) give unspecified results
// but never an access outside the array.
__device__ __forceinline__ int64_t clampn(int64_t v, int64_t n) { return layout::seg_clamp(v, n); }

// One block of kPlanBlock threads, kPlanPer consecutive segments per thread:
// unit counts and their exclusive prefix over the segments, a chunk of
// kPlanBlock * kPlanPer segments per pass with a running carry; then per-op
// initialisation.  Reduce: the outputs of segments that do not have exactly
// one unit are zeroed (atomics add into them; an empty segment sums to 0).
// Scan: the look-back status words are cleared.
constexpr int kPlanBlock = 1024, kPlanPer = 4, kPlanWaves = kPlanBlock / kWave;

template <class C, bool kScan>
__global__ __launch_bounds__(kPlanBlock) void plan_kernel(const int64_t* __restrict__ offsets,
                                                          int64_t n, int64_t S,
                                                          int64_t* __restrict__ total,
                                                          int64_t* __restrict__ unit_start,
                                                          int64_t* __restrict__ red_out,
                                                          uint64_t* __restrict__ status,
                                                          int64_t max_units) {
  __shared__ int64_t s_wsum[kPlanWaves];
  __shared__ int64_t s_carry;
  auto thread = thread_x<kPlanBlock>();
  auto wv = wave_of_block<kPlanBlock>();
  auto lane = lane_of_wave();
  auto off = array(offsets, S + 1);
  auto us = array(unit_start, S + 1);
  if (thread.index() == 0) s_carry = 0;
  sync(thread);
  for (idx_t base = 0; base < S; base += kPlanBlock * kPlanPer) {
    const idx_t s0 = base + thread.index() * kPlanPer;
    int64_t u[kPlanPer];
    int64_t mine = 0;
#pragma unroll
    for (int j = 0; j < kPlanPer; ++j) {
      const idx_t s = s0 + j;
      const int64_t len = s < S ? clampn(off[s + 1], n) - clampn(off[s], n) : 0;
      u[j] = s < S ? units_of<C>(len > 0 ? len : 0) : 0;
      if constexpr (!kScan) {
        if (s < S && u[j] != 1) array(red_out, S)[s] = 0;
      }
      mine += u[j];
    }
    // block-wide exclusive prefix of the per-thread unit counts (int64)
    int64_t incl = mine;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int64_t t = __shfl_up(incl, d, kWave);
      if ((int)lane.index() >= d) incl += t;
    }
    if (lane.index() == kWave - 1) s_wsum[wv.index()] = incl;
    sync(thread);
    int64_t before = s_carry;
    for (int w = 0; w < kPlanWaves; ++w) before += (w < wv.index()) ? s_wsum[w] : 0;
    int64_t at = before + incl - mine;
#pragma unroll
    for (int j = 0; j < kPlanPer; ++j) {
      if (s0 + j < S) us[s0 + j] = at;
      at += u[j];
    }
    sync(thread);
    if (thread.index() == kPlanBlock - 1) s_carry = before + incl;
    sync(thread);
  }
  if (thread.index() == 0) {
    us[S] = s_carry;
    total[0] = s_carry;
  }
  if constexpr (kScan) {
    auto st = array(status, max_units);
    for (idx_t i = thread.index(); i < max_units; i += kPlanBlock) st[i] = 0;
  }
}

struct UnitInfo {
  idx_t seg, j, begin, len;   // segment, unit index inside it, first position, length
  bool single;                // the segment has one unit only
};

// Unit u of this block (layout::seg_unit, read by thread 0 and shared).
template <class C>
__device__ __forceinline__ bool unit_info(const int64_t* offsets, const int64_t* unit_start,
                                          int64_t n, int64_t S, int64_t total, UnitInfo* out) {
  __shared__ int64_t s_info[5];
  auto thread = thread_x<C::block>();
  const idx_t u = block_x().index();
  if (u >= total) return false;
  if (thread.index() == 0) {
    const layout::SegUnit su =
        layout::seg_unit(array(offsets, S + 1), array(unit_start, S + 1), n, S, C::unit, u);
    s_info[0] = su.seg; s_info[1] = su.j; s_info[2] = su.begin;
    s_info[3] = su.len; s_info[4] = su.single;
  }
  sync(thread);
  *out = UnitInfo{s_info[0], s_info[1], s_info[2], s_info[3], s_info[4] != 0};
  return true;
}

// Unit u from a unit prefix kept in LDS (int32, S + 1 entries): read by
// thread 0 and shared; the caller synchronises before the next unit.
template <class C>
__device__ __forceinline__ UnitInfo unit_info_lds(const int64_t* offsets, const int32_t* s_us,
                                                 int64_t n, int64_t S, idx_t u) {
  __shared__ int64_t s_info[5];
  auto thread = thread_x<C::block>();
  if (thread.index() == 0) {
    const layout::SegUnit su =
        layout::seg_unit(array(offsets, S + 1), array(s_us, S + 1), n, S, C::unit, u);
    s_info[0] = su.seg; s_info[1] = su.j; s_info[2] = su.begin;
    s_info[3] = su.len; s_info[4] = su.single;
  }
  sync(thread);
  return UnitInfo{s_info[0], s_info[1], s_info[2], s_info[3], s_info[4] != 0};
}

// Every block's plan for the persistent forms: s_us[s] = units before
// segment s (exclusive prefix of the unit counts), s_us[S] = the total.
// The counts are computed with strided, independent loads of the offsets
// (in flight together), then thread t scans ceil(S / kThreads) consecutive
// counts in LDS.
template <int kThreads>
__device__ __forceinline__ int32_t lds_unit_plan(const int64_t* offsets, int64_t n, int64_t S,
                                                 int64_t unit, int32_t* s_us, int32_t* s_wsum) {
  auto thread = thread_x<kThreads>();
  auto wv = wave_of_block<kThreads>();
  auto lane = lane_of_wave();
  auto off = array(offsets, S + 1);
  auto us = array(s_us, S + 1);
  for (idx_t s = thread.index(); s < S; s += kThreads) {
    const int64_t len = layout::seg_clamp(off[s + 1], n) - layout::seg_clamp(off[s], n);
    us[s] = (int32_t)layout::seg_units(len, unit);
  }
  sync(thread);
  const idx_t per = (S + kThreads - 1) / kThreads;
  const idx_t s0 = thread.index() * per, s1 = s0 + per < S ? s0 + per : S;
  int32_t mine = 0;
  for (idx_t s = s0; s < s1; ++s) mine += us[s];
  int32_t incl = mine;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t t = __shfl_up(incl, d, kWave);
    if ((int)lane.index() >= d) incl += t;
  }
  if (lane.index() == kWave - 1) s_wsum[wv.index()] = incl;
  sync(thread);
  int32_t at = incl - mine, total = 0;
  for (int w = 0; w < kThreads / kWave; ++w) {
    const int32_t v = s_wsum[w];
    at += w < (int)wv.index() ? v : 0;
    total += v;
  }
  for (idx_t s = s0; s < s1; ++s) {
    const int32_t c = us[s];
    us[s] = at;
    at += c;
  }
  if (thread.index() == 0) us[S] = total;
  sync(thread);
  return total;
}

// The thread's wave and lane, through an empty asm: in the persistent
// loops the compiler would otherwise hoist every per-lane address of a unit
// out of the loop and keep them live across units (about twice the
// registers).
__device__ __forceinline__ uint32_t opaque_thread() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// The unit's elements as [waves][rounds][lanes][4]; x[r][k] gets element
// (w * rounds + r) * 256 + lane * 4 + k (0 beyond the unit's length).
// kNt: non-temporal 16-byte loads (the reduce, which only streams its input;
// 4 % faster there, 3 % slower for the scan, which writes as it reads).
template <class C, bool kNt = false>
__device__ __forceinline__ void load_unit(const int32_t* in, const UnitInfo& ui,
                                          uint32_t (&x)[C::rounds][4]) {
  constexpr int kWaves = C::waves, kRounds = C::rounds, kUnit = C::unit;
  const uint32_t t = opaque_thread();
  const Wave<kWaves> wv{(idx_t)(t / kWave), kWaves};
  const Lane<kWave> lane{(idx_t)(t % kWave), kWave};
  auto unit = array(in, 0).snd(ui.begin);
  if (ui.len == kUnit) {
    auto mine = layout::wave_striped<kWaves, kRounds>(array((const i32x4u*)&unit[0], kUnit / 4),
                                                      0, wv, lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      i32x4u q;
      if constexpr (kNt) q = __builtin_nontemporal_load(&mine[r]);
      else q = mine[r];
      x[r][0] = (uint32_t)q.x; x[r][1] = (uint32_t)q.y;
      x[r][2] = (uint32_t)q.z; x[r][3] = (uint32_t)q.w;
    }
  } else {
    auto mine = layout::wave_striped<kWaves, kRounds>(array(&unit[0], kUnit).group<4>(), 0, wv,
                                                      lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      auto g = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k) x[r][k] = g.pos(k) < ui.len ? (uint32_t)g[k] : 0u;
    }
  }
}

// The unit's sum (int64), valid in thread 0.
template <class C>
__device__ __forceinline__ int64_t reduce_unit(const int32_t* in, const UnitInfo& ui,
                                               int64_t* s_w) {
  constexpr int kBlock = C::block, kWaves = C::waves, kRounds = C::rounds;
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  uint32_t x[kRounds][4];
  load_unit<C, true>(in, ui, x);
  int64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += (int64_t)(int32_t)x[r][k];
  acc = wave::sum_i64(acc);
  if (lane_of_wave().index() == 0) s_w[wv.index()] = acc;
  sync(thread);
  int64_t t = 0;
  if (thread.index() == 0) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += s_w[w];
  }
  return t;
}

template <class C>
__global__ __launch_bounds__(C::block) void seg_reduce_kernel(const int32_t* __restrict__ in,
                                                            int64_t n,
                                                            const int64_t* __restrict__ offsets,
                                                            int64_t S,
                                                            const int64_t* __restrict__ total,
                                                            const int64_t* __restrict__ unit_start,
                                                            int64_t* __restrict__ out) {
  __shared__ int64_t s_w[C::waves];
  UnitInfo ui;
  if (!unit_info<C>(offsets, unit_start, n, S, total[0], &ui)) return;
  const int64_t t = reduce_unit<C>(in, ui, s_w);
  if (thread_x<C::block>().index() == 0) {
    auto o = array(out, S);
    if (ui.single) o[ui.seg] = t;
    else __hip_atomic_fetch_add(&o[ui.seg], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The persistent reduce (up to kSegLds segments): see the file comment.
// Block b takes the contiguous units [T b / G, T (b + 1) / G) and walks
// them in order, each thread adding its elements into a running int64 sum
// for the current segment; at the end of a segment (or of the range) the
// block adds the threads' sums.  A segment that starts and ends in the range
// is stored at once.  The range's last segment, when it continues past the
// range, is the block's tail: its part is published (every block publishes
// one tail word pair, 0 when it has none).  The range's first segment, when
// it started in an earlier range and ends in this one, is resolved at the
// end: its part here plus the tails of the earlier blocks back to the one
// where it starts -- blocks of smaller index, dispatched earlier, which
// publish once their ranges are done.  Block G - 1 ends the call.
template <class C>
__global__ __launch_bounds__(C::block) void seg_reduce_persistent_kernel(
    const int32_t* __restrict__ in, int64_t n, const int64_t* __restrict__ offsets, int64_t S,
    int64_t* __restrict__ out, uint64_t* __restrict__ words, WsHeader* __restrict__ hdr) {
  constexpr int kRounds = C::rounds;
  __shared__ int32_t s_us[kSegLds + 1];
  __shared__ int32_t s_wsum[C::waves];
  __shared__ int64_t s_w[C::waves];
  __shared__ CallState s_call;
  auto block = block_x();
  auto thread = thread_x<C::block>();
  auto wv = wave_of_block<C::block>();
  if (thread.index() == 0) s_call = read_call_state(hdr);
  const int32_t T = lds_unit_plan<C::block>(offsets, n, S, C::unit, s_us, s_wsum);  // syncs
  const uint32_t gen = s_call.gen;
  const uint64_t tag = handover::tag_of(gen);
  const idx_t G = block.count(), b = block.index();
  auto first_unit = [&](idx_t k) { return (idx_t)((int64_t)T * k / G); };
  const idx_t u0 = first_unit(b), u1 = first_unit(b + 1);
  auto o = array(out, S);
  auto off = array(offsets, S + 1);
  auto us = array(s_us, S + 1);
  auto tails = array(words, 2 * G).group<2>();              // [G][2]
  for (idx_t s = b * C::block + thread.index(); s < S; s += G * C::block)
    if (us[s] == us[s + 1]) o[s] = 0;                       // empty segment
  // the threads' sums added over the block, valid in thread 0
  auto block_total = [&](int64_t v) {
    v = wave::sum_i64(v);
    sync(thread);                                           // earlier readers of s_w are done
    if (lane_of_wave().index() == 0) s_w[wv.index()] = v;
    sync(thread);
    int64_t t = 0;
    if (thread.index() == 0)
      for (int w = 0; w < C::waves; ++w) t += s_w[w];
    return t;
  };
  int64_t tail = 0, head = 0;
  idx_t head_seg = -1;
  int64_t acc = 0;
  idx_t seg = u0 < u1 ? layout::seg_of_unit(us, S, u0) : 0;
  int64_t sb = layout::seg_clamp(off[seg], n), se = layout::seg_clamp(off[seg + 1], n);
#pragma clang loop unroll(disable)
  for (idx_t u = u0; u < u1; ++u) {
    if (us[seg + 1] <= u) {                                  // the next non-empty segment
      do ++seg; while (us[seg + 1] <= u);
      sb = layout::seg_clamp(off[seg], n);
      se = layout::seg_clamp(off[seg + 1], n);
    }
    const idx_t j = u - us[seg], begin = sb + j * C::unit;
    const UnitInfo ui{seg, j, begin, se - begin < C::unit ? se - begin : C::unit, false};
    uint32_t x[kRounds][4];
    load_unit<C, true>(in, ui, x);
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc += (int64_t)(int32_t)x[r][k];
    if (u + 1 == us[seg + 1] || u + 1 == u1) {               // the segment's part here ends
      const int64_t total = block_total(acc);
      acc = 0;
      if (thread.index() == 0) {
        if (us[seg + 1] > u1) tail = total;                  // continues past the range
        else if (us[seg] < u0) { head = total; head_seg = seg; }
        else o[seg] = total;
      }
    }
  }
  if (thread.index() == 0) {
    handover::publish(&tails.idx(b)[0], tag, (uint64_t)tail);
    if (head_seg >= 0) {                                     // add the earlier blocks' tails
      bool ok = true;
      for (idx_t k = b - 1; k >= 0; --k) {
        if (first_unit(k) == first_unit(k + 1)) continue;   // an empty range
        uint64_t v = 0;
        ok = handover::poll(&tails.idx(k)[0], tag, v, s_call.polls) && ok;
        head += (int64_t)v;
        if (first_unit(k) <= us[head_seg]) break;            // the block where it starts
      }
      if (!ok) set_error(hdr, kDevWaitLimit);
      o[head_seg] = head;
    }
  }
  if (b == G - 1) {
    // every block publishes its tail after reading the generation: once all
    // have, advance it and clear what the previous call left past 2 G words
    sync(thread);
    bool ok = true;
    for (idx_t k = thread.index(); k < G; k += C::block) {
      uint64_t v = 0;
      ok = handover::poll(&tails.idx(k)[0], tag, v, s_call.polls) && ok;
    }
    if (!ok) set_error(hdr, kDevWaitLimit);
    sync(thread);
    const uint64_t used = 2 * (uint64_t)G;
    const uint64_t hw = __hip_atomic_load(&hdr->hw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    clear_words<C::block>(words, used, hw, thread.index());
    if (thread.index() == 0) {
      __hip_atomic_store(&hdr->hw, used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      store_u32(&hdr->gen, next_gen(gen));
    }
  }
}

__device__ __forceinline__ uint64_t pack(uint64_t flag, uint32_t v) { return (flag << 62) | v; }

// Exclusive prefix of unit u from the earlier units of its segment
// (j of them, layout::lookback_unit's windows); one whole wave.
// At most `max_polls` polls (none with max_polls = 0); a wait that runs out
// records kDevWaitLimit and returns the partial prefix.
__device__ __forceinline__ uint32_t seg_look_back(const uint64_t* status, idx_t u, idx_t j,
                                                  uint32_t max_polls, WsHeader* hdr) {
  const int lane = wave::lane_id();
  uint32_t excl = 0;
  auto st = array(status, u);
  idx_t window = 0;
  for (uint32_t polls = 0; kWave * window < j; ++polls) {
    if (polls == max_polls) {
      if (lane == 0) set_error(hdr, kDevWaitLimit);
      break;
    }
    const bool in_seg = layout::lookback_in_segment(j, window, lane);
    const uint64_t w =
        in_seg ? load_status(&st[layout::lookback_unit(u, window, lane)]) : pack(kFlagPrefix, 0u);
    const uint32_t flag = (uint32_t)(w >> 62);
    const uint64_t pmask = __ballot(flag == kFlagPrefix && in_seg);
    const idx_t left = j - kWave * window;
    const int width = left < kWave ? (int)left : kWave;
    const int first_p = pmask ? __builtin_ctzll(pmask) : width - 1;
    const uint64_t need = first_p == 63 ? ~0ull : ((2ull << first_p) - 1);
    if (__ballot(flag == 0 && in_seg) & need) {
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    excl += wave::sum_u32(lane <= first_p && in_seg ? (uint32_t)w : 0u);
    if (pmask) break;
    ++window;
  }
  return excl;
}

struct ScanShared {
  uint32_t wtot[16];   // wave totals (up to 1024 threads)
  uint32_t prefix;     // the unit's exclusive prefix
};

// One unit of the segmented scan (u its index).
template <class C>
__device__ __forceinline__ void scan_unit(const int32_t* __restrict__ in,
                                          int32_t* __restrict__ out, const UnitInfo& ui, idx_t u,
                                          uint64_t* __restrict__ status, uint32_t polls,
                                          WsHeader* __restrict__ hdr, ScanShared& sh) {
  constexpr int kBlock = C::block, kWaves = C::waves, kRounds = C::rounds, kUnit = C::unit;
  static_assert(kWaves <= 16, "wave totals fit ScanShared");
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  auto lane = lane_of_wave();
  uint32_t x[kRounds][4];
  load_unit<C>(in, ui, x);

  uint32_t lsum = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) lsum += x[r][0] + x[r][1] + x[r][2] + x[r][3];
  const uint32_t wsum = wave::sum_u32(lsum);
  if (lane.index() == 0) sh.wtot[wv.index()] = wsum;
  sync(thread);
  uint32_t wex = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t v = sh.wtot[w];
    wex += (w < wv.index()) ? v : 0u;
    agg += v;
  }
  auto st = array(status, u + 1);
  if (wv.index() == 0) {
    uint32_t excl = 0;
    if (ui.j == 0) {
      if (lane.index() == 0) store_status(&st[u], pack(kFlagPrefix, agg));
    } else {
      if (lane.index() == 0) store_status(&st[u], pack(kFlagAggregate, agg));
      excl = seg_look_back(status, u, ui.j, polls, hdr);
      if (lane.index() == 0) store_status(&st[u], pack(kFlagPrefix, excl + agg));
    }
    if (lane.index() == 0) sh.prefix = excl;
  }
  uint32_t carry = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    x[r][1] += x[r][0];
    x[r][2] += x[r][1];
    x[r][3] += x[r][2];
    const uint32_t t = x[r][3];
    const uint32_t incl = wave::inclusive_add_u32(t);
    const uint32_t ex = carry + incl - t;
#pragma unroll
    for (int k = 0; k < 4; ++k) x[r][k] += ex;
    carry += wave::lane_read_u32(incl, kWave - 1);
  }
  sync(thread);
  const uint32_t add = sh.prefix + wex;
  auto unit = array(out, 0).snd(ui.begin);
  const uint32_t ot = opaque_thread();
  const Wave<kWaves> owv{(idx_t)(ot / kWave), kWaves};
  const Lane<kWave> olane{(idx_t)(ot % kWave), kWave};
  if (ui.len == kUnit) {
    auto mine = layout::wave_striped<kWaves, kRounds>(array((i32x4u*)&unit[0], kUnit / 4), 0,
                                                      owv, olane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      i32x4u q;
      q.x = (int32_t)(x[r][0] + add); q.y = (int32_t)(x[r][1] + add);
      q.z = (int32_t)(x[r][2] + add); q.w = (int32_t)(x[r][3] + add);
      mine[r] = q;
    }
  } else {
    auto mine = layout::wave_striped<kWaves, kRounds>(array(&unit[0], kUnit).group<4>(), 0,
                                                      owv, olane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      auto g = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (g.pos(k) < ui.len) g[k] = (int32_t)(x[r][k] + add);
    }
  }
}

template <class C>
__global__ __launch_bounds__(C::block) void seg_scan_kernel(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out, int64_t n,
                                                          const int64_t* __restrict__ offsets,
                                                          int64_t S,
                                                          const int64_t* __restrict__ total,
                                                          const int64_t* __restrict__ unit_start,
                                                          uint64_t* __restrict__ status,
                                                          WsHeader* __restrict__ hdr) {
  __shared__ ScanShared sh;
  UnitInfo ui;
  if (!unit_info<C>(offsets, unit_start, n, S, total[0], &ui)) return;
  scan_unit<C>(in, out, ui, block_x().index(), status,
               max_polls(__hip_atomic_load(&hdr->wait_limit, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT)),
               hdr, sh);
}

// Upper bound on the units of any configuration (the smallest unit).
int64_t max_units(int64_t n, int64_t S) { return S + (n + kMinUnit - 1) / kMinUnit; }
int64_t round64(int64_t b) { return (b + 63) & ~(int64_t)63; }

// Workspace: header; the unit total of the two-launch form (one 64-byte
// line); the state words at a fixed place, so that the extent a call leaves
// in the header (hw) means the same words to the next call whatever its
// size -- for the scan the status words (one per unit, both forms), for the
// reduce the persistent form's tail words (two per block); then
// the two-launch form's unit prefix (S + 1 int64), whose values (below
// 2^31) never carry a tag or a flag if a later call finds them among its
// state words.
constexpr int64_t kMaxReduceBlocks = 4096;   // grid of the persistent reduce, at most
int64_t state_words(int64_t n, int64_t S, bool scan) {
  const int64_t mu = max_units(n, S);
  return scan ? mu : 2 * (mu < kMaxReduceBlocks ? mu : kMaxReduceBlocks);
}

SegWs carve(void* ws, int64_t n, int64_t S, bool scan) {
  uint8_t* w = (uint8_t*)ws;
  SegWs r;
  r.total = (int64_t*)(w + sizeof(WsHeader));
  r.status = (uint64_t*)(w + sizeof(WsHeader) + 64);
  r.words = r.status;
  r.unit_start = (int64_t*)(w + sizeof(WsHeader) + 64 + round64(state_words(n, S, scan) * 8));
  return r;
}

// The persistent forms: up to kSegLds segments and unit counts in int32.
bool persistent_fits(int64_t n, int64_t S) {
  return S > 0 && S <= kSegLds && max_units(n, S) < (1ll << 31);
}

template <class C>
hipError_t launch_reduce(const int32_t* in, int64_t n, const int64_t* offsets, int64_t S,
                         int64_t* out, void* ws, hipStream_t s, bool persistent) {
  const SegWs w = carve(ws, n, S, false);
  const int64_t units = S + (n + C::unit - 1) / C::unit;   // at least the units of the call
  if (persistent && persistent_fits(n, S)) {
    static int resident[64] = {0};
    int64_t g = launch::resident_grid(seg_reduce_persistent_kernel<C>, resident, 1, C::block);
    if (g > units) g = units;
    if (g > kMaxReduceBlocks) g = kMaxReduceBlocks;
    hipLaunchKernelGGL(seg_reduce_persistent_kernel<C>, dim3((unsigned)g), dim3(C::block), 0, s,
                       in, n, offsets, S, out, w.words, (WsHeader*)ws);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((plan_kernel<C, false>), dim3(1), dim3(kPlanBlock), 0, s, offsets, n, S,
                     w.total, w.unit_start, out, (uint64_t*)nullptr, (int64_t)0);
  if (units > 0)
    hipLaunchKernelGGL(seg_reduce_kernel<C>, dim3((unsigned)units), dim3(C::block), 0, s, in, n,
                       offsets, S, w.total, w.unit_start, out);
  return hipGetLastError();
}

// The scan stays in the two-launch form: in a persistent grid the units of
// one round run together, so a unit's look-back finds its predecessors still
// running, where in-order dispatch has started them earlier (measured on the
// 4096-segment workload: 535 us against 469 us).
template <class C>
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, const int64_t* offsets,
                       int64_t S, void* ws, hipStream_t s) {
  const SegWs w = carve(ws, n, S, true);
  const int64_t mu = S + (n + C::unit - 1) / C::unit;
  hipLaunchKernelGGL((plan_kernel<C, true>), dim3(1), dim3(kPlanBlock), 0, s, offsets, n, S,
                     w.total, w.unit_start, (int64_t*)nullptr, w.status, mu);
  if (mu > 0)
    hipLaunchKernelGGL(seg_scan_kernel<C>, dim3((unsigned)mu), dim3(C::block), 0, s, in, out, n,
                       offsets, S, w.total, w.unit_start, w.status, (WsHeader*)ws);
  return hipGetLastError();
}

// The reduce has no 64K unit: holding 16 rounds in 1024 threads spills.
constexpr const char* kNames[] = {"unit8k", "unit16k", "unit32k", "unit32k_w16", "unit64k_w16"};
constexpr int kReduceDefaults[tune::kClasses] = {0, 0, 0, 1};
constexpr int kScanDefaults[tune::kClasses] = {0, 0, 0, 2};
const bool kRegistered =
    (tune::register_op(tune::kSegReduceI32, "seg_reduce_i32", 4, kNames, kReduceDefaults),
     tune::register_op(tune::kSegScanI32, "seg_scan_i32", 5, kNames, kScanDefaults), true);

}  // namespace

namespace launch {

size_t segmented_workspace(int64_t n, int64_t S, bool scan) {
  return (size_t)(sizeof(WsHeader) + 64 + round64(state_words(n, S, scan) * 8) + (S + 1) * 8);
}

int64_t segmented_max_grid(int64_t n, int64_t S) { return max_units(n, S); }

hipError_t reduce_segmented_i32(const int32_t* in, int64_t n, const int64_t* offsets, int64_t S,
                                int64_t* out, void* ws, hipStream_t s, bool persistent) {
  (void)kRegistered;
  switch (tune::get(tune::kSegReduceI32, tune::size_class(tune::kSegReduceI32, n))) {
    case 1: return launch_reduce<UnitCfg<256, 16>>(in, n, offsets, S, out, ws, s, persistent);
    case 2: return launch_reduce<UnitCfg<512, 16>>(in, n, offsets, S, out, ws, s, persistent);
    case 3: return launch_reduce<UnitCfg<1024, 8>>(in, n, offsets, S, out, ws, s, persistent);
    default: return launch_reduce<UnitCfg<256, 8>>(in, n, offsets, S, out, ws, s, persistent);
  }
}

hipError_t scan_segmented_i32(const int32_t* in, int32_t* out, int64_t n, const int64_t* offsets,
                              int64_t S, void* ws, hipStream_t s) {
  (void)kRegistered;
  switch (tune::get(tune::kSegScanI32, tune::size_class(tune::kSegScanI32, n))) {
    case 1: return launch_scan<UnitCfg<256, 16>>(in, out, n, offsets, S, ws, s);
    case 2: return launch_scan<UnitCfg<512, 16>>(in, out, n, offsets, S, ws, s);
    case 3: return launch_scan<UnitCfg<1024, 8>>(in, out, n, offsets, S, ws, s);
    case 4: return launch_scan<UnitCfg<1024, 16>>(in, out, n, offsets, S, ws, s);
    default: return launch_scan<UnitCfg<256, 8>>(in, out, n, offsets, S, ws, s);
  }
}

}  // namespace launch
}  // namespace desc
