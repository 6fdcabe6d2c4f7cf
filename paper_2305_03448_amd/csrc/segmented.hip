// segmented.hip -- reduce and inclusive scan restarted at every segment
// (the batched form of the Sec. 5 reduction and scan): segment s covers
// positions [offsets[s], offsets[s+1]) of one int32 array.
//
// Work is cut into units: segment s of length L_s gives ceil(L_s / UNIT)
// units of at most UNIT consecutive elements (an empty segment gives none);
// UNIT is 8K to 64K elements, picked per size class by the tuning table.
//
//   plan kernel (one block of 1024 threads, 4096 segments per pass): unit
//     counts and their exclusive prefix over the segments, written to the
//     workspace with the total; for the reduction,
//     the outputs of segments spanning several units are zeroed (and empty
//     segments get 0); for the scan, the look-back status words are cleared.
//   main kernel: block b handles unit b (the grid is launched for the upper
//     bound S + n / UNIT units and blocks past the total return at once).  A
//     block finds its segment by binary search over the unit prefix, loads
//     its elements with dword-aligned 16-byte loads (segments start
//     anywhere), and
//       reduce: sums them in int64 and stores the sum, or adds it with one
//               device-scope atomic when the segment spans several units;
//       scan:   publishes the unit aggregate, looks back over the earlier
//               units of the same segment only (the look-back of the plain
//               scan, stopped at the segment's first unit), and writes its
//               part of the segment's scan.
//
// Units are handed out in block order, so a unit waits only on units whose
// blocks are already running.  Integer addition is associative, so results
// are exact and independent of the order.
#include "common.hpp"
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

// Workspace: header (total units), unit prefix [S + 1] int64, status [units].
struct SegWs {
  int64_t* total;        // number of units
  int64_t* unit_start;   // S + 1 entries
  uint64_t* status;      // one word per unit (scan)
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

// The unit's elements as [waves][rounds][lanes][4]; x[r][k] gets element
// (w * rounds + r) * 256 + lane * 4 + k (0 beyond the unit's length).
template <class C>
__device__ __forceinline__ void load_unit(const int32_t* in, const UnitInfo& ui,
                                          uint32_t (&x)[C::rounds][4]) {
  constexpr int kWaves = C::waves, kRounds = C::rounds, kUnit = C::unit;
  auto wv = wave_of_block<C::block>();
  auto lane = lane_of_wave();
  auto unit = array(in, 0).snd(ui.begin);
  if (ui.len == kUnit) {
    auto mine = layout::wave_striped<kWaves, kRounds>(array((const i32x4u*)&unit[0], kUnit / 4),
                                                      0, wv, lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const i32x4u q = mine[r];
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

template <class C>
__global__ __launch_bounds__(C::block) void seg_reduce_kernel(const int32_t* __restrict__ in,
                                                            int64_t n,
                                                            const int64_t* __restrict__ offsets,
                                                            int64_t S,
                                                            const int64_t* __restrict__ total,
                                                            const int64_t* __restrict__ unit_start,
                                                            int64_t* __restrict__ out) {
  constexpr int kBlock = C::block, kWaves = C::waves, kRounds = C::rounds;
  __shared__ int64_t s_w[kWaves];
  UnitInfo ui;
  if (!unit_info<C>(offsets, unit_start, n, S, total[0], &ui)) return;
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  uint32_t x[kRounds][4];
  load_unit<C>(in, ui, x);
  int64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += (int64_t)(int32_t)x[r][k];
  acc = wave::sum_i64(acc);
  if (lane_of_wave().index() == 0) s_w[wv.index()] = acc;
  sync(thread);
  if (thread.index() == 0) {
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += s_w[w];
    auto o = array(out, S);
    if (ui.single) o[ui.seg] = t;
    else __hip_atomic_fetch_add(&o[ui.seg], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ uint64_t pack(uint64_t flag, uint32_t v) { return (flag << 62) | v; }

// Exclusive prefix of unit u from the earlier units of its segment
// (j of them); one whole wave.
// At most `max_polls` polls (none with max_polls = 0); a wait that runs out
// records kDevWaitLimit and returns the partial prefix.
__device__ __forceinline__ uint32_t seg_look_back(const uint64_t* status, idx_t u, idx_t j,
                                                  uint32_t max_polls, WsHeader* hdr) {
  const int lane = wave::lane_id();
  uint32_t excl = 0;
  auto st = array(status, u);
  idx_t window = 0;                   // layout::lookback_unit's windows
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

template <class C>
__global__ __launch_bounds__(C::block) void seg_scan_kernel(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out, int64_t n,
                                                          const int64_t* __restrict__ offsets,
                                                          int64_t S,
                                                          const int64_t* __restrict__ total,
                                                          const int64_t* __restrict__ unit_start,
                                                          uint64_t* __restrict__ status,
                                                          WsHeader* __restrict__ hdr) {
  constexpr int kBlock = C::block, kWaves = C::waves, kRounds = C::rounds, kUnit = C::unit;
  __shared__ uint32_t s_wtot[kWaves];
  __shared__ uint32_t s_prefix;
  UnitInfo ui;
  if (!unit_info<C>(offsets, unit_start, n, S, total[0], &ui)) return;
  auto thread = thread_x<kBlock>();
  auto wv = wave_of_block<kBlock>();
  auto lane = lane_of_wave();
  const idx_t u = block_x().index();
  uint32_t x[kRounds][4];
  load_unit<C>(in, ui, x);

  uint32_t lsum = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) lsum += x[r][0] + x[r][1] + x[r][2] + x[r][3];
  const uint32_t wsum = wave::sum_u32(lsum);
  if (lane.index() == 0) s_wtot[wv.index()] = wsum;
  sync(thread);
  uint32_t wex = 0, agg = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t v = s_wtot[w];
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
      excl = seg_look_back(status, u, ui.j,
                           max_polls(__hip_atomic_load(&hdr->wait_limit, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)),
                           hdr);
      if (lane.index() == 0) store_status(&st[u], pack(kFlagPrefix, excl + agg));
    }
    if (lane.index() == 0) s_prefix = excl;
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
  const uint32_t add = s_prefix + wex;
  auto unit = array(out, 0).snd(ui.begin);
  if (ui.len == kUnit) {
    auto mine = layout::wave_striped<kWaves, kRounds>(array((i32x4u*)&unit[0], kUnit / 4), 0, wv,
                                                      lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      i32x4u q;
      q.x = (int32_t)(x[r][0] + add); q.y = (int32_t)(x[r][1] + add);
      q.z = (int32_t)(x[r][2] + add); q.w = (int32_t)(x[r][3] + add);
      mine[r] = q;
    }
  } else {
    auto mine = layout::wave_striped<kWaves, kRounds>(array(&unit[0], kUnit).group<4>(), 0, wv,
                                                      lane);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      auto g = mine.idx(r);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (g.pos(k) < ui.len) g[k] = (int32_t)(x[r][k] + add);
    }
  }
}

// Upper bound on the units of any configuration (the smallest unit).
int64_t max_units(int64_t n, int64_t S) { return S + (n + kMinUnit - 1) / kMinUnit; }

SegWs carve(void* ws, int64_t S) {
  uint8_t* w = (uint8_t*)ws;
  SegWs r;
  r.total = (int64_t*)(w + sizeof(WsHeader));
  r.unit_start = (int64_t*)(w + sizeof(WsHeader) + 64);
  r.status = (uint64_t*)(w + sizeof(WsHeader) + 64 + (((S + 1) * 8 + 63) & ~(int64_t)63));
  return r;
}

template <class C>
hipError_t launch_reduce(const int32_t* in, int64_t n, const int64_t* offsets, int64_t S,
                         int64_t* out, void* ws, hipStream_t s) {
  const SegWs w = carve(ws, S);
  hipLaunchKernelGGL((plan_kernel<C, false>), dim3(1), dim3(kPlanBlock), 0, s, offsets, n, S,
                     w.total, w.unit_start, out, (uint64_t*)nullptr, (int64_t)0);
  const int64_t grid = S + (n + C::unit - 1) / C::unit;
  if (grid > 0)
    hipLaunchKernelGGL(seg_reduce_kernel<C>, dim3((unsigned)grid), dim3(C::block), 0, s, in, n,
                       offsets, S, w.total, w.unit_start, out);
  return hipGetLastError();
}

template <class C>
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, const int64_t* offsets,
                       int64_t S, void* ws, hipStream_t s) {
  const SegWs w = carve(ws, S);
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
  const size_t head = sizeof(WsHeader) + 64 + (((S + 1) * 8 + 63) & ~(int64_t)63);
  return head + (scan ? (size_t)max_units(n, S) * 8 : 0);
}

int64_t segmented_max_grid(int64_t n, int64_t S) { return max_units(n, S); }

hipError_t reduce_segmented_i32(const int32_t* in, int64_t n, const int64_t* offsets, int64_t S,
                                int64_t* out, void* ws, hipStream_t s) {
  (void)kRegistered;
  switch (tune::get(tune::kSegReduceI32, tune::size_class(tune::kSegReduceI32, n))) {
    case 1: return launch_reduce<UnitCfg<256, 16>>(in, n, offsets, S, out, ws, s);
    case 2: return launch_reduce<UnitCfg<512, 16>>(in, n, offsets, S, out, ws, s);
    case 3: return launch_reduce<UnitCfg<1024, 8>>(in, n, offsets, S, out, ws, s);
    default: return launch_reduce<UnitCfg<256, 8>>(in, n, offsets, S, out, ws, s);
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
