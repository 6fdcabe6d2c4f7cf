// lookback.hpp -- the inter-tile carry of the single-pass scans (decoupled
// look-back), shared by the plain and the segmented scan.
//
// Every tile owns one 64-bit status word {flag:2, generation tag:30,
// value:32}, read and written with single relaxed agent-scope atomics, so
// no fence is needed to make the value visible to blocks on other XCDs.
// flag 1 (aggregate): the value is the tile's own sum; flag 2 (prefix): the
// value is the inclusive prefix up to the tile's end.  Words whose tag is
// not the current generation read as "not ready", which lets the next call
// reuse the workspace without a clearing pass.  A call writes the word of
// every one of its tiles, and the block that advances the generation clears
// the words the previous call left beyond its own tiles, so no word older
// than the previous call survives to match a later call's tag.
#pragma once
#include "common.hpp"
#include "view.hpp"
#include "wave.hpp"

namespace desc {
namespace scan_detail {

constexpr uint64_t kFlagAggregate = 1, kFlagPrefix = 2;
constexpr uint32_t kTagMask = 0x3fffffffu;
constexpr int kLookWords = 4;                     // status words per lane per poll
constexpr int kWindow = kWave * kLookWords;       // tiles per poll

__device__ __forceinline__ uint64_t pack(uint64_t flag, uint32_t gen, uint32_t v) {
  return (flag << 62) | ((uint64_t)(gen & kTagMask) << 32) | (uint64_t)v;
}
// Exclusive prefix of tile `tile` from the status words of its predecessors.
// Called by one whole wave; the result is valid in every lane.  Window
// position p = q * 64 + lane (q < kLookWords) reads tile pos - p, so the
// window runs backwards from `pos` in order of p.
// At most `max_polls` polls (none with max_polls = 0); a wait that runs out
// records kDevWaitLimit and returns the partial prefix.
__device__ __forceinline__ uint32_t look_back(const uint64_t* __restrict__ status, idx_t tile,
                                              uint32_t gen, uint32_t max_polls,
                                              WsHeader* __restrict__ hdr) {
  const int lane = wave::lane_id();
  const uint32_t tag = gen & kTagMask;
  uint32_t excl = 0;
  idx_t pos = tile - 1;
  auto st = array(status, tile);
  for (uint32_t polls = 0;; ++polls) {
    if (polls == max_polls) {      // inconsistent workspace: give up, flag it
      if (lane == 0) set_error(hdr, kDevWaitLimit);
      break;
    }
    uint64_t w[kLookWords];
#pragma unroll
    for (int q = 0; q < kLookWords; ++q) {
      const idx_t j = pos - (q * kWave + lane);
      w[q] = j >= 0 ? load_status(&st[j]) : pack(kFlagPrefix, gen, 0u);
    }
    // First window position holding an inclusive prefix, and whether every
    // position up to it has published.
    int first_p = kWindow;         // none
    bool missing = false;
#pragma unroll
    for (int q = kLookWords - 1; q >= 0; --q) {
      const uint32_t flag = (uint32_t)(w[q] >> 62);
      const bool valid = flag != 0 && (uint32_t)((w[q] >> 32) & kTagMask) == tag;
      const uint64_t pm = __ballot(valid && flag == kFlagPrefix);
      if (pm) first_p = q * kWave + __builtin_ctzll(pm);
    }
#pragma unroll
    for (int q = 0; q < kLookWords; ++q) {
      const uint32_t flag = (uint32_t)(w[q] >> 62);
      const bool valid = flag != 0 && (uint32_t)((w[q] >> 32) & kTagMask) == tag;
      missing |= __ballot(!valid && q * kWave + lane <= first_p) != 0;
    }
    if (missing) {                 // a predecessor we need has not published yet
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    uint32_t part = 0;
#pragma unroll
    for (int q = 0; q < kLookWords; ++q) part += (q * kWave + lane <= first_p) ? (uint32_t)w[q] : 0u;
    excl += wave::sum_u32(part);
    if (first_p < kWindow) break;
    pos -= kWindow;
  }
  return excl;
}

// 16-byte global accesses, optionally non-temporal (streaming).
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

}  // namespace scan_detail
}  // namespace desc
