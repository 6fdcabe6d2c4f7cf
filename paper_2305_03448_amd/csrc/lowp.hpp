// lowp.hpp -- the number-format conversions of the low-precision GEMM modes,
// written from the format definitions.
//
// bfloat16: the upper 16 bits of an IEEE binary32, rounded to nearest with
// ties to even on the 16 dropped bits; a NaN keeps its upper payload bits
// with the quiet bit set.  The operand split of the three-product GEMM is
// hi = bf16(a), lo = bf16(a - hi), where a - hi is exact in FP32.  Pairs of
// values are rounded with the hardware conversion, which gives the same bits
// as the definition on all 2^32 inputs.
//
// e4m3 (OCP 8-bit float "E4M3"): sign, 4 exponent bits with bias 7, 3
// mantissa bits, no infinities, S.1111.111 is NaN, so the largest finite
// magnitude is 448; subnormals are m * 2^-9.  Encoding rounds to nearest
// even and saturates magnitudes above 448 (infinities included) to 448.
// e4m3_rne_sat is the encoding written out; e4m3x4 reaches the same codes
// four at a time with the hardware conversion.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace desc {
namespace lowp {

__device__ __forceinline__ uint16_t bf16_rne(float a) {
  const uint32_t u = __float_as_uint(a);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0)
    return (uint16_t)((u >> 16) | 0x0040u);                 // quiet NaN
  const uint32_t upper = u >> 16, lower = u & 0xffffu;
  const uint32_t up = (lower > 0x8000u || (lower == 0x8000u && (upper & 1u))) ? 1u : 0u;
  return (uint16_t)(upper + up);                            // may carry into the exponent
}

// Two values rounded by the gfx950 conversion instruction (round to nearest
// even), a in the low half.
__device__ __forceinline__ uint32_t bf16x2_hw(float a, float b) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// bf16_rne of two values, a in the low half.  The hardware conversion gives
// the same bits as bf16_rne on every one of the 2^32 inputs, NaNs included
// (checked exhaustively on the device), so it is used as is.
__device__ __forceinline__ uint32_t bf16x2_rne(float a, float b) { return bf16x2_hw(a, b); }

// The three-product split of two values: hi = bf16(a), lo = bf16(a - hi),
// each pair packed with a in the low half.
struct Split2 {
  uint32_t hi, lo;
};
__device__ __forceinline__ Split2 split_bf16x2(float a, float b) {
  const uint32_t h = bf16x2_rne(a, b);
  const float ha = __uint_as_float(h << 16), hb = __uint_as_float(h & 0xffff0000u);
  return {h, bf16x2_rne(a - ha, b - hb)};
}

// Four values: the bf16 bit patterns of hi and lo in element order.
typedef uint16_t bf16x4_bits __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_bits __attribute__((ext_vector_type(2)));
struct Split4 {
  bf16x4_bits hi, lo;
};
__device__ __forceinline__ Split4 split_bf16x4(float a, float b, float c, float d) {
  const Split2 p = split_bf16x2(a, b), q = split_bf16x2(c, d);
  const u32x2_bits hi = {p.hi, q.hi}, lo = {p.lo, q.lo};
  return {__builtin_bit_cast(bf16x4_bits, hi), __builtin_bit_cast(bf16x4_bits, lo)};
}

__device__ __forceinline__ uint8_t e4m3_rne_sat(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return (uint8_t)(sign | 0x7fu);      // NaN
  if (a >= 0x43e00000u) return (uint8_t)(sign | 0x7eu);     // |x| >= 448, inf: saturate
  const int e = (int)(a >> 23) - 127;                       // |x| in [2^e, 2^(e+1))
  if (e < -6) {                                             // subnormal range, quantum 2^-9
    const float m = rintf(__uint_as_float(a) * 512.0f);     // exact scaling, ties to even
    return (uint8_t)(sign | (uint32_t)m);                   // m = 8 is the code of 2^-6
  }
  uint32_t q = (a & 0x7fffffu) >> 20;                       // 3 kept mantissa bits
  const uint32_t rest = a & 0xfffffu;                       // 20 dropped bits
  if (rest > 0x80000u || (rest == 0x80000u && (q & 1u))) ++q;
  uint32_t E = (uint32_t)(e + 7);
  if (q == 8u) { q = 0u; ++E; }
  return (uint8_t)(sign | (E << 3) | q);                    // |x| < 448 keeps E.q <= 15.6
}

// Four values at once with the format conversion instruction of gfx950
// (v_cvt_pk_fp8_f32: OCP E4M3, round to nearest even; a, b, c, d land in
// bytes 0..3).  Compared with e4m3_rne_sat over every binary32 input it
// gives the same code for every finite |x| <= 448, and the NaN code instead
// of the saturated one from 464 up, so a group holding a NaN or a magnitude
// above 448 is encoded by e4m3_rne_sat instead.
__device__ __forceinline__ uint32_t e4m3x4(float a, float b, float c, float d) {
  if (fabsf(a) <= 448.0f && fabsf(b) <= 448.0f && fabsf(c) <= 448.0f && fabsf(d) <= 448.0f) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
  }
  return (uint32_t)e4m3_rne_sat(a) | ((uint32_t)e4m3_rne_sat(b) << 8) |
         ((uint32_t)e4m3_rne_sat(c) << 16) | ((uint32_t)e4m3_rne_sat(d) << 24);
}

}  // namespace lowp
}  // namespace desc
