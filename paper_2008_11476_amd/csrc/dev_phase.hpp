// Phase of two gradient pairs at once, in packed 16-bit arithmetic.
//
// Phase (Table 2) maps atan2(gy, gx) in [0, 2 pi) to 256 levels.  The angle
// is reduced to the first octant: with mn = min(|gx|, |gy|) and
// mx = max(|gx|, |gy|), alpha = atan(mn / mx) lies in [0, 32] levels.  alpha
// uses the arctangent approximation
//   atan(z) ~ (pi/4) z + 0.273 z (1 - z)   on [0, 1]
// of S. Rajan, S. Wang, R. Inkol and A. Joyal, "Efficient approximations for
// the arctangent function", IEEE Signal Processing Magazine 23(3), 2006
// (error below 0.0038 rad, 0.16 of a level); in levels that is
// z (c0 - c1 z) with c1 = 0.273 * 128 / pi and c0 = 32 + c1.
//
// Two pixels (the two 16-bit halves of a register) are handled per
// instruction, in half precision:
//  - an integer m < 2048 read as a half is the subnormal m * 2^-24 (exact),
//    so mn needs no conversion and mx one exact multiply, F = mx * 2^-9
//    (half-precision subnormals are kept, the default mode of HIP kernels);
//  - R ~ 64 / F starts from a bit-pattern estimate K - bits(F) and takes one
//    Newton step; with the scalings above, zz = (mn R) (128 - F R) is z / 8;
//  - 8 z (c0 - c1 z) + 1024, written zz (8 c0 - 64 c1 zz) + 1024, is rounded
//    once by the last fused multiply-add to the half grid around 1024
//    (spacing 1), so the low byte of its bit pattern is alpha rounded to a
//    whole level (1024.0 is 0x6400);
//  - the octant (|gy| > |gx|, gx < 0, gy < 0) selects, by a byte permute
//    from two 8-entry tables, whether alpha is negated and which multiple of
//    64 levels is added; negation is xor 0xFF plus one, folded into the added
//    constant.  Only the low byte of each half is meaningful (arithmetic
//    modulo 256 is the wrap of the level circle);
//  - the table index is built from bits 13..15 of gx, gy and |gx| - |gy|:
//    values within [-1024, 1023] repeat their sign in bits 10..15, so
//    bit 15 of gy, bit 14 of gx ^ gy and bit 13 of gx ^ gy ^ d carry the three
//    octant bits in an invertible code, and one 16-bit shift brings them down.
// Over every (gx, gy) in [-1023, 1023]^2 the octant angle is within 0.71 of
// the exact alpha, so the level is within one of round(exact level).  Inputs
// must satisfy |g| <= 1023; larger S16 values are scaled by the caller.
#pragma once
// hipRTC (kernels generated at run time) provides the HIP and integer types itself
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

namespace hvx {

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short w16x2 __attribute__((ext_vector_type(2)));

// byte tables indexed by the code c = p | (s2 ^ s3) << 1 | s3 << 2 with
// p = s1 ^ s2 ^ s3 (s1: |gy| > |gx|, s2: gx < 0, s3: gy < 0)
constexpr uint32_t kPhaseNegLo = 0xFF00FF00u, kPhaseNegHi = 0xFF00FF00u;  // 0xFF: alpha negated
constexpr uint32_t kPhaseAddLo = 0x81404100u, kPhaseAddHi = 0x01C0C180u;  // 64 q (+1 when negated)
// reciprocal estimate 2^6 / F ~ bits^-1(kRcpMagic - bits(F)), in 16-bit wrap-around
constexpr unsigned short kRcpMagic = 0x8F9C;

// The octant angle's two factors for two pixels, from mn = min(|gx|, |gy|)
// and mx = max(|gx|, |gy|) (integers below 1024 in 16-bit halves): zz = z / 8
// and p = 8 c0 - 64 c1 zz, so that zz p is 8 alpha (before rounding).
struct PhaseZP {
  h16x2 zz, p;
};
__device__ __forceinline__ PhaseZP phase_zp(i16x2 mn, i16x2 mx) {
  const h16x2 k32768 = {(_Float16)32768.0f, (_Float16)32768.0f};
  // mx = 0 needs no guard: the estimate for F = 0 is finite, so zz = 0
  const h16x2 F = __builtin_bit_cast(h16x2, mx) * k32768;  // mx 2^-9
  const w16x2 magic = {kRcpMagic, kRcpMagic};
  const h16x2 R = __builtin_bit_cast(h16x2, magic - __builtin_bit_cast(w16x2, F));
  const h16x2 k128 = {(_Float16)128.0f, (_Float16)128.0f};
  const h16x2 E = __builtin_elementwise_fma(-F, R, k128);
  PhaseZP r;
  r.zz = (__builtin_bit_cast(h16x2, mn) * R) * E;
  const h16x2 c0 = {(_Float16)345.0f, (_Float16)345.0f}, c1 = {(_Float16)712.0f, (_Float16)712.0f};
  r.p = __builtin_elementwise_fma(-c1, r.zz, c0);
  return r;
}

// gx, gy: two signed 16-bit gradients each (|g| <= 1023).  Returns the two
// phase levels in the low bytes of the two halves.
__device__ __forceinline__ uint32_t phase_pair(uint32_t gx, uint32_t gy) {
  const i16x2 x = __builtin_bit_cast(i16x2, gx), y = __builtin_bit_cast(i16x2, gy);
  const i16x2 z0 = {0, 0};
  const i16x2 ax = __builtin_elementwise_max(x, z0 - x);
  const i16x2 ay = __builtin_elementwise_max(y, z0 - y);
  const PhaseZP f = phase_zp(__builtin_elementwise_min(ax, ay), __builtin_elementwise_max(ax, ay));
  const h16x2 k1024 = {(_Float16)1024.0f, (_Float16)1024.0f};
  const uint32_t a = __builtin_bit_cast(uint32_t, __builtin_elementwise_fma(f.zz, f.p, k1024));
  const uint32_t d = __builtin_bit_cast(uint32_t, ax - ay);  // sign where |gy| > |gx|
  // t = gy ^ (gx & bits 13,14) ^ (d & bit 13), as two three-input bit operations
  // (truth table 0x78 is s0 ^ (s1 & s2))
  const uint32_t t = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_bitop3_b32(gy, gx, 0x60006000u, 0x78), d,
                                                 0x20002000u, 0x78);
  const uint32_t o = __builtin_bit_cast(uint32_t, __builtin_bit_cast(w16x2, t) >> (unsigned short)13);
  const uint32_t neg = __builtin_amdgcn_perm(kPhaseNegHi, kPhaseNegLo, o);
  const uint32_t add = __builtin_amdgcn_perm(kPhaseAddHi, kPhaseAddLo, o);
  return (a ^ neg) + add;
}

// 64 q by the code o = 4 f + 3 s1 of phase_pair_sm (entries 1, 2, 5, 6 unused)
constexpr uint32_t kPhaseSmAddLo = 0xC0000000u, kPhaseSmAddHi = 0x40000080u;

// phase_pair for gradients in sign-magnitude form: gx and gy are the
// half-precision bit patterns of integers with |g| <= 1023 (the sign in bit
// 15, the magnitude as a subnormal below it), as sums and differences of
// such integers in half precision produce them exactly; ax and ay are gx and
// gy with the sign bits cleared, i.e. |gx| and |gy| as integers.  Returns
// the same levels as phase_pair, each in the low byte of its half.
//  - d = gx - gy as 16-bit integers is |gx| - |gy| plus 2^15 (s2 ^ s3):
//    bits 10..14 hold s1 and bit 15 holds s1 ^ s2 ^ s3, which is whether
//    alpha is negated;
//  - the negation goes into the sign of the polynomial factor, and the last
//    fused multiply-add rounds 1280 +- alpha to the grid of spacing 1
//    (rounding to nearest even treats +x and -x alike around an even base,
//    so the low byte is the negated level exactly);
//  - the multiple q of 64 levels is a function of s1 and one bit of
//    (s2, s3, s1 ^ s2 ^ s3); one three-input bit operation on gx, gy and d
//    puts that bit in bit 15 (truth table 0x72) and s1 in bits 13 and 14,
//    and one shift and one byte permute look q up.
__device__ __forceinline__ uint32_t phase_pair_sm(uint32_t gx, uint32_t gy, uint32_t ax, uint32_t ay) {
  const i16x2 x = __builtin_bit_cast(i16x2, ax), y = __builtin_bit_cast(i16x2, ay);
  const PhaseZP f = phase_zp(__builtin_elementwise_min(x, y), __builtin_elementwise_max(x, y));
  const uint32_t d = __builtin_bit_cast(uint32_t, __builtin_bit_cast(w16x2, gx) - __builtin_bit_cast(w16x2, gy));
  const h16x2 ps = __builtin_bit_cast(
      h16x2, __builtin_amdgcn_bitop3_b32(__builtin_bit_cast(uint32_t, f.p), d, 0x80008000u, 0x78));
  const h16x2 k1280 = {(_Float16)1280.0f, (_Float16)1280.0f};
  const uint32_t a = __builtin_bit_cast(uint32_t, __builtin_elementwise_fma(f.zz, ps, k1280));
  const uint32_t t = __builtin_amdgcn_bitop3_b32(gx, gy, d, 0x72);
  const uint32_t o = __builtin_bit_cast(uint32_t, __builtin_bit_cast(w16x2, t) >> (unsigned short)13);
  return a + __builtin_amdgcn_perm(kPhaseSmAddHi, kPhaseSmAddLo, o);
}

}  // namespace hvx
