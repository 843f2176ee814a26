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
//  - |g| <= 1023 is turned into an exact half by adding the bit pattern of
//    1024.0 and subtracting 1024.0;
//  - 1 / mx starts from the bit-pattern estimate K - bits(mx) and takes one
//    Newton step, folded into z = (mn r)(2 - mx r);
//  - z (c0 - c1 z) + 1024 is rounded once by the last fused multiply-add to
//    the half grid around 1024 (spacing 1), so the low byte of its bit
//    pattern is alpha rounded to a whole level (1024.0 is 0x6400);
//  - the octant (|gy| > |gx|, gx < 0, gy < 0) selects, by a byte permute
//    from two 8-entry tables, whether alpha is negated and which multiple of
//    64 levels is added; negation is xor 0xFF plus one, folded into the added
//    constant.  Only the low byte of each half is meaningful (arithmetic
//    modulo 256 is the wrap of the level circle).
// Over every (gx, gy) in [-1020, 1020]^2 the octant angle is within 0.71 of
// the exact alpha, so the level is within one of round(exact level).  Inputs
// must satisfy |g| <= 1023; larger S16 values are scaled by the caller.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hvx {

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short w16x2 __attribute__((ext_vector_type(2)));

// byte tables indexed by the octant code o = s1 | s2 << 1 | s3 << 2
// (s1: |gy| > |gx|, s2: gx < 0, s3: gy < 0)
constexpr uint32_t kPhaseNegLo = 0x00FFFF00u, kPhaseNegHi = 0xFF0000FFu;  // 0xFF: alpha negated
constexpr uint32_t kPhaseAddLo = 0x40814100u, kPhaseAddHi = 0xC180C001u;  // 64 q (+1 when negated)
constexpr unsigned short kRcpMagic = 0x779C;

// gx, gy: two signed 16-bit gradients each (|g| <= 1023).  Returns the two
// phase levels in the low bytes of the two halves.
__device__ __forceinline__ uint32_t phase_pair(uint32_t gx, uint32_t gy) {
  const i16x2 x = __builtin_bit_cast(i16x2, gx), y = __builtin_bit_cast(i16x2, gy);
  const i16x2 z0 = {0, 0};
  const i16x2 ax = __builtin_elementwise_max(x, z0 - x);
  const i16x2 ay = __builtin_elementwise_max(y, z0 - y);
  const i16x2 mn = __builtin_elementwise_min(ax, ay);
  // mx = 0 needs no guard: the reciprocal estimate of 0 is finite, so z = 0
  const i16x2 mx = __builtin_elementwise_max(ax, ay);
  const w16x2 bias = {0x6400, 0x6400};
  const h16x2 k1024 = {(_Float16)1024.0f, (_Float16)1024.0f};
  const h16x2 fmn = __builtin_bit_cast(h16x2, __builtin_bit_cast(w16x2, mn) + bias) - k1024;
  const h16x2 fmx = __builtin_bit_cast(h16x2, __builtin_bit_cast(w16x2, mx) + bias) - k1024;
  const w16x2 magic = {kRcpMagic, kRcpMagic};
  const h16x2 r = __builtin_bit_cast(h16x2, magic - __builtin_bit_cast(w16x2, fmx));
  const h16x2 two = {(_Float16)2.0f, (_Float16)2.0f};
  const h16x2 e = __builtin_elementwise_fma(-fmx, r, two);
  const h16x2 z = (fmn * r) * e;
  const h16x2 c0 = {(_Float16)43.125f, (_Float16)43.125f}, c1 = {(_Float16)11.125f, (_Float16)11.125f};
  const h16x2 p = __builtin_elementwise_fma(-c1, z, c0);
  const uint32_t a = __builtin_bit_cast(uint32_t, __builtin_elementwise_fma(z, p, k1024));
  const uint32_t d = __builtin_bit_cast(uint32_t, ax - ay);  // sign bit set where |gy| > |gx|
  const uint32_t o = ((d >> 15) & 0x00010001u) | ((gx >> 14) & 0x00020002u) | ((gy >> 13) & 0x00040004u) |
                     0x0C000C00u;
  const uint32_t neg = __builtin_amdgcn_perm(kPhaseNegHi, kPhaseNegLo, o);
  const uint32_t add = __builtin_amdgcn_perm(kPhaseAddHi, kPhaseAddLo, o);
  return (a ^ neg) + add;
}

}  // namespace hvx
