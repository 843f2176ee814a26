// Hand-fused register-streaming kernel bodies for gfx950.
//
// Work decomposition: one wave (64 lanes) owns a vertical strip of the image
// and a band of output rows.  Lane l covers 16 consecutive pixels starting at
// x = strip * 992 + 16 * (l - 1); lanes 1..62 produce output, lanes 0 and 63
// only supply halo pixels to their neighbours.  The wave streams its band top
// to bottom, keeping the few rows each stencil needs in registers, so every
// input byte is read from HBM once and every intermediate stays in VGPRs.
//
// Pixel layout in registers: the 16 pixels of a lane are held as 8 packed
// 16-bit pairs, P[k] = (pixel k) | (pixel k+8) << 16.  With this layout the
// horizontal neighbour of both halves of P[k] is P[k +- 1]; only the pairs at
// the lane ends need pixels of the adjacent lanes, which arrive through DPP
// wave shifts (one VALU move each).  Packed 16-bit arithmetic then handles
// two pixels per instruction for the Gaussian and Sobel stages.
//
// Border semantics are those of node-by-node execution (each local operator
// applies its border mode to its own input, intermediates included): before
// a stencil reads a value array, the positions just outside the image are
// filled with what that operator's border rule says (the nearest in-image
// value of the same array, or the constant).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hvx_desc.h"

namespace hvx {

typedef uint32_t u32;
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32 perm(u32 hi, u32 lo, u32 sel) { return __builtin_amdgcn_perm(hi, lo, sel); }
__device__ __forceinline__ u32 alignbit16(u32 hi, u32 lo) { return __builtin_amdgcn_alignbit(hi, lo, 16); }
// lane i receives lane i-1's value / lane i+1's value (whole-wave shifts)
__device__ __forceinline__ u32 from_left(u32 v) { return __builtin_amdgcn_update_dpp(0u, v, 0x138, 0xF, 0xF, false); }
__device__ __forceinline__ u32 from_right(u32 v) { return __builtin_amdgcn_update_dpp(0u, v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ u32 bfi(u32 mask, u32 a, u32 b) { return (mask & a) | (~mask & b); }

__device__ __forceinline__ u32 add2(u32 a, u32 b) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ u32 sub2(u32 a, u32 b) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ u32 shl2(u32 a, int s) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(u16x2, a) << (unsigned short)s);
}
__device__ __forceinline__ u32 shr2(u32 a, int s) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(u16x2, a) >> (unsigned short)s);
}

// 16 bytes -> 8 pairs (pixel k, pixel k+8)
__device__ __forceinline__ void unpack16(u32x4 r, u32 p[8]) {
  p[0] = perm(r.z, r.x, 0x0c040c00u);
  p[1] = perm(r.z, r.x, 0x0c050c01u);
  p[2] = perm(r.z, r.x, 0x0c060c02u);
  p[3] = perm(r.z, r.x, 0x0c070c03u);
  p[4] = perm(r.w, r.y, 0x0c040c00u);
  p[5] = perm(r.w, r.y, 0x0c050c01u);
  p[6] = perm(r.w, r.y, 0x0c060c02u);
  p[7] = perm(r.w, r.y, 0x0c070c03u);
}

// 8 pairs of byte values -> 16 bytes in pixel order
__device__ __forceinline__ u32x4 pack16(const u32 p[8]) {
  u32 t0 = perm(p[1], p[0], 0x06020400u);  // p0.lo p1.lo p0.hi p1.hi
  u32 t1 = perm(p[3], p[2], 0x06020400u);
  u32 t2 = perm(p[5], p[4], 0x06020400u);
  u32 t3 = perm(p[7], p[6], 0x06020400u);
  u32x4 r;
  r.x = perm(t1, t0, 0x05040100u);
  r.y = perm(t3, t2, 0x05040100u);
  r.z = perm(t1, t0, 0x07060302u);
  r.w = perm(t3, t2, 0x07060302u);
  return r;
}

// Per-lane geometry of a strip work item and its border masks.
struct Lanes {
  int lane, xs;       // lane id, first pixel of the lane
  int xl;             // clamped load column
  bool store;         // lane writes output
  u32 mL;             // 0xFFFF in the lane holding x = 0 (fix pixel -1, -2)
  u32 mR;             // 0xFFFF0000 in the lane whose last pixel is W-1 (W % 16 == 0)
  u32 mRag;           // all ones in the lane holding W-1 when W % 16 != 0
  int m;              // W % 16
  bool edgeL, edgeR;  // wave-uniform: strip touches the left / right border
};

__device__ __forceinline__ Lanes make_lanes(const StripGrid& g, int strip) {
  Lanes L;
  L.lane = threadIdx.x & 63;
  L.xs = strip * kStripPx + (L.lane - 1) * kLanePx;
  const int wr = (g.w + 15) & ~15;
  L.xl = min(max(L.xs, 0), wr - 16);
  L.store = L.lane >= 1 && L.lane <= 62 && L.xs >= 0 && L.xs < g.w;
  L.m = g.w & 15;
  L.mL = L.xs == 0 ? 0x0000FFFFu : 0u;
  L.mR = (L.m == 0 && L.xs + 16 == g.w) ? 0xFFFF0000u : 0u;
  L.mRag = (L.m != 0 && L.xs == g.w - L.m) ? 0xFFFFFFFFu : 0u;
  L.edgeL = strip == 0;
  L.edgeR = strip >= g.nstrips - 2;
  return L;
}

// Extended row: e[0] = pixel pair at offset -2, e[1] at -1, e[2..9] = P, e[10] at +1 past, e[11] +2
struct Ext {
  u32 v[12];
};

// Value of pixel m-1 (the last in-image pixel of the lane holding W-1 when
// W % 16 = m != 0) in both halves.  m is wave-uniform.
__device__ __forceinline__ u32 last_pixel_pair(const u32 p[8], int m) {
  const int pos = m - 1;  // 0..14
  const int k = pos & 7;
  u32 r = p[0];
#pragma unroll
  for (int kk = 1; kk < 8; ++kk)
    if (kk == k) r = p[kk];
  u32 v = pos >= 8 ? (r >> 16) : (r & 0xFFFFu);
  return v | (v << 16);
}

// Build the extended row of a value array before a stencil of radius R (1 or
// 2) reads it.  `repl` selects REPLICATE (else CONSTANT with `cpair` = the
// constant in both halves).  In the lane holding W-1 with W % 16 = m != 0,
// pixels m .. m+R-1 of p are overwritten with the border value.
template <int R>
__device__ __forceinline__ void extend(u32 p[8], Ext& e, const Lanes& L, bool repl, u32 cpair) {
  const bool rag = L.edgeR && L.m != 0;
  u32 fill_rag = cpair;
  if (rag) {
    if (repl) fill_rag = last_pixel_pair(p, L.m);
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int pos = L.m + t;  // 1..16; 16 is handled on the extended row
      if (pos < 16) {
        const u32 hm = pos >= 8 ? 0xFFFF0000u : 0x0000FFFFu;
        const int k = pos & 7;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          if (kk == k) p[kk] = bfi(L.mRag & hm, fill_rag, p[kk]);
      }
    }
  }
  e.v[1] = alignbit16(p[7], from_left(p[7]));
  e.v[10] = alignbit16(from_right(p[0]), p[0]);
  if (R >= 2) {
    e.v[0] = alignbit16(p[6], from_left(p[6]));
    e.v[11] = alignbit16(from_right(p[1]), p[1]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) e.v[k + 2] = p[k];
  if (L.edgeL) {
    const u32 f = repl ? p[0] : cpair;  // low half: pixel 0 or the constant
    e.v[1] = bfi(L.mL, f, e.v[1]);
    if (R >= 2) e.v[0] = bfi(L.mL, f, e.v[0]);
  }
  if (L.edgeR) {
    const u32 f = repl ? p[7] : cpair;  // high half: pixel 15 or the constant
    e.v[10] = bfi(L.mR, f, e.v[10]);
    if (R >= 2) e.v[11] = bfi(L.mR, f, e.v[11]);
    // pixel 16 of the ragged lane is read only when m + R - 1 >= 16
    if (rag && L.m + R - 1 >= 16) e.v[10] = bfi(L.mRag & 0xFFFF0000u, fill_rag, e.v[10]);
  }
}

// ---- Gaussian 3x3 -> Sobel 3x3 -> Magnitude -> Threshold (+ Phase) ----------

// Phase in 1/256 turns from an octant reduction and the arctangent
// approximation atan(z) ~ (pi/4) z + 0.273 z (1 - z) on [0, 1]
// (S. Rajan, S. Wang, R. Inkol, A. Joyal, "Efficient approximations for the
// arctangent function", IEEE Signal Processing Magazine 23(3), 2006), whose
// error is below 0.004 rad (0.16 of one level), so the rounded result is
// within one level of the rounded exact angle.
__device__ __forceinline__ int phase_level(int gx, int gy) {
  const float kA = 0.273f * 128.0f / 3.14159265358979f;
  float ax = fabsf((float)gx), ay = fabsf((float)gy);
  float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
  float z = mn * __builtin_amdgcn_rcpf(fmaxf(mx, 1.0f));
  float a = z * fmaf(-kA, z, 32.0f + kA);
  float t = ay > ax ? 64.0f - a : a;
  t = gx < 0 ? 128.0f - t : t;
  t = gy < 0 ? 256.0f - t : t;
  return ((int)(t + 0.5f)) & 255;
}

template <bool PHASE>
__device__ void edge_item(const EdgeDesc& d, int strip, int band) {
  const StripGrid& g = d.g;
  const Lanes L = make_lanes(g, strip);
  const int W = g.w, H = g.h;
  (void)W;
  const int y0 = band * g.rows;
  const int y1 = min(y0 + g.rows, H);
  const bool repl0 = d.b0 != B_CONSTANT, repl1 = d.b1 != B_CONSTANT;
  const u32 c0 = (u32)d.c0 & 0xFF, c1 = (u32)d.c1 & 0xFFFF;
  const u32 cin = c0 | (c0 << 16);        // input constant
  const u32 cv0 = (4 * c0) | ((4 * c0) << 16);  // vertical (1 2 1) sum of the constant
  const u32 cg = c1 | (c1 << 16);         // Gaussian-output constant
  const u32 cs1 = (4 * c1) | ((4 * c1) << 16);
  const uint8_t* inb = d.in + L.xl;

  auto fetch = [&](int y, u32 p[8]) {
    const int yc = min(max(y, 0), H - 1);
    u32x4 r = __builtin_nontemporal_load((const u32x4*)(inb + (size_t)yc * d.in_pitch));
    unpack16(r, p);
    if (!repl0 && (y < 0 || y >= H)) {
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = cin;
    }
  };
  // G row from input rows a (y-1), b (y), c (y+1)
  auto gauss = [&](const u32 a[8], const u32 b[8], const u32 c[8], u32 out[8]) {
    u32 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = add2(add2(a[k], c[k]), shl2(b[k], 1));
    Ext e;
    extend<1>(v, e, L, repl0, cv0);
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = shr2(add2(add2(e.v[k + 1], e.v[k + 3]), shl2(e.v[k + 2], 1)), 4);
  };

  u32 ia[8], ib[8], ic[8], g0[8], g1[8], g2[8];
  // G(y0 - 1)
  fetch(y0 - 2, ia);
  fetch(y0 - 1, ib);
  fetch(y0, ic);
  if (y0 >= 1) gauss(ia, ib, ic, g0);
  // G(y0)
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    ia[k] = ib[k];
    ib[k] = ic[k];
  }
  fetch(y0 + 1, ic);
  gauss(ia, ib, ic, g1);
  if (y0 == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) g0[k] = repl1 ? g1[k] : cg;
  }
  const int64_t op = d.out_pitch;
  uint8_t* outb = d.out + L.xs;
  for (int y = y0; y < y1; ++y) {
    // G(y + 1)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      ia[k] = ib[k];
      ib[k] = ic[k];
    }
    if (y + 1 < H) {
      fetch(y + 2, ic);
      gauss(ia, ib, ic, g2);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) g2[k] = repl1 ? g1[k] : cg;
    }
    // Sobel on G rows (y-1, y, y+1): vertical (1 2 1) sum and difference first
    u32 sv[8], dv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      sv[k] = add2(add2(g0[k], g2[k]), shl2(g1[k], 1));
      dv[k] = sub2(g2[k], g0[k]);
    }
    Ext es, ed;
    extend<1>(sv, es, L, repl1, cs1);
    extend<1>(dv, ed, L, repl1, 0u);
    u32 gx[8], gy[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      gx[k] = sub2(es.v[k + 3], es.v[k + 1]);
      gy[k] = add2(add2(ed.v[k + 1], ed.v[k + 3]), shl2(ed.v[k + 2], 1));
    }
    // magnitude + threshold as one integer test: gx^2 + gy^2 > T
    int r[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      u32 lo = perm(gy[k], gx[k], 0x05040100u);  // (gx_k, gy_k)
      u32 hi = perm(gy[k], gx[k], 0x07060302u);  // (gx_k+8, gy_k+8)
      r[k] = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, lo), __builtin_bit_cast(s16x2, lo), d.thr_not, false);
      r[k + 8] = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, hi), __builtin_bit_cast(s16x2, hi), d.thr_not, false);
    }
    // sign bytes: 0xFF where r < 0 (no edge)
    u32x4 o;
    u32 q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      u32 lo2 = perm((u32)r[4 * j + 1], (u32)r[4 * j + 0], 0x0c0c0b09u);
      u32 hi2 = perm((u32)r[4 * j + 3], (u32)r[4 * j + 2], 0x0b090c0cu);
      q[j] = bfi(lo2 | hi2, d.fv4, d.tv4);
    }
    o.x = q[0];
    o.y = q[1];
    o.z = q[2];
    o.w = q[3];
    if (L.store) __builtin_nontemporal_store(o, (u32x4*)(outb + (size_t)y * op));
    if (PHASE) {
      u32 ph[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        int lo = phase_level((int)(short)(gx[k] & 0xFFFF), (int)(short)(gy[k] & 0xFFFF));
        int hi = phase_level(((int)gx[k]) >> 16, ((int)gy[k]) >> 16);
        ph[k] = (u32)lo | ((u32)hi << 16);
      }
      u32x4 po = pack16(ph);
      if (L.store) __builtin_nontemporal_store(po, (u32x4*)(d.phase + L.xs + (size_t)y * d.phase_pitch));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      g0[k] = g1[k];
      g1[k] = g2[k];
    }
  }
}

// ---- Gaussian 5x5 (optionally of the luma of a UYVY frame) -----------------

template <bool UYVY>
__device__ void gauss5_item(const Gauss5Desc& d, int strip, int band) {
  const StripGrid& g = d.g;
  const Lanes L = make_lanes(g, strip);
  const int H = g.h;
  const int y0 = band * g.rows;
  const int y1 = min(y0 + g.rows, H);
  const bool repl = d.b0 != B_CONSTANT;
  const u32 c = (u32)d.c0 & 0xFF;
  const u32 cin = c | (c << 16);
  const u32 cv = (16 * c) | ((16 * c) << 16);
  const uint8_t* inb = d.in + (UYVY ? 2 * L.xl : L.xl);

  auto fetch = [&](int y, u32 p[8]) {
    const int yc = min(max(y, 0), H - 1);
    const uint8_t* row = inb + (size_t)yc * d.in_pitch;
    if (UYVY) {
      // 32 bytes U Y V Y ...: luma bytes are the odd ones
      u32x4 a = __builtin_nontemporal_load((const u32x4*)row);
      u32x4 b = __builtin_nontemporal_load((const u32x4*)(row + 16));
      // pixel k (k < 8) lives in a, pixel k+8 in b; luma of pixel k is byte 2k+1
      p[0] = perm(b.x, a.x, 0x0c050c01u);
      p[1] = perm(b.x, a.x, 0x0c070c03u);
      p[2] = perm(b.y, a.y, 0x0c050c01u);
      p[3] = perm(b.y, a.y, 0x0c070c03u);
      p[4] = perm(b.z, a.z, 0x0c050c01u);
      p[5] = perm(b.z, a.z, 0x0c070c03u);
      p[6] = perm(b.w, a.w, 0x0c050c01u);
      p[7] = perm(b.w, a.w, 0x0c070c03u);
    } else {
      unpack16(__builtin_nontemporal_load((const u32x4*)row), p);
    }
    if (!repl && (y < 0 || y >= H)) {
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = cin;
    }
  };

  u32 r0[8], r1[8], r2[8], r3[8], r4[8];
  fetch(y0 - 2, r0);
  fetch(y0 - 1, r1);
  fetch(y0, r2);
  fetch(y0 + 1, r3);
  uint8_t* outb = d.out + L.xs;
  for (int y = y0; y < y1; ++y) {
    fetch(y + 2, r4);
    // vertical (1 4 6 4 1): max 16*255 = 4080 per column
    u32 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      u32 a = add2(r0[k], r4[k]);
      u32 b = add2(r1[k], r3[k]);
      v[k] = add2(add2(a, shl2(b, 2)), add2(shl2(r2[k], 2), shl2(r2[k], 1)));
    }
    Ext e;
    extend<2>(v, e, L, repl, cv);
    u32 o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      // horizontal (1 4 6 4 1): max 65280, fits 16 bits
      u32 a = add2(e.v[k], e.v[k + 4]);
      u32 b = add2(e.v[k + 1], e.v[k + 3]);
      u32 s = add2(add2(a, shl2(b, 2)), add2(shl2(e.v[k + 2], 2), shl2(e.v[k + 2], 1)));
      o[k] = shr2(s, 8);
    }
    if (L.store) __builtin_nontemporal_store(pack16(o), (u32x4*)(outb + (size_t)y * d.out_pitch));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      r0[k] = r1[k];
      r1[k] = r2[k];
      r2[k] = r3[k];
      r3[k] = r4[k];
    }
  }
}

}  // namespace hvx
