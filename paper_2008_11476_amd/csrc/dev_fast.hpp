// Hand-fused register-streaming kernel bodies for gfx950.
//
// Work decomposition: one wave (64 lanes) owns a vertical strip of the image
// and a band of output rows.  Lane l covers 16 consecutive pixels starting at
// x = strip * 960 + 16 * (l - 1); lanes 1..60 produce output, lanes 0 and 61
// only supply halo pixels to their neighbours (lanes 62 and 63 idle).  The
// wave streams its band top to bottom, keeping the few rows each stencil
// needs in registers, so every input byte is read from HBM once and every
// intermediate stays in VGPRs.
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

#include "dev_phase.hpp"
#include "hvx_desc.h"

namespace hvx {

typedef uint32_t u32;
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32 perm(u32 hi, u32 lo, u32 sel) { return __builtin_amdgcn_perm(hi, lo, sel); }

// Images are in global memory (address space 1): global rather than flat
// instructions.
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

// The start of a row is the same in every lane.  Reading it back through
// readfirstlane keeps the row arithmetic on the scalar unit; with the lane's
// 32-bit byte offset redefined in the same block (keep_vgpr, an empty asm),
// the access takes the scalar-base global form and costs no vector address
// arithmetic.
__device__ __forceinline__ uintptr_t uniform_addr(uintptr_t a) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  return ((uintptr_t)hi << 32) | lo;
}
__device__ __forceinline__ void keep_vgpr(u32& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void store_row16_uniform(uint8_t* base, int64_t pitch, int y, u32 off, u32x4 v) {
  const uintptr_t row = uniform_addr((uintptr_t)base + (uintptr_t)((int64_t)y * pitch));
  __builtin_nontemporal_store(v, (g_u32x4*)(row + off));
}

__device__ __forceinline__ u32 alignbit16(u32 hi, u32 lo) { return __builtin_amdgcn_alignbit(hi, lo, 16); }
// lane i receives lane i-1's value / lane i+1's value (whole-wave shifts; the lane
// without a source reads 0, which only halo lanes ever see)
__device__ __forceinline__ u32 from_left(u32 v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ u32 from_right(u32 v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
// The same shifts kept as separate v_mov_b32_dpp instructions (the empty asm
// stops the compiler from folding them into the consuming add or subtract).
// Folded into v_add_u32_dpp / v_subrev_u32_dpp with wave_shr:1, they gave
// wrong corner-kernel results on gfx950 in every lane.
__device__ __forceinline__ u32 from_left_mov(u32 v) {
  u32 r = from_left(v);
  asm("" : "+v"(r));
  return r;
}
__device__ __forceinline__ u32 from_right_mov(u32 v) {
  u32 r = from_right(v);
  asm("" : "+v"(r));
  return r;
}
__device__ __forceinline__ u32 bfi(u32 mask, u32 a, u32 b) { return (mask & a) | (~mask & b); }

__device__ __forceinline__ u32 add2(u32 a, u32 b) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ u32 sub2(u32 a, u32 b) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
// sums and differences of integers below 1024 held as half-precision bit
// patterns (subnormals, exact; a difference of equal values is +0)
__device__ __forceinline__ u32 hadd2(u32 a, u32 b) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(h16x2, a) + __builtin_bit_cast(h16x2, b));
}
__device__ __forceinline__ u32 hsub2(u32 a, u32 b) {
  return __builtin_bit_cast(u32, __builtin_bit_cast(h16x2, a) - __builtin_bit_cast(h16x2, b));
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
  L.store = L.lane >= 1 && L.lane <= kOutLanes && L.xs >= 0 && L.xs < g.w;
  L.m = g.w & 15;
  L.mL = L.xs == 0 ? 0x0000FFFFu : 0u;
  L.mR = (L.m == 0 && L.xs + 16 == g.w) ? 0xFFFF0000u : 0u;
  L.mRag = (L.m != 0 && L.xs == g.w - L.m) ? 0xFFFFFFFFu : 0u;
  L.edgeL = strip == 0;
  // some lane of the strip (halo lanes included) holds W-1 or W
  L.edgeR = g.w <= (strip + 1) * kStripPx + kLanePx;
  return L;
}

// Extended row: e[0] = pixel pair at offset -2, e[1] at -1, e[2..9] = P, e[10] at +1 past, e[11] +2
struct Ext {
  u32 v[12];
};

// Value of pixel m-1 (the last in-image pixel of the lane holding W-1 when
// W % 16 = m != 0) in both halves; m is wave-uniform.
__device__ __forceinline__ u32 last_pixel_pair(const u32 p[8], int m) {
  // an explicit switch: a select chain over p[] would be turned into a
  // dynamically indexed (scratch) access
  u32 v;
  switch (m - 1) {
    case 0: v = p[0] & 0xFFFFu; break;
    case 1: v = p[1] & 0xFFFFu; break;
    case 2: v = p[2] & 0xFFFFu; break;
    case 3: v = p[3] & 0xFFFFu; break;
    case 4: v = p[4] & 0xFFFFu; break;
    case 5: v = p[5] & 0xFFFFu; break;
    case 6: v = p[6] & 0xFFFFu; break;
    case 7: v = p[7] & 0xFFFFu; break;
    case 8: v = p[0] >> 16; break;
    case 9: v = p[1] >> 16; break;
    case 10: v = p[2] >> 16; break;
    case 11: v = p[3] >> 16; break;
    case 12: v = p[4] >> 16; break;
    case 13: v = p[5] >> 16; break;
    default: v = p[6] >> 16; break;
  }
  return v | (v << 16);
}

// Build the extended row of a value array before a stencil of radius R (1 or
// 2) reads it.  HEDGE: the strip touches the left or right image border, so
// the pixels just outside the image are replaced by the border value
// (`repl`: the nearest in-image value of the same array, else `cpair`, the
// constant in both halves).  In the lane holding W-1 with W % 16 = m != 0,
// pixels m .. m+R-1 of p are overwritten in place.
template <int R, bool HEDGE>
__device__ __forceinline__ void extend(u32 p[8], Ext& e, const Lanes& L, bool repl, u32 cpair) {
  u32 fill_rag = cpair;
  if (HEDGE && L.m != 0) {
    if (repl) fill_rag = last_pixel_pair(p, L.m);
    // per register k: halves at positions m .. m+R-1 of the ragged lane
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      u32 hm = 0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int pos = L.m + t;
        hm |= (pos == k) ? 0x0000FFFFu : 0u;
        hm |= (pos == k + 8) ? 0xFFFF0000u : 0u;
      }
      p[k] = bfi(L.mRag & hm, fill_rag, p[k]);
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
  if (HEDGE) {
    const u32 fl = repl ? p[0] : cpair;  // low half: pixel 0 or the constant
    e.v[1] = bfi(L.mL, fl, e.v[1]);
    if (R >= 2) e.v[0] = bfi(L.mL, fl, e.v[0]);
    const u32 fr = repl ? p[7] : cpair;  // high half: pixel 15 or the constant
    // pixel 16 (and 17) beyond a lane ending at W, or of the ragged lane when m + R - 1 >= 16
    const u32 m16 = L.mR | ((L.m + R - 1 >= 16) ? (L.mRag & 0xFFFF0000u) : 0u);
    const u32 f16 = L.mR ? fr : fill_rag;
    e.v[10] = bfi(m16, f16, e.v[10]);
    if (R >= 2) e.v[11] = bfi(L.mR, fr, e.v[11]);
  }
}

// ---- input row queue in LDS -------------------------------------------------
// The row streams read input row y+2 at output row y.  Rows travel through a
// queue of Q rows in the wave's LDS (NB x 16 bytes per lane and row), filled
// by direct-to-LDS loads Q rows ahead, so the prefetch holds no registers.
// The compiler does not track these loads against the LDS reads, so the
// waits are explicit.  The vector-memory counter drains in issue order,
// stores included; a row is complete once no more operations are
// outstanding than were issued after its last load:
//  - the loads of rows y+3 .. y+Q+1 (NB each), except those past the band's
//    last input row y1+1, which are never issued;
//  - the stores (S per output row) of the rows y0 .. y-1 issued after it,
//    at most Q rows' worth.
// The count is rounded down to one of four immediates.
template <int N>
__device__ __forceinline__ void wait_vmem() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

template <int NB, int S, int Q>
struct LdsRows {
  static_assert(Q >= 4 && (Q & (Q - 1)) == 0, "queue of a power of two rows, at least 4");
  static constexpr int kLds = Q * 64 * NB;  // 16-byte entries
  u32x4* q;  // row r in slot (r - qbase) mod Q
  const uint8_t* base;
  int64_t pitch;
  u32 lin;  // lane byte offset
  int H, lane, qbase, y0, y1;
  // the image row of stream row r is ab + ad r (ad = -1: a band streamed
  // bottom-up, its rows reflected within the band)
  int ab = 0, ad = 1;

  // direct-to-LDS load of input row r (clamped to the image) into its slot
  __device__ __forceinline__ void issue(int r) const {
    const int rc = min(max(ab + ad * r, 0), H - 1);
    const uintptr_t row = uniform_addr((uintptr_t)base + (uintptr_t)((int64_t)rc * pitch));
    u32x4* slot = q + ((r - qbase) & (Q - 1)) * (64 * NB);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      __builtin_amdgcn_global_load_lds((const void*)(row + lin + 16 * b),
                                       (__attribute__((address_space(3))) void*)(slot + 64 * b), 16, 0, 0);
  }
  // row r from its slot; the read completes before the slot is refilled
  __device__ __forceinline__ void read(int r, u32x4 v[NB]) const {
    const u32x4* slot = q + ((r - qbase) & (Q - 1)) * (64 * NB) + lane;
#pragma unroll
    for (int b = 0; b < NB; ++b) v[b] = slot[64 * b];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  }
  // band [b0, b1): load input rows b0-2 .. b0+Q-3, wait for the first four
  __device__ __forceinline__ void start(int b0, int b1) {
    qbase = b0 - 2;
    y0 = b0;
    y1 = b1;
#pragma unroll
    for (int k = 0; k < Q; ++k) issue(b0 - 2 + k);
    wait_vmem<NB*(Q - 4)>();
  }
  // after the first four rows are read: rows b0+Q-2 .. b0+Q+1 into their slots
  __device__ __forceinline__ void refill() const {
#pragma unroll
    for (int k = 0; k < 4; ++k) issue(y0 + Q - 2 + k);
  }
  // at output row y: wait for row y+2, read it, queue row y+Q+2
  __device__ __forceinline__ void take(int y, u32x4 v[NB]) {
    keep_vgpr(lin);
    constexpr int F = Q * S + (Q - 1) * NB;
    constexpr int A = Q * S, B = (Q - 1) * NB;
    constexpr int X = A > B ? A : B, Y = A > B ? B : A;
    const int n = min(y - y0, Q) * S + NB * (Q - 1 - min(max(y + Q - y1, 0), Q - 1));
    if (n >= F) wait_vmem<F>();
    else if (n >= X) wait_vmem<X>();
    else if (n >= Y) wait_vmem<Y>();
    else wait_vmem<0>();
    read(y + 2, v);
    if (y + Q + 2 <= y1 + 1) issue(y + Q + 2);
  }
};

// queue depths (rows).  The Gaussian5x5 streams run few rows per band, so
// their queues are deeper; eight UYVY rows (16 KB per wave) leave room for
// 10 waves per CU, which measured faster than 16 waves with four rows.
constexpr int kEdgeQ = 4, kGauss5Q = 8, kUyvyQ = 8;

// ---- Gaussian 3x3 -> Sobel 3x3 -> Magnitude -> Threshold (+ Phase) ----------

// One wave streams its band: at output row y it finishes Gaussian row y+1 and
// Sobel/magnitude/threshold row y.  All (1 2 1) sums are formed from pairwise
// sums shared between neighbouring rows or pixels (a + 2b + c = (a+b) + (b+c)).
// The loop is unrolled by six so that every rotating row buffer (periods two
// and three) is renamed statically.  Input rows arrive through an LdsRows
// queue.
// WIDE selects the 32-bit magnitude test; otherwise the bound fits the
// saturating 16-bit test (thr_not >= -32768).
// A band can stream bottom-up: stream row u is image row ab + ad u with
// ad = -1, i.e. the band reflected within itself.  The vertical filters are
// then applied upwards, which flips the sign of gy and nothing else, so only
// the magnitude (gy squared) may use it.  Neighbouring bands that stream in
// opposite directions read the rows they share at about the same time (both
// at their start or both at their end), so the second read hits L2.
template <bool PHASE, bool HEDGE, bool WIDE>
struct EdgeStream {
  const EdgeDesc& d;
  Lanes L;
  int H;
  bool repl0, repl1;
  u32 cin, cv0, cg, cs1;
  // image bases and pitches copied out of the descriptor (wave-uniform, so
  // row addresses are scalar arithmetic) and the lane's byte offsets
  const uint8_t* in0;
  uint8_t* out0;
  uint8_t* ph0;
  int64_t ip, op, pp;
  u32 lin, lout;
  int thr;
  u32 thr2;  // thr_not in both halves (16-bit test)
  u32 tv4, x4;
  // rotating state
  u32 inr[2][8];  // input row y+1 (role alternates)
  u32 tr[2][8];   // in(y) + in(y+1)
  u32 gr[3][8];   // Gaussian rows y-1, y, y+1
  u32 sr[2][8];   // G(y-1) + G(y)
  LdsRows<1, PHASE ? 2 : 1, kEdgeQ> rows;  // input rows (one 16-byte load per row; 1 or 2 stores)
  int ab = 0, ad = 1;                      // image row of stream row u: ab + ad u
  __device__ __forceinline__ int act(int u) const { return ab + ad * u; }

  __device__ __forceinline__ EdgeStream(const EdgeDesc& d_, int strip, u32x4* lds) : d(d_) {
    L = make_lanes(d.g, strip);
    H = d.g.h;
    repl0 = d.b0 != B_CONSTANT;
    repl1 = d.b1 != B_CONSTANT;
    const u32 c0 = (u32)d.c0 & 0xFF, c1 = (u32)d.c1 & 0xFF;
    cin = c0 | (c0 << 16);
    cv0 = (4 * c0) | ((4 * c0) << 16);
    cg = c1 | (c1 << 16);
    cs1 = (4 * c1) | ((4 * c1) << 16);
    in0 = d.in;
    out0 = d.out;
    ph0 = PHASE ? d.phase : nullptr;
    ip = d.in_pitch;
    op = d.out_pitch;
    pp = PHASE ? d.phase_pitch : 0;
    lin = (u32)L.xl;
    lout = (u32)L.xs;  // wraps for the left halo lane, which never stores
    thr = d.thr_not;
    thr2 = ((u32)d.thr_not & 0xFFFFu) * 0x10001u;
    tv4 = d.tv4;
    x4 = d.tv4 ^ d.fv4;
    rows.q = lds;
    rows.base = in0;
    rows.pitch = ip;
    rows.lin = lin;
    rows.H = H;
    rows.lane = L.lane;
  }
  __device__ __forceinline__ void unpk(u32x4 r, int y, u32 p[8]) const {
    unpack16(r, p);
    const int ya = act(y);
    if (!repl0 && (ya < 0 || ya >= H)) {
      // a rare, wave-uniform case: the empty asm keeps it a branch (the
      // compiler would otherwise select all eight registers on every row)
      asm volatile("");
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = cin;
    }
  }
  // Gaussian row from the vertical (1 2 1) sums v of its three input rows
  __device__ __forceinline__ void gauss_h(u32 v[8], u32 g[8]) const {
    Ext e;
    extend<1, HEDGE>(v, e, L, repl0, cv0);
    u32 u[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) u[i] = add2(e.v[i + 1], e.v[i + 2]);
#pragma unroll
    for (int k = 0; k < 8; ++k) g[k] = shr2(add2(u[k], u[k + 1]), 4);
  }
  __device__ __forceinline__ void emit(int y, u32 sv[8], u32 dv[8]) {
    Ext es, ed;
    extend<1, HEDGE>(sv, es, L, repl1, cs1);
    extend<1, HEDGE>(dv, ed, L, repl1, 0u);
    u32 gx[8], gy[8], eu[9];
    // With the phase, the gradients are formed in half precision (dv is
    // already): sums of integers below 1024 as subnormals are exact, and the
    // sign-magnitude results give |gx| and |gy| by clearing one bit each,
    // for the phase and the magnitude alike.
#pragma unroll
    for (int i = 0; i < 9; ++i) eu[i] = PHASE ? hadd2(ed.v[i + 1], ed.v[i + 2]) : add2(ed.v[i + 1], ed.v[i + 2]);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      gx[k] = PHASE ? hsub2(es.v[k + 3], es.v[k + 1]) : sub2(es.v[k + 3], es.v[k + 1]);
      gy[k] = PHASE ? hadd2(eu[k], eu[k + 1]) : add2(eu[k], eu[k + 1]);
    }
    if (PHASE) {
      // levels of pixels k and k+8 in the low bytes of lv[k]'s halves; output
      // word j holds pixels 4j .. 4j+3
      u32 lv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const u32 ax = gx[k] & 0x7FFF7FFFu, ay = gy[k] & 0x7FFF7FFFu;
        lv[k] = phase_pair_sm(gx[k], gy[k], ax, ay);
        gx[k] = ax;
        gy[k] = ay;
      }
      u32x4 po;
      const u32 a01 = perm(lv[1], lv[0], 0x06020400u), a23 = perm(lv[3], lv[2], 0x06020400u);
      const u32 a45 = perm(lv[5], lv[4], 0x06020400u), a67 = perm(lv[7], lv[6], 0x06020400u);
      po.x = perm(a23, a01, 0x05040100u);
      po.y = perm(a67, a45, 0x05040100u);
      po.z = perm(a23, a01, 0x07060302u);
      po.w = perm(a67, a45, 0x07060302u);
      if (L.store) store_row16_uniform(ph0, pp, act(y), lout, po);
    }
    // magnitude + threshold as one integer test: gx^2 + gy^2 > T, i.e. the
    // sign of gx^2 + gy^2 + thr_not (thr_not = -T - 1); mask bytes are 0xFF
    // where that sum is negative (no edge), and out = tv ^ (mask & (tv ^ fv))
    // picks fv there and tv elsewhere.
    u32x4 o;
    if (!WIDE) {
      // v_pk_mad_i16 with clamp forms each full product and sum before it
      // saturates to 16 bits.  gx^2 + thr_not cannot saturate low
      // (thr_not >= -32768), and a saturated value keeps its sign, so bit
      // 15 of each half of m is the sign of the exact sum.
      u32 m[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        u32 t;
        asm("v_pk_mad_i16 %0, %1, %1, %2 clamp" : "=v"(t) : "v"(gx[k]), "s"(thr2));
        asm("v_pk_mad_i16 %0, %1, %1, %2 clamp" : "=v"(m[k]) : "v"(gy[k]), "v"(t));
      }
      // byte permute selectors 8..11 replicate bit 15 / 31 of the sources:
      // a01 = masks of pixels 0, 1, 8, 9
      const u32 a01 = perm(m[1], m[0], 0x0B090A08u), a23 = perm(m[3], m[2], 0x0B090A08u);
      const u32 a45 = perm(m[5], m[4], 0x0B090A08u), a67 = perm(m[7], m[6], 0x0B090A08u);
      o.x = tv4 ^ (perm(a23, a01, 0x05040100u) & x4);
      o.y = tv4 ^ (perm(a67, a45, 0x05040100u) & x4);
      o.z = tv4 ^ (perm(a23, a01, 0x07060302u) & x4);
      o.w = tv4 ^ (perm(a67, a45, 0x07060302u) & x4);
    } else {
      // v_mad_i32_i16 multiplies the selected signed 16-bit halves of its
      // sources into a 32-bit sum (op_sel picks the high halves), so each
      // pixel takes two instructions and no repacking.
      u32 r[16];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        int t0, t1, r0, r1;
        asm("v_mad_i32_i16 %0, %1, %1, %2" : "=v"(t0) : "v"(gx[k]), "s"(thr));
        asm("v_mad_i32_i16 %0, %1, %1, %2" : "=v"(r0) : "v"(gy[k]), "v"(t0));
        asm("v_mad_i32_i16 %0, %1, %1, %2 op_sel:[1,1,0,0]" : "=v"(t1) : "v"(gx[k]), "s"(thr));
        asm("v_mad_i32_i16 %0, %1, %1, %2 op_sel:[1,1,0,0]" : "=v"(r1) : "v"(gy[k]), "v"(t1));
        r[k] = (u32)r0;
        r[k + 8] = (u32)r1;
      }
      o.x = tv4 ^ ((perm(r[1], r[0], 0x0c0c0b09u) | perm(r[3], r[2], 0x0b090c0cu)) & x4);
      o.y = tv4 ^ ((perm(r[5], r[4], 0x0c0c0b09u) | perm(r[7], r[6], 0x0b090c0cu)) & x4);
      o.z = tv4 ^ ((perm(r[9], r[8], 0x0c0c0b09u) | perm(r[11], r[10], 0x0b090c0cu)) & x4);
      o.w = tv4 ^ ((perm(r[13], r[12], 0x0c0c0b09u) | perm(r[15], r[14], 0x0b090c0cu)) & x4);
    }
    if (L.store) store_row16_uniform(out0, op, act(y), lout, o);
  }
  // Output row y; J is the phase of y in the six-row unrolled sequence.
  template <int J>
  __device__ __forceinline__ void step(int y) {
    u32(&in1)[8] = inr[J % 2];
    u32(&in2)[8] = inr[(J + 1) % 2];
    u32(&t0)[8] = tr[J % 2];
    u32(&t1)[8] = tr[(J + 1) % 2];
    u32(&gm1)[8] = gr[J % 3];
    u32(&g0)[8] = gr[(J + 1) % 3];
    u32(&g1)[8] = gr[(J + 2) % 3];
    u32(&s0)[8] = sr[J % 2];
    u32(&s1)[8] = sr[(J + 1) % 2];
    u32x4 cur;
    rows.take(y, &cur);
    keep_vgpr(lout);
    const int ga = act(y + 1);  // image row of Gaussian row y+1 (past the band's end)
    if (ad > 0 ? ga < H : ga >= 0) {
      unpk(cur, y + 2, in2);
      u32 v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        t1[k] = add2(in1[k], in2[k]);
        v[k] = add2(t0[k], t1[k]);
      }
      gauss_h(v, g1);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) g1[k] = repl1 ? g0[k] : cg;
    }
    u32 sv[8], dv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      s1[k] = add2(g0[k], g1[k]);
      sv[k] = add2(s0[k], s1[k]);
      dv[k] = PHASE ? hsub2(g1[k], gm1[k]) : sub2(g1[k], gm1[k]);
    }
    emit(y, sv, dv);
  }
  // Output rows [y0, y1), top to bottom, or bottom to top when `up` (which
  // only the magnitude may use: gy changes sign).
  __device__ __forceinline__ void run(int y0, int y1, bool up = false) {
    ab = up ? y0 + y1 - 1 : 0;
    ad = up ? -1 : 1;
    rows.ab = ab;
    rows.ad = ad;
    // prologue: G(y0-1), G(y0) and the pairwise state for row y0
    rows.start(y0, y1);
    u32 a[8], b[8], c[8], e[8];
    u32x4 t;
    rows.read(y0 - 2, &t);
    unpk(t, y0 - 2, a);
    rows.read(y0 - 1, &t);
    unpk(t, y0 - 1, b);
    rows.read(y0, &t);
    unpk(t, y0, c);
    rows.read(y0 + 1, &t);
    unpk(t, y0 + 1, e);
    rows.refill();
    u32 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = add2(add2(b[k], c[k]), add2(c[k], e[k]));
    gauss_h(v, gr[1]);  // G(y0)
    const int pa = act(y0 - 1);  // image row of Gaussian row y0-1 (before the band's start)
    if (ad > 0 ? pa >= 0 : pa < H) {
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = add2(add2(a[k], b[k]), add2(b[k], c[k]));
      gauss_h(v, gr[0]);  // G(y0-1)
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) gr[0][k] = repl1 ? gr[1][k] : cg;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      inr[0][k] = e[k];
      tr[0][k] = add2(c[k], e[k]);
      sr[0][k] = add2(gr[0][k], gr[1][k]);
    }
    // counted loop over the band's rows (measured faster than a loop on y)
    const int n = y1 - y0;
    for (int i = 0; i < n; i += 6) {
      const int y = y0 + i;
      step<0>(y);
      if (i + 1 >= n) break;
      step<1>(y + 1);
      if (i + 2 >= n) break;
      step<2>(y + 2);
      if (i + 3 >= n) break;
      step<3>(y + 3);
      if (i + 4 >= n) break;
      step<4>(y + 4);
      if (i + 5 >= n) break;
      step<5>(y + 5);
    }
  }
};

// LDS the item functions need, in 16-byte units (the kernels provide one
// buffer of the largest size among the kinds they run)
constexpr int kEdgeLds = kEdgeQ * 64;

template <bool PHASE>
__device__ __forceinline__ void edge_item(const EdgeDesc& d, int strip, int band, u32x4* lds) {
  const int y0 = band * d.g.rows;
  const int y1 = min(y0 + d.g.rows, d.g.h);
  // without the phase, odd bands stream bottom-up
  const bool up = !PHASE && (band & 1);
  if (d.thr_not < -32768) {
    // bounds above 32767 (thresholds of 181 and more): the 32-bit test, with
    // the border-aware stream on every strip
    EdgeStream<PHASE, true, true> s(d, strip, lds);
    s.run(y0, y1, up);
  } else if (strip == 0 || d.g.w <= (strip + 1) * kStripPx + kLanePx) {
    EdgeStream<PHASE, true, false> s(d, strip, lds);
    s.run(y0, y1, up);
  } else {
    EdgeStream<PHASE, false, false> s(d, strip, lds);
    s.run(y0, y1, up);
  }
  // no load into the queue may still be in flight when the wave moves on
  wait_vmem<0>();
}

// ---- Gaussian 5x5 (optionally of the luma of a UYVY frame) -----------------
// (1 4 6 4 1) = (1 1) applied four times: vertically each level keeps one
// pairwise sum per row (four packed adds per pixel pair per row);
// horizontally the four levels run over the extended row.
template <bool UYVY, bool HEDGE>
struct G5Stream {
  const Gauss5Desc& d;
  Lanes L;
  int H;
  bool repl;
  u32 cin, cv;
  // wave-uniform bases and pitches, lane byte offsets
  const uint8_t* in0;
  uint8_t* out0;
  int64_t ip, op;
  u32 lin, lout;
  u32 rr[2][8];  // last input row
  u32 p1[2][8];  // level-1 vertical sums (rows y, y+1) ...
  u32 p2[2][8];
  u32 p3[2][8];
  LdsRows<UYVY ? 2 : 1, 1, UYVY ? kUyvyQ : kGauss5Q> rows;  // input rows (UYVY: 32 bytes per lane)

  __device__ __forceinline__ G5Stream(const Gauss5Desc& d_, int strip, u32x4* lds) : d(d_) {
    L = make_lanes(d.g, strip);
    H = d.g.h;
    repl = d.b0 != B_CONSTANT;
    const u32 c = (u32)d.c0 & 0xFF;
    cin = c | (c << 16);
    cv = (16 * c) | ((16 * c) << 16);
    in0 = d.in;
    out0 = d.out;
    ip = d.in_pitch;
    op = d.out_pitch;
    lin = (u32)(UYVY ? 2 * L.xl : L.xl);
    lout = (u32)L.xs;  // wraps for the left halo lane, which never stores
    rows.q = lds;
    rows.base = in0;
    rows.pitch = ip;
    rows.lin = lin;
    rows.H = H;
    rows.lane = L.lane;
  }
  __device__ __forceinline__ void unpk(const u32x4 r[2], int y, u32 p[8]) const {
    if (UYVY) {
      // pixel k (k < 8) is in the first 16 bytes, pixel k+8 in the next; luma is byte 2k+1
      const u32x4 a = r[0], b = r[1];
      p[0] = perm(b.x, a.x, 0x0c050c01u);
      p[1] = perm(b.x, a.x, 0x0c070c03u);
      p[2] = perm(b.y, a.y, 0x0c050c01u);
      p[3] = perm(b.y, a.y, 0x0c070c03u);
      p[4] = perm(b.z, a.z, 0x0c050c01u);
      p[5] = perm(b.z, a.z, 0x0c070c03u);
      p[6] = perm(b.w, a.w, 0x0c050c01u);
      p[7] = perm(b.w, a.w, 0x0c070c03u);
    } else {
      unpack16(r[0], p);
    }
    if (!repl && (y < 0 || y >= H)) {
      asm volatile("");  // keep the rare case a branch (see EdgeStream::unpk)
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = cin;
    }
  }
  __device__ __forceinline__ void horiz_store(int y, u32 v[8]) {
    Ext e;
    extend<2, HEDGE>(v, e, L, repl, cv);
    u32 a[11], b[10], c[9];
#pragma unroll
    for (int i = 0; i < 11; ++i) a[i] = add2(e.v[i], e.v[i + 1]);
#pragma unroll
    for (int i = 0; i < 10; ++i) b[i] = add2(a[i], a[i + 1]);
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = add2(b[i], b[i + 1]);
    u32 o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = shr2(add2(c[k], c[k + 1]), 8);
    if (L.store) store_row16_uniform(out0, op, y, lout, pack16(o));
  }
  // output row y: the new input row is y+2
  template <int J>
  __device__ __forceinline__ void step(int y) {
    u32(&r0)[8] = rr[J % 2];
    u32(&r1)[8] = rr[(J + 1) % 2];
    u32(&a0)[8] = p1[J % 2];
    u32(&a1)[8] = p1[(J + 1) % 2];
    u32(&b0)[8] = p2[J % 2];
    u32(&b1)[8] = p2[(J + 1) % 2];
    u32(&c0)[8] = p3[J % 2];
    u32(&c1)[8] = p3[(J + 1) % 2];
    u32x4 cur[2];
    rows.take(y, cur);
    keep_vgpr(lout);
    unpk(cur, y + 2, r1);
    u32 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a1[k] = add2(r0[k], r1[k]);  // rows y+1, y+2
      b1[k] = add2(a0[k], a1[k]);  // rows y .. y+2
      c1[k] = add2(b0[k], b1[k]);  // rows y-1 .. y+2
      v[k] = add2(c0[k], c1[k]);   // rows y-2 .. y+2
    }
    horiz_store(y, v);
  }
  __device__ __forceinline__ void run(int y0, int y1) {
    u32 q[4][8];
    u32x4 t[2];
    rows.start(y0, y1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rows.read(y0 - 2 + j, t);
      unpk(t, y0 - 2 + j, q[j]);
    }
    rows.refill();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const u32 s01 = add2(q[0][k], q[1][k]), s12 = add2(q[1][k], q[2][k]), s23 = add2(q[2][k], q[3][k]);
      rr[0][k] = q[3][k];
      p1[0][k] = s23;                        // rows y0, y0+1
      p2[0][k] = add2(s12, s23);             // rows y0-1 .. y0+1
      p3[0][k] = add2(add2(s01, s12), p2[0][k]);  // rows y0-2 .. y0+1
    }
    for (int y = y0; y < y1; y += 6) {
      step<0>(y);
      if (y + 1 >= y1) break;
      step<1>(y + 1);
      if (y + 2 >= y1) break;
      step<2>(y + 2);
      if (y + 3 >= y1) break;
      step<3>(y + 3);
      if (y + 4 >= y1) break;
      step<4>(y + 4);
      if (y + 5 >= y1) break;
      step<5>(y + 5);
    }
  }
};

template <bool UYVY>
constexpr int kGauss5Lds = UYVY ? kUyvyQ * 128 : kGauss5Q * 64;

template <bool UYVY>
__device__ __forceinline__ void gauss5_item(const Gauss5Desc& d, int strip, int band, u32x4* lds) {
  const int y0 = band * d.g.rows;
  const int y1 = min(y0 + d.g.rows, d.g.h);
  if (strip == 0 || d.g.w <= (strip + 1) * kStripPx + kLanePx) {
    G5Stream<UYVY, true> s(d, strip, lds);
    s.run(y0, y1);
  } else {
    G5Stream<UYVY, false> s(d, strip, lds);
    s.run(y0, y1);
  }
  // no load into the queue may still be in flight when the wave moves on
  wait_vmem<0>();
}

// ---- Sobel 3x3 -> products -> Box5x5 (x3) -> corner response -> Threshold ----
//
// Four pixels per lane in 32-bit registers (the products need 21 bits, the
// window sums 25).  Strip: lanes 1..62 produce 4 output pixels each.  The
// structure-tensor sums are exact integers: each row's 5-pixel horizontal
// sums go into a ring of the last five rows and a running vertical sum is
// updated by adding the entering row and subtracting the leaving one.  The
// response is then evaluated in F32 from the exact sums.
namespace corner {

constexpr int LPX = 4;
constexpr int STRIP = 62 * LPX;

struct Lanes4 {
  int lane, xs, xl;
  bool store;
  bool mL;        // lane holding x = 0
  bool mR;        // lane whose last pixel is W-1 (W % 4 == 0)
  bool mRag;      // lane holding W-1 when W % 4 != 0
  int m;          // W % 4
  bool edgeL, edgeR;
};

__device__ __forceinline__ Lanes4 make_lanes(const StripGrid& g, int strip) {
  Lanes4 L;
  L.lane = threadIdx.x & 63;
  L.xs = strip * STRIP + (L.lane - 1) * LPX;
  const int wr = (g.w + 3) & ~3;
  L.xl = min(max(L.xs, 0), wr - 4);
  L.store = L.lane >= 1 && L.lane <= 62 && L.xs >= 0 && L.xs < g.w;
  L.m = g.w & 3;
  L.mL = L.xs == 0;
  L.mR = L.m == 0 && L.xs + 4 == g.w;
  L.mRag = L.m != 0 && L.xs == g.w - L.m;
  L.edgeL = strip == 0;
  L.edgeR = g.w <= (strip + 1) * STRIP + LPX;
  return L;
}

__device__ __forceinline__ int ileft(int v) { return (int)from_left_mov((u32)v); }
__device__ __forceinline__ int iright(int v) { return (int)from_right_mov((u32)v); }

// e[0..7] = values at x-2, x-1, x..x+3, x+4, x+5 after the border rule.
// HEDGE: the strip touches the left or right image edge; other strips need
// no border work at all.
template <int R, bool HEDGE>
__device__ __forceinline__ void extend4(int p[4], int e[8], const Lanes4& L, bool repl, int c) {
  if (HEDGE && L.edgeR && L.m != 0) {
    const int last = L.m == 1 ? p[0] : (L.m == 2 ? p[1] : p[2]);
    const int f = repl ? last : c;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int pos = L.m + t;  // 1..4
#pragma unroll
      for (int k = 1; k < 4; ++k)
        if (k == pos) p[k] = L.mRag ? f : p[k];
    }
  }
  e[1] = ileft(p[3]);
  e[6] = iright(p[0]);
  if (R >= 2) {
    e[0] = ileft(p[2]);
    e[7] = iright(p[1]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) e[k + 2] = p[k];
  if (HEDGE && L.edgeL && L.mL) {
    const int f = repl ? p[0] : c;
    e[1] = f;
    if (R >= 2) e[0] = f;
  }
  if (HEDGE && L.edgeR) {
    if (L.mR) {
      const int f = repl ? p[3] : c;
      e[6] = f;
      if (R >= 2) e[7] = f;
    }
    if (L.m != 0 && L.mRag && L.m + R - 1 >= 4) {  // pixel 4 of the ragged lane (m = 3, R = 2)
      e[6] = repl ? p[2] : c;
    }
  }
}

struct St {
  Lanes4 L;
  const uint8_t* inb;
  bool repl0, repl1;
  int c0, c1;
};

__device__ __forceinline__ int byte_of(u32 r, int k) { return (int)((r >> (8 * k)) & 0xFF); }

// Input rows travel through a queue of kQ rows in this wave's LDS, filled by
// direct-to-LDS loads (64 lanes x 4 bytes per row): the loads run kQ rows
// ahead without holding VGPRs.  The compiler does not track these loads
// against the LDS reads, so the waits are explicit, and the read completes
// before its slot is refilled.  Vector-memory operations complete in issue
// order, stores included.  A row's load is followed by the loads of the
// next kQ - 1 rows (every take issues one, clamped rows included) and by
// the output stores made since: one per output row between the take that
// issued it and the take that reads it, kQ in the steady state, fewer while
// the band starts (the first takes fill the ring, with no store between).
// The wait lets that many operations remain outstanding, rounded down.
constexpr int kQ = 8;

struct RowQueue {
  u32* buf;  // kQ x 64 dwords of LDS
  const uint8_t* src;
  int64_t pitch;
  int H, base, lane;
  bool repl;
  u32 fill;
  int stores;  // output rows stored so far in the band
  __device__ __forceinline__ void issue(int y) {
    const int yc = min(max(y, 0), H - 1);
    __builtin_amdgcn_global_load_lds((const void*)(src + (size_t)yc * pitch),
                                     (__attribute__((address_space(3))) void*)(buf + ((y - base) & (kQ - 1)) * 64), 4,
                                     0, 0);
  }
  __device__ __forceinline__ u32 take(int y) {
    static_assert(kQ == 8, "wait counts below assume eight rows");
    if (stores >= 8) asm volatile("s_waitcnt vmcnt(15)" ::: "memory");
    else if (stores >= 4) asm volatile("s_waitcnt vmcnt(11)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(7)" ::: "memory");
    u32 r = buf[((y - base) & (kQ - 1)) * 64 + lane];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (!repl && (y < 0 || y >= H)) r = fill;
    return r;
  }
};

// The lane's four pixels x0..x3 of an input row as two registers of 16-bit
// pairs: even (x0, x2) and odd (x1, x3).  The selector is an operand in a
// scalar register (the compiler otherwise rebuilds it in a vector register
// on every row).
__device__ __forceinline__ u32 perm_zero_s(u32 r, u32 sel) {
  u32 o;
  asm("v_perm_b32 %0, 0, %1, %2" : "=v"(o) : "v"(r), "s"(sel));
  return o;
}
__device__ __forceinline__ u32 even_pair(u32 r) { return perm_zero_s(r, 0x0C020C00u); }
__device__ __forceinline__ u32 odd_pair(u32 r) { return perm_zero_s(r, 0x0C030C01u); }
// a + 2 b + c on 16-bit pairs (one packed multiply-add; the inline constant 2
// sits in the low half, which op_sel_hi feeds to both halves)
__device__ __forceinline__ u32 sum121(u32 a, u32 b, u32 c) {
  u32 r;
  asm("v_pk_mad_u16 %0, %1, 2, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(b), "v"(add2(a, c)));
  return r;
}
// a + b + c in one instruction
__device__ __forceinline__ int add3(int a, int b, int c) {
  int r;
  asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
// signed 16-bit half h0 of a times half h1 of b (0 low, 1 high), into 32 bits
template <int H0, int H1>
__device__ __forceinline__ int mul_half(u32 a, u32 b) {
  int r;
  if (H0 == 0 && H1 == 0) asm("v_mad_i32_i16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  else if (H0 == 1 && H1 == 1) asm("v_mad_i32_i16 %0, %1, %2, 0 op_sel:[1,1,0,0]" : "=v"(r) : "v"(a), "v"(b));
  else if (H0 == 1) asm("v_mad_i32_i16 %0, %1, %2, 0 op_sel:[1,0,0,0]" : "=v"(r) : "v"(a), "v"(b));
  else asm("v_mad_i32_i16 %0, %1, %2, 0 op_sel:[0,1,0,0]" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Horizontal 5-sums of the three products at in-image row r (rows r-1, r, r+1
// given).  The Sobel part runs on 16-bit pairs (two pixels per instruction):
// sv = a + 2b + c and dv = c - a per column, their left and right neighbours
// by wave shifts and v_alignbit, the border of the Sobel's input applied to
// those neighbour columns (a column of border pixels has sv = 4c, dv = 0).
template <bool HEDGE>
__device__ __forceinline__ void hsums(const St& s, u32 a, u32 b, u32 c, int h[3][4]) {
  const Lanes4& L = s.L;
  u32 s0 = sum121(even_pair(a), even_pair(b), even_pair(c));  // sv (x0, x2)
  u32 s1 = sum121(odd_pair(a), odd_pair(b), odd_pair(c));     // sv (x1, x3)
  u32 d0 = sub2(even_pair(c), even_pair(a));                  // dv (x0, x2)
  u32 d1 = sub2(odd_pair(c), odd_pair(a));                    // dv (x1, x3)
  const u32 cs = (u32)(4 * s.c0) * 0x10001u;  // sv of a border column, both halves
  if (HEDGE && L.edgeR && L.m != 0 && L.mRag) {
    // the pixel just past W (position m of the ragged lane) becomes the border
    if (L.m == 1) {
      s1 = bfi(0x0000FFFFu, s.repl0 ? s0 : cs, s1);
      d1 = bfi(0x0000FFFFu, s.repl0 ? d0 : 0u, d1);
    } else if (L.m == 2) {
      s0 = s.repl0 ? perm(s1, s0, 0x05040100u) : bfi(0xFFFF0000u, cs, s0);
      d0 = s.repl0 ? perm(d1, d0, 0x05040100u) : (d0 & 0x0000FFFFu);
    } else {
      s1 = bfi(0xFFFF0000u, s.repl0 ? s0 : cs, s1);
      d1 = bfi(0xFFFF0000u, s.repl0 ? d0 : 0u, d1);
    }
  }
  // columns x-1, x1 and x2, x4 around the lane
  u32 ls = alignbit16(s1, from_left_mov(s1)), rs = alignbit16(from_right_mov(s0), s0);
  u32 ld = alignbit16(d1, from_left_mov(d1)), rd = alignbit16(from_right_mov(d0), d0);
  if (HEDGE && L.edgeL && L.mL) {  // x-1 left of the image
    ls = bfi(0x0000FFFFu, s.repl0 ? s0 : cs, ls);
    ld = bfi(0x0000FFFFu, s.repl0 ? d0 : 0u, ld);
  }
  if (HEDGE && L.edgeR && L.mR) {  // x4 right of the image (W % 4 == 0)
    rs = bfi(0xFFFF0000u, s.repl0 ? s1 : cs, rs);
    rd = bfi(0xFFFF0000u, s.repl0 ? d1 : 0u, rd);
  }
  const u32 gx0 = sub2(s1, ls), gx1 = sub2(rs, s0);          // gx (x0, x2), (x1, x3)
  const u32 gy0 = sum121(ld, d0, d1), gy1 = sum121(d0, d1, rd);  // gy (x0, x2), (x1, x3)
  int p[3][4];
  p[0][0] = mul_half<0, 0>(gx0, gx0);
  p[0][1] = mul_half<0, 0>(gx1, gx1);
  p[0][2] = mul_half<1, 1>(gx0, gx0);
  p[0][3] = mul_half<1, 1>(gx1, gx1);
  p[1][0] = mul_half<0, 0>(gy0, gy0);
  p[1][1] = mul_half<0, 0>(gy1, gy1);
  p[1][2] = mul_half<1, 1>(gy0, gy0);
  p[1][3] = mul_half<1, 1>(gy1, gy1);
  p[2][0] = mul_half<0, 0>(gx0, gy0);
  p[2][1] = mul_half<0, 0>(gx1, gy1);
  p[2][2] = mul_half<1, 1>(gx0, gy0);
  p[2][3] = mul_half<1, 1>(gx1, gy1);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    int e[8];
    extend4<2, HEDGE>(p[q], e, s.L, s.repl1, s.c1);
    // six three-input adds: m and n are the sums of the middle and right
    // triples, each output adds the rest of its window (written out, as the
    // compiler re-associates the sums into eight two- and three-input adds)
    const int m = add3(e[2], e[3], e[4]), n = add3(e[5], e[6], e[7]);
    h[q][0] = add3(e[0], e[1], m);
    h[q][1] = add3(e[1], m, e[5]);
    h[q][2] = add3(m, e[5], e[6]);
    h[q][3] = add3(e[3], e[4], n);
  }
}

}  // namespace corner

template <bool HEDGE>
__device__ __forceinline__ void corner_band(const CornerDesc& d, const corner::Lanes4& lanes, int band, u32* qbuf) {
  using namespace corner;
  St s;
  s.L = lanes;
  s.inb = d.in + s.L.xl;
  s.repl0 = d.b0 != B_CONSTANT;
  s.repl1 = d.b1 != B_CONSTANT;
  s.c0 = d.c0 & 0xFF;
  s.c1 = (int)d.c1;
  const int H = d.g.h;
  const int y0 = band * d.g.rows;
  const int y1 = min(y0 + d.g.rows, H);

  // input rows r-1, r, r+1 for the next gradient row r = nr, then rows
  // further down through the LDS queue
  int nr = max(y0 - 2, 0);
  RowQueue q{qbuf, s.inb, d.in_pitch, H, nr - 1, s.L.lane, s.repl0, 0x01010101u * (u32)s.c0, 0};
#pragma unroll
  for (int k = 0; k < kQ; ++k) q.issue(nr - 1 + k);
  u32 ia = q.take(nr - 1);
  q.issue(nr - 1 + kQ);
  u32 ib = q.take(nr);
  q.issue(nr + kQ);
  u32 ic = q.take(nr + 1);
  q.issue(nr + 1 + kQ);
  // H rows of the product planes; row y of the box needs rows y-2..y+2
  int ring[5][3][4];
  // H row r into out; `prev` holds H row r-1 (rows below the image repeat it
  // under REPLICATE, so no separate copy of the last in-image row is kept)
  auto next_h = [&](int r, int out[3][4], const int prev[3][4]) {
    if (r >= H) {
      // rows below the image: border of the box filters' input
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) out[q][k] = s.repl1 ? prev[q][k] : 5 * s.c1;
      return;
    }
    hsums<HEDGE>(s, ia, ib, ic, out);
    ia = ib;
    ib = ic;
    ic = q.take(r + 2);
    q.issue(r + 2 + kQ);
  };
  // prologue: rows y0-2 .. y0+2; above the image REPLICATE needs row 0 first
  if (y0 - 2 < 0) {
    int h0[3][4];
    next_h(0, h0, h0);  // row 0 (H >= 1, so never below the image)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int r = y0 - 2 + j;
      if (r < 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int k = 0; k < 4; ++k) ring[j][q][k] = s.repl1 ? h0[q][k] : 5 * s.c1;
      } else if (r == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int k = 0; k < 4; ++k) ring[j][q][k] = h0[q][k];
      } else {
        next_h(r, ring[j], ring[j - 1]);  // r > 0 here, so j >= 1
      }
    }
  } else {
    next_h(y0 - 2, ring[0], ring[0]);  // y0 - 2 < H
#pragma unroll
    for (int j = 1; j < 5; ++j) next_h(y0 - 2 + j, ring[j], ring[j - 1]);
  }
  int v[3][4];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      v[q][k] = ring[0][q][k] + ring[1][q][k] + ring[2][q][k] + ring[3][q][k] + ring[4][q][k];

  // descriptor fields the row loop needs, read once (the stores could alias
  // the descriptor as far as the compiler knows, which would make it reload
  // them every row)
  uint8_t* const out0 = d.out;
  const int64_t op = d.out_pitch;
  const u32 lout = (u32)s.L.xs;  // wraps for the left halo lane, which never stores
  const float kk = d.k, thr = d.thr;
  const u32 fv4 = d.fv4, x4 = d.tv4 ^ d.fv4;
  auto emit = [&](int y) {
    // thr - R = thr + Sxy^2 + k (Sxx + Syy)^2 - Sxx Syy in three fused
    // multiply-adds; its sign bit is set exactly where R > thr (equality
    // gives +0)
    u32 t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float sxx = (float)v[0][k], syy = (float)v[1][k], sxy = (float)v[2][k];
      const float tr = sxx + syy;
      t[k] = __float_as_uint(fmaf(-sxx, syy, fmaf(kk * tr, tr, fmaf(sxy, sxy, thr))));
    }
    // byte permute selectors 9 and 11 replicate bit 31 of the low and high
    // source: mask bytes 0xFF where R > thr, which pick tv over fv
    const u32 m = perm(t[1], t[0], 0x0C0C0B09u) | perm(t[3], t[2], 0x0B090C0Cu);
    const u32 o = fv4 ^ (m & x4);
    if (s.L.store) __builtin_nontemporal_store(o, (u32*)(out0 + lout + (size_t)((int64_t)y * op)));
    ++q.stores;
  };
  // unrolled by the ring length so that every ring slot index is a
  // compile-time constant; each step is guarded by a uniform branch
  for (int y = y0; y < y1; y += 5) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      if (y + j < y1) {
        emit(y + j);
        // the oldest row leaves the running sums, and its slot takes the new
        // row in place (no copy between registers)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int k = 0; k < 4; ++k) v[q][k] -= ring[j][q][k];
        next_h(y + j + 3, ring[j], ring[(j + 4) % 5]);
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int k = 0; k < 4; ++k) v[q][k] += ring[j][q][k];
      }
    }
  }
}

constexpr int kCornerLds = corner::kQ * 64 / 4;

__device__ __forceinline__ void corner_item(const CornerDesc& d, int strip, int band, u32x4* lds) {
  u32* qbuf = (u32*)lds;
  const corner::Lanes4 L = corner::make_lanes(d.g, strip);
  if (L.edgeL || L.edgeR) corner_band<true>(d, L, band, qbuf);
  else corner_band<false>(d, L, band, qbuf);
  // no load into the queue may still be in flight when the wave moves on
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

}  // namespace hvx
