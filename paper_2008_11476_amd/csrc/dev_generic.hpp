// Generic fused-group kernel body: an LDS tile interpreter.
//
// One work-group computes one output tile of a group of point and local
// operators (Section 4).  Group inputs are staged into LDS with the halo the
// group's stencils need; each operator then computes its output over the
// tile plus the halo its consumers still need, into LDS, and group outputs
// are written to global memory for the tile itself.  Intermediates that are
// virtual never leave LDS (transfer reduction and fusion, Sections 5.2.1 and
// 6.3).
//
// Border semantics are those of node-by-node execution: a local operator
// applies its own border mode to its own input, intermediates included.
// Intermediate values exist only at in-image coordinates; a read outside
// the image takes the constant (CONSTANT) or the nearest in-image value of
// the same intermediate (REPLICATE, UNDEFINED).  The clamped coordinate
// always lies in the region computed for that value.
#pragma once
// hipRTC (kernels generated at run time) provides the HIP and integer types itself
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "dev_phase.hpp"
#include "dev_reduce.hpp"

#include "gen_abi.h"
#include "hvx_desc.h"

namespace hvx {

__device__ __forceinline__ int gload(int df, const void* base, int64_t pitch, int x, int y) {
  const uint8_t* row = (const uint8_t*)base + (size_t)y * pitch;
  switch (df) {
    case DF_U8: return row[x];
    case DF_S16: return ((const int16_t*)row)[x];
    case DF_UYVY: return ((const uint16_t*)row)[x];
    default: return ((const int32_t*)row)[x];
  }
}

__device__ __forceinline__ void gstore(int df, void* base, int64_t pitch, int x, int y, int v) {
  uint8_t* row = (uint8_t*)base + (size_t)y * pitch;
  switch (df) {
    case DF_U8: row[x] = (uint8_t)v; break;
    case DF_S16: ((int16_t*)row)[x] = (int16_t)v; break;
    default: ((int32_t*)row)[x] = v; break;
  }
}

struct TileCtx {
  const GProg* P;
  const IOTable* io;
  const int32_t* lds;
  int tx0, ty0;
};

// Position read for x outside [0, n) under the MIRROR border: reflected
// about the first and last pixel (period 2 (n - 1)); a one-pixel axis
// repeats its pixel.
__device__ __forceinline__ int mirror_pos(int x, int n) {
  if (n == 1) return 0;
  const int per = 2 * (n - 1);
  x %= per;
  if (x < 0) x += per;
  return x < n ? x : per - x;
}

// Position read for x outside [0, n) under the REPEAT border: the image
// tiled periodically.
__device__ __forceinline__ int repeat_pos(int x, int n) {
  const int r = x % n;
  return r < 0 ? r + n : r;
}

// Read value `vi` at (x, y) as seen by operator `o` (border applied).  A
// mirrored position lies within the operator's radius of the image edge,
// inside the tile's extent of the value.  Under REPEAT the value is a group
// input whose tile extent outside the image was loaded from the periodic
// positions, so the position is read as it is.
__device__ __forceinline__ int rd(const TileCtx& t, const GOp& o, int vi, int x, int y) {
  const GProg& P = *t.P;
  const GVal& v = P.vals[vi];
  if ((x < 0 || y < 0 || x >= P.w || y >= P.h) && o.border != B_REPEAT) {
    if (o.border == B_CONSTANT) return v.df == DF_F32 ? __float_as_int(o.cf) : o.cint;
    if (o.border == B_MIRROR) {
      x = mirror_pos(x, P.w);
      y = mirror_pos(y, P.h);
    }
    x = min(max(x, 0), P.w - 1);
    y = min(max(y, 0), P.h - 1);
  }
  const int e = v.ext;
  const int rw = P.tw + 2 * e;
  return t.lds[v.lds + (y - (t.ty0 - e)) * rw + (x - (t.tx0 - e))];
}

__device__ __forceinline__ float rdf(const TileCtx& t, const GOp& o, int vi, int x, int y) {
  return __int_as_float(rd(t, o, vi, x, y));
}

// floor(sqrt(s)) for s < 2^32, exact: float estimate, then integer correction.
__device__ __forceinline__ uint32_t isqrt_u32(uint32_t s) {
  uint32_t q = (uint32_t)__builtin_sqrtf((float)s);
  if (q > 65535u) q = 65535u;
  while (q * q > s) --q;
  while ((q + 1) * (q + 1) <= s && q < 65535u) ++q;
  return q;
}

__device__ __forceinline__ int sat_u8(int v) { return min(max(v, 0), 255); }
__device__ __forceinline__ int sat_s16(int v) { return min(max(v, -32768), 32767); }

// The EqualizeHist mapping table of an OP_LUT operator: the 256 bytes after
// the counts in its second input, a buffer in device memory.
__device__ __forceinline__ const uint8_t* lut_table(const GProg& P, const IOTable& io, const GOp& o) {
  return (const uint8_t*)io.ptr[P.vals[o.in[1]].io] + 256 * 4;
}

// A user kernel (Section 5.1) at one pixel: its postfix program.  in(op,
// arg) returns an input element (int bits; F32 inputs as bit patterns, marked
// in o.p2): for X_IN input `arg`, for X_INW input a at a window offset.
// Integer kernels compute in 32-bit two's complement: + - * and negation
// wrap, / truncates toward zero, x / 0 = 0 and INT_MIN / -1 wraps to INT_MIN;
// the result saturates to the output type.  Float kernels (o.p1) compute in
// F32 and return F32 bits.
//
// Every lane runs the same program, so the stack position is the same in
// the whole wave.  The stack lives in LDS, one column per thread (entry k of
// thread t at [k][t]: the lanes of a wave touch consecutive words, no bank
// conflicts): a per-lane array indexed by the run-time position would be
// placed in scratch memory.  The kernels that run user kernels use
// kExprThreads-thread groups.
constexpr int kExprThreads = 256;
// one stack per work-group, shared by every place a kernel runs user kernels
__shared__ int32_t g_expr_stack[kExprStack][kExprThreads];

template <class IN>
__device__ __forceinline__ int expr_run(const GOp& o, int out_df, const IN& in) {
  int32_t* st = &g_expr_stack[0][threadIdx.x];
  auto at = [&](int k) -> int32_t& { return st[k * kExprThreads]; };
  const int n = o.p0;
  int sp = 0;
  if (o.p1) {
    auto f = [&](int k) { return __int_as_float(at(k)); };
    auto setf = [&](int k, float v) { at(k) = __float_as_int(v); };
    for (int k = 0; k < n; ++k) {
      const int op = o.code[k] & 0xFF, arg = o.code[k] >> 8;
      switch (op) {
        case X_IN:
        case X_INW: {
          const int v = in(op, arg);
          setf(sp++, ((o.p2 >> (op == X_IN ? arg : 0)) & 1) ? __int_as_float(v) : (float)v);
          break;
        }
        case X_CONST: at(sp++) = o.kc[arg]; break;
        case X_ADD: --sp; setf(sp - 1, f(sp - 1) + f(sp)); break;
        case X_SUB: --sp; setf(sp - 1, f(sp - 1) - f(sp)); break;
        case X_MUL: --sp; setf(sp - 1, f(sp - 1) * f(sp)); break;
        case X_DIV: --sp; setf(sp - 1, f(sp - 1) / f(sp)); break;
        case X_NEG: setf(sp - 1, -f(sp - 1)); break;
        case X_MIN: --sp; setf(sp - 1, fminf(f(sp - 1), f(sp))); break;
        case X_MAX: --sp; setf(sp - 1, fmaxf(f(sp - 1), f(sp))); break;
        case X_ABS: setf(sp - 1, fabsf(f(sp - 1))); break;
        case X_CLAMP: sp -= 2; setf(sp - 1, fminf(fmaxf(f(sp - 1), f(sp)), f(sp + 1))); break;
        case X_GT: --sp; setf(sp - 1, f(sp - 1) > f(sp) ? 1.f : 0.f); break;
        case X_SEL: sp -= 2; setf(sp - 1, f(sp - 1) != 0.f ? f(sp) : f(sp + 1)); break;
        case X_SQRT: setf(sp - 1, __builtin_sqrtf(f(sp - 1))); break;
      }
    }
    return at(0);
  }
  for (int k = 0; k < n; ++k) {
    const int op = o.code[k] & 0xFF, arg = o.code[k] >> 8;
    switch (op) {
      case X_IN:
      case X_INW: at(sp++) = in(op, arg); break;
      case X_CONST: at(sp++) = o.kc[arg]; break;
      case X_ADD: --sp; at(sp - 1) = (int)((uint32_t)at(sp - 1) + (uint32_t)at(sp)); break;
      case X_SUB: --sp; at(sp - 1) = (int)((uint32_t)at(sp - 1) - (uint32_t)at(sp)); break;
      case X_MUL: --sp; at(sp - 1) = (int)((uint32_t)at(sp - 1) * (uint32_t)at(sp)); break;
      case X_DIV: {
        --sp;
        const int x = at(sp - 1), y = at(sp);
        at(sp - 1) = y == 0 ? 0 : (y == -1 ? (int)(0u - (uint32_t)x) : x / y);
        break;
      }
      case X_NEG: at(sp - 1) = (int)(0u - (uint32_t)at(sp - 1)); break;
      case X_MIN: --sp; at(sp - 1) = min(at(sp - 1), at(sp)); break;
      case X_MAX: --sp; at(sp - 1) = max(at(sp - 1), at(sp)); break;
      case X_ABS: at(sp - 1) = at(sp - 1) < 0 ? (int)(0u - (uint32_t)at(sp - 1)) : at(sp - 1); break;
      case X_CLAMP: sp -= 2; at(sp - 1) = min(max(at(sp - 1), at(sp)), at(sp + 1)); break;
      case X_GT: --sp; at(sp - 1) = at(sp - 1) > at(sp) ? 1 : 0; break;
      case X_SEL: sp -= 2; at(sp - 1) = at(sp - 1) != 0 ? at(sp) : at(sp + 1); break;
    }
  }
  const int r = at(0);
  return out_df == DF_U8 ? min(max(r, 0), 255) : min(max(r, -32768), 32767);
}

__device__ __forceinline__ int expr_eval(const GOp& o, int out_df, int a, int b, int c) {
  return expr_run(o, out_df, [&](int, int arg) { return arg == 0 ? a : (arg == 1 ? b : c); });
}

// Readers whose offsets may be run-time values (the tile reader) declare
// kAnyOffset; the one-operator local kernel's window reader takes constant
// offsets only, so user local kernels are compiled into the tile path alone.
template <class T, class = void>
struct any_offset {
  static constexpr bool value = false;
};
template <class T>
struct any_offset<T, decltype((void)T::kAnyOffset)> {
  static constexpr bool value = true;
};

// A point operator (Section 4) on one pixel: a, b, c are its input elements
// (int bits; F32 as bit patterns; a UYVY input as its 16-bit U/V,Y pair),
// `in_f32` says whether the first input is F32.  Returns the output element.
__device__ __forceinline__ int point_eval(const GOp& o, int out_df, bool in_f32, int a, int b, int c) {
  switch (o.kind) {
    case OP_CHANNEL_Y: return (a >> 8) & 0xFF;
    case OP_MAGNITUDE: {
      uint32_t sq = (uint32_t)(a * a) + (uint32_t)(b * b);
      uint32_t q = isqrt_u32(sq);
      uint32_t m = q + ((sq - q * q) > q ? 1u : 0u);
      return (int)min(m, 32767u);
    }
    case OP_PHASE: {
      // the fused kernels' phase function; S16 gradients beyond 1023 are
      // first scaled down by a common power of two (the angle depends on
      // their ratio only; the truncation moves it by under 0.1 level)
      const int ua = a < 0 ? -a : a, ub = b < 0 ? -b : b;
      const int m = ua > ub ? ua : ub;
      const int sh = m >= 1024 ? 22 - __clz(m) : 0;
      const int sa = ua >> sh, sb = ub >> sh;
      const uint32_t ga = (uint32_t)(uint16_t)(a < 0 ? -sa : sa), gb = (uint32_t)(uint16_t)(b < 0 ? -sb : sb);
      return (int)(phase_pair(ga, gb) & 0xFF);
    }
    case OP_THRESHOLD: {
      bool hit = in_f32 ? (__int_as_float(a) > o.pf) : (a >= o.p2);
      return hit ? o.p0 : o.p1;
    }
    case OP_ADD: {
      int sm = a + b;
      if (out_df == DF_U8) return o.p0 == 0 ? sat_u8(sm) : (sm & 0xFF);
      return o.p0 == 0 ? sat_s16(sm) : (int)(int16_t)(uint16_t)(sm & 0xFFFF);
    }
    case OP_MULF: return __float_as_int((float)a * (float)b);
    case OP_EXPR: return expr_eval(o, out_df, a, b, c);
    case OP_HARRIS: {
      float sxx = __int_as_float(a), syy = __int_as_float(b), sxy = __int_as_float(c);
      float det = sxx * syy - sxy * sxy;
      float tr = sxx + syy;
      return __float_as_int(det - o.pf * tr * tr);
    }
  }
  return 0;
}

// Evaluate operator `o` at (x, y).  Returns the output element as int bits
// (F32 outputs as their bit pattern).
// A local operator (Section 4) at one pixel.  rd(dx, dy) returns its input
// at offset (dx, dy) from that pixel, border rule applied (int bits; F32 as
// bit patterns).  The Convolve mask is walked over the full 5 x 5 extent with
// the cells outside cols x rows skipped, so that every window offset is a
// compile-time constant.
// NonLinearFilter at one pixel (see OP_NONLINEAR).
template <class RD>
__device__ __forceinline__ int nonlinear_eval(const GOp& o, const RD& rd) {
    // the p0 x p1 mask selects window pixels (nonzero entries); p2: 0 the
    // median, 1 the minimum, 2 the maximum of them.  The median of n
    // pixels is the one at index n / 2 of their ascending order: a pixel
    // with at most n / 2 selected pixels below it and more than n / 2 at
    // or below it.
    const int cols = o.p0, rows = o.p1, rx = cols / 2, ry = rows / 2;
    int v[25];
    uint32_t sel = 0;
#pragma unroll
    for (int j = -2; j <= 2; ++j)
#pragma unroll
      for (int i = -2; i <= 2; ++i) {
        const int k = (j + 2) * 5 + (i + 2);
        v[k] = 0;
        if (i >= -rx && i <= rx && j >= -ry && j <= ry && o.mask[(j + ry) * cols + (i + rx)] != 0) {
          v[k] = rd(i, j);
          sel |= 1u << k;
        }
      }
    if (o.p2 != 0) {
      int m = o.p2 == 1 ? 255 : 0;
#pragma unroll
      for (int k = 0; k < 25; ++k)
        if ((sel >> k) & 1) m = o.p2 == 1 ? min(m, v[k]) : max(m, v[k]);
      return m;
    }
    const int half = __popc(sel) / 2;
    int r = 0;
#pragma unroll
    for (int a = 0; a < 25; ++a) {
      int below = 0, upto = 0;
#pragma unroll
      for (int b = 0; b < 25; ++b) {
        const int in = (sel >> b) & 1;
        below += in & (v[b] < v[a] ? 1 : 0);
        upto += in & (v[b] <= v[a] ? 1 : 0);
      }
      if (((sel >> a) & 1) && below <= half && half < upto) r = v[a];
    }
    return r;
}

template <bool NL, class RD>
__device__ __forceinline__ int local_eval(const GOp& o, int out_df, const RD& rd) {
  switch (o.kind) {
    case OP_GAUSS3: {
      int s = 0;
#pragma unroll
      for (int j = -1; j <= 1; ++j) {
        const int wj = j == 0 ? 2 : 1;
        int r = rd(-1, j) + 2 * rd(0, j) + rd(1, j);
        s += wj * r;
      }
      return s >> 4;
    }
    case OP_GAUSS5: {
      const int wt[5] = {1, 4, 6, 4, 1};
      int s = 0;
#pragma unroll
      for (int j = -2; j <= 2; ++j) {
        int r = 0;
#pragma unroll
        for (int i = -2; i <= 2; ++i) r += wt[i + 2] * rd(i, j);
        s += wt[j + 2] * r;
      }
      return s >> 8;
    }
    case OP_BOX3: {
      int s = 0;
#pragma unroll
      for (int j = -1; j <= 1; ++j)
#pragma unroll
        for (int i = -1; i <= 1; ++i) s += rd(i, j);
      return s / 9;
    }
    case OP_DILATE3:
    case OP_ERODE3: {
      const bool mx = o.kind == OP_DILATE3;
      int m = rd(0, 0);
#pragma unroll
      for (int j = -1; j <= 1; ++j)
#pragma unroll
        for (int i = -1; i <= 1; ++i) m = mx ? max(m, rd(i, j)) : min(m, rd(i, j));
      return m;
    }
    case OP_MEDIAN3: {
      // Sorting each row of the window and then each column leaves the
      // median of the nine on the anti-diagonal: the largest row minimum,
      // the median of the row medians and the smallest row maximum.
      int lo = 0, md[3], hi = 255;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int a = rd(-1, j - 1), b = rd(0, j - 1), c = rd(1, j - 1);
        lo = max(lo, min(a, min(b, c)));
        md[j] = max(min(a, b), min(max(a, b), c));
        hi = min(hi, max(a, max(b, c)));
      }
      const int mm = max(min(md[0], md[1]), min(max(md[0], md[1]), md[2]));
      return max(min(lo, mm), min(max(lo, mm), hi));
    }
    case OP_EXPR_LOCAL:
      if constexpr (any_offset<RD>::value)
        return expr_run(o, out_df, [&](int op, int arg) { return op == X_IN ? rd(0, 0) : rd(arg % 5 - 2, arg / 5 - 2); });
      break;
    case OP_NONLINEAR:
      // compiled only into the kernels built for it: its window and counters
      // would otherwise set the register budget of every generic kernel
      if constexpr (NL) return nonlinear_eval(o, rd);
      break;
    case OP_NONMAX: {
      // kept where every window pixel before it in raster order is smaller
      // and every one after it is not larger: the largest of each group
      // decides.  Window positions are read through the border rule, so a
      // border copy of the pixel itself counts like any other position.
      const int r = o.p0, p = rd(0, 0);
      int before = -65536, after = -65536;
#pragma unroll
      for (int j = -2; j <= 0; ++j)
#pragma unroll
        for (int i = -2; i <= 2; ++i) {
          if (j == 0 && i >= 0) continue;
          if (i >= -r && i <= r && j >= -r) before = max(before, rd(i, j));
          if (i >= -r && i <= r && j >= -r) after = max(after, rd(-i, -j));
        }
      return before < p && after <= p ? p : (out_df == DF_U8 ? 0 : -32768);
    }
    case OP_BOX5F: {
      // fixed order: each column top to bottom, columns left to right (a
      // thread that evaluates neighbouring outputs from one window forms the
      // column sums they share once)
      float s = 0.f;
#pragma unroll
      for (int i = -2; i <= 2; ++i) {
        float c = 0.f;
#pragma unroll
        for (int j = -2; j <= 2; ++j) c += __int_as_float(rd(i, j));
        s += c;
      }
      return __float_as_int(s);
    }
    case OP_SOBEL_X: {
      int s = 0;
#pragma unroll
      for (int j = -1; j <= 1; ++j) {
        const int wj = j == 0 ? 2 : 1;
        s += wj * (rd(1, j) - rd(-1, j));
      }
      return s;
    }
    case OP_SOBEL_Y: {
      int s = 0;
#pragma unroll
      for (int i = -1; i <= 1; ++i) {
        const int wi = i == 0 ? 2 : 1;
        s += wi * (rd(i, 1) - rd(i, -1));
      }
      return s;
    }
    case OP_CONVOLVE: {
      const int cols = o.p0, rows = o.p1, rx = cols / 2, ry = rows / 2;
      int s = 0;
#pragma unroll
      for (int j = -2; j <= 2; ++j)
#pragma unroll
        for (int i = -2; i <= 2; ++i)
          if (i >= -rx && i <= rx && j >= -ry && j <= ry)
            s += o.mask[(j + ry) * cols + (i + rx)] * rd(-i, -j);
      int q = s >= 0 ? (s >> o.p2) : -((-s) >> o.p2);  // divide by 2^p2 toward zero
      return out_df == DF_U8 ? sat_u8(q) : sat_s16(q);
    }
  }
  return 0;
}

__host__ __device__ inline int local_radius(int kind) {
  return (kind == OP_GAUSS5 || kind == OP_BOX5F || kind == OP_CONVOLVE || kind == OP_NONLINEAR || kind == OP_NONMAX ||
          kind == OP_EXPR_LOCAL)
             ? 2
             : 1;
}

// reads value `vi` of a tile as operator `o` sees it
struct TileRd {
  static constexpr bool kAnyOffset = true;
  const TileCtx* t;
  const GOp* o;
  int vi, x, y;
  __device__ __forceinline__ int operator()(int dx, int dy) const { return rd(*t, *o, vi, x + dx, y + dy); }
};

// Evaluate operator `o` at (x, y) inside a tile.  Returns the output element
// as int bits (F32 outputs as their bit pattern).
template <bool NL>
__device__ __forceinline__ int eval_op(const TileCtx& t, const GOp& o, int x, int y) {
  const GProg& P = *t.P;
  if (o.kind == OP_LUT) return lut_table(P, *t.io, o)[rd(t, o, o.in[0], x, y) & 0xFF];
  if (is_point_op(o.kind)) {
    const int a = rd(t, o, o.in[0], x, y);
    const int b = o.in[1] >= 0 ? rd(t, o, o.in[1], x, y) : 0;
    const int c = o.in[2] >= 0 ? rd(t, o, o.in[2], x, y) : 0;
    return point_eval(o, P.vals[o.out].df, P.vals[o.in[0]].df == DF_F32, a, b, c);
  }
  const int vi = o.in[0];
  return local_eval<NL>(o, P.vals[o.out].df, TileRd{&t, &o, vi, x, y});
}

// ---- global operators reduced over the tiles of a fused kernel --------------
// A work-group visits many tiles; for each global operator of the program
// (slot r, in program order) every thread keeps running partial results over
// the pixels it evaluates, the histogram counts go to an LDS histogram of the
// group, and the group merges everything into the operator's result once, at
// the end.  Only the tile's own pixels count (never the halo), so each pixel
// of the image is counted once.
// One global operator's running partial results in a thread.
struct RedSlot {
  int mn, mx;
  uint32_t cmn, cmx;
  unsigned long long s1, s2;
};

// kMaxRed slots as separate members, chosen by uniform branches: an array
// indexed by the run-time slot number would be placed in scratch memory.
struct RedState {
  RedSlot a, b;
  uint32_t* hist;   // this wave's copy of the histogram in LDS (kHistWords words)
  uint32_t* hist0;  // the first copy
  int copies;       // copies of the histogram, one per wave (or one in all)
  template <class F>
  __device__ __forceinline__ void with(int k, F&& f) {
    if (k == 0) f(a);
    else f(b);
  }
};
static_assert(kMaxRed == 2, "RedState holds two slots");

// HC copies of the histogram (1, or one per wave: waves then do not contend
// for the same LDS words); `hist` holds HC * kHistWords words.
template <int NT, int HC = 1>
__device__ __forceinline__ void red_begin(RedState& r, uint32_t* hist) {
  static_assert(HC == 1 || HC == NT / 64, "one histogram, or one per wave");
  r.a.mn = r.b.mn = 2147483647;
  r.a.mx = r.b.mx = -2147483647 - 1;
  r.a.cmn = r.a.cmx = r.b.cmn = r.b.cmx = 0;
  r.a.s1 = r.a.s2 = r.b.s1 = r.b.s2 = 0;
  r.hist0 = hist;
  r.copies = HC;
  r.hist = hist + (HC > 1 ? (int)(threadIdx.x >> 6) * kHistWords : 0);
  for (int b = threadIdx.x; b < HC * kHistWords; b += NT) hist[b] = 0;
  __syncthreads();
}

__device__ __forceinline__ void red_add(RedState& r, int k, const GOp& o, int v) {
  switch (o.kind) {
    case OP_HISTOGRAM:
    case OP_EQHIST: {
      const uint32_t x = (uint32_t)(v - o.p1);
      atomicAdd(&r.hist[x < (uint32_t)o.p2 ? x * (uint32_t)o.p0 / (uint32_t)o.p2 : 256u], 1u);
      break;
    }
    case OP_MMCOUNT:
      r.with(k, [&](RedSlot& q) {
        q.cmn = v < q.mn ? 1u : q.cmn + (v == q.mn ? 1u : 0u);
        q.cmx = v > q.mx ? 1u : q.cmx + (v == q.mx ? 1u : 0u);
        q.mn = min(q.mn, v);
        q.mx = max(q.mx, v);
      });
      break;
    case OP_MINMAX:
      r.with(k, [&](RedSlot& q) {
        q.mn = min(q.mn, v);
        q.mx = max(q.mx, v);
      });
      break;
    case OP_SUMS:
      r.with(k, [&](RedSlot& q) {
        q.s1 += (unsigned)v;
        q.s2 += (unsigned)(v * v);
      });
      break;
  }
}

// The group's partial results merged into the operators' results: waves
// reduce by lane exchange, the group through LDS, and one thread applies
// one atomic (or compare-and-swap loop) per result word.
template <int NT>
__device__ __forceinline__ void red_end(const GProg& P, const IOTable& io, RedState& r) {
  __shared__ unsigned long long part[4][NT / 64];
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  __syncthreads();  // the LDS histogram is complete
  int k = 0;
  for (int oi = 0; oi < P.nops; ++oi) {
    const GOp& o = P.ops[oi];
    if (!is_reduce_op(o.kind)) continue;
    void* out = io.ptr[P.vals[o.out].io];
    if (o.kind == OP_HISTOGRAM || o.kind == OP_EQHIST) {
      for (int b = t; b < o.p0; b += NT) {
        uint32_t c = 0;
        for (int h = 0; h < r.copies; ++h) c += r.hist0[h * kHistWords + b];
        if (c) atomicAdd((uint32_t*)out + b, c);
      }
    } else {
      RedSlot q;
      r.with(k, [&](RedSlot& x) { q = x; });
      int mn = q.mn, mx = q.mx;
      uint32_t cmn = q.cmn, cmx = q.cmx;
      unsigned long long s1 = q.s1, s2 = q.s2;
      if (o.kind == OP_SUMS) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          s1 += __shfl_xor(s1, off);
          s2 += __shfl_xor(s2, off);
        }
      } else if (o.kind == OP_MINMAX) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          mn = min(mn, __shfl_xor(mn, off));
          mx = max(mx, __shfl_xor(mx, off));
        }
      } else {
        wave_merge_extremes(mn, cmn, mx, cmx);
      }
      if (lane == 0) {
        if (o.kind == OP_SUMS) {
          part[0][wv] = s1;
          part[1][wv] = s2;
        } else {
          // a wave that saw no pixel holds the identities INT_MAX / INT_MIN,
          // which are no pixel values: it contributes the neutral keys
          part[0][wv] = o.kind == OP_MINMAX ? (unsigned long long)(unsigned)mn : (cmn ? mm_key(mn, cmn) : kMinKeyInit);
          part[1][wv] = o.kind == OP_MINMAX ? (unsigned long long)(unsigned)mx : (cmx ? mm_key(mx, cmx) : kMaxKeyInit);
        }
      }
      __syncthreads();
      if (t == 0) {
        if (o.kind == OP_SUMS) {
          for (int w = 1; w < NT / 64; ++w) {
            s1 += part[0][w];
            s2 += part[1][w];
          }
          atomicAdd((unsigned long long*)out, s1);
          atomicAdd((unsigned long long*)out + 1, s2);
        } else if (o.kind == OP_MINMAX) {
          for (int w = 1; w < NT / 64; ++w) {
            mn = min(mn, (int)(unsigned)part[0][w]);
            mx = max(mx, (int)(unsigned)part[1][w]);
          }
          int32_t* mm = (int32_t*)out;
          if (mn < __atomic_load_n(&mm[0], __ATOMIC_RELAXED)) atomicMin(&mm[0], mn);
          if (mx > __atomic_load_n(&mm[1], __ATOMIC_RELAXED)) atomicMax(&mm[1], mx);
        } else {
          unsigned long long kmin = kMinKeyInit, kmax = kMaxKeyInit;
          for (int w = 0; w < NT / 64; ++w) {
            kmin = mm_merge(kmin, part[0][w], true);
            kmax = mm_merge(kmax, part[1][w], false);
          }
          unsigned long long* keys = (unsigned long long*)((uint8_t*)out + kMMKeyOffset);
          const int sub = blockIdx.x % kMMSubKeys;
          merge_key(&keys[sub], kmin, true);
          merge_key(&keys[kMMSubKeys + sub], kmax, false);
        }
      }
      __syncthreads();
    }
    ++k;
  }
}

// As red_end, but the group writes its partial results to its own slot of
// a workspace (red_slot_words(P) words) instead of merging them into the
// results: a second kernel merges the slots (launch_merge_partials).
template <int NT>
__device__ __forceinline__ void red_end_partial(const GProg& P, RedState& r, uint32_t* slot) {
  __shared__ unsigned long long part[2][NT / 64];
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  __syncthreads();  // the LDS histogram is complete
  int k = 0, off = 0;
  for (int oi = 0; oi < P.nops; ++oi) {
    const GOp& o = P.ops[oi];
    if (!is_reduce_op(o.kind)) continue;
    if (o.kind == OP_HISTOGRAM || o.kind == OP_EQHIST) {
      for (int b = t; b < o.p0; b += NT) {
        uint32_t c = 0;
        for (int h = 0; h < r.copies; ++h) c += r.hist0[h * kHistWords + b];
        slot[off + b] = c;
      }
    } else {
      RedSlot q;
      r.with(k, [&](RedSlot& x) { q = x; });
      int mn = q.mn, mx = q.mx;
      uint32_t cmn = q.cmn, cmx = q.cmx;
      unsigned long long s1 = q.s1, s2 = q.s2;
      if (o.kind == OP_SUMS) {
#pragma unroll
        for (int sh = 32; sh > 0; sh >>= 1) {
          s1 += __shfl_xor(s1, sh);
          s2 += __shfl_xor(s2, sh);
        }
      } else if (o.kind == OP_MINMAX) {
#pragma unroll
        for (int sh = 32; sh > 0; sh >>= 1) {
          mn = min(mn, __shfl_xor(mn, sh));
          mx = max(mx, __shfl_xor(mx, sh));
        }
      } else {
        wave_merge_extremes(mn, cmn, mx, cmx);
      }
      if (lane == 0) {
        if (o.kind == OP_SUMS) {
          part[0][wv] = s1;
          part[1][wv] = s2;
        } else if (o.kind == OP_MINMAX) {
          part[0][wv] = (unsigned long long)(unsigned)mn;
          part[1][wv] = (unsigned long long)(unsigned)mx;
        } else {
          part[0][wv] = cmn ? mm_key(mn, cmn) : kMinKeyInit;
          part[1][wv] = cmx ? mm_key(mx, cmx) : kMaxKeyInit;
        }
      }
      __syncthreads();
      if (t == 0) {
        unsigned long long a = part[0][0], b = part[1][0];
        for (int w = 1; w < NT / 64; ++w) {
          if (o.kind == OP_SUMS) {
            a += part[0][w];
            b += part[1][w];
          } else if (o.kind == OP_MINMAX) {
            a = (unsigned long long)(unsigned)min((int)(unsigned)a, (int)(unsigned)part[0][w]);
            b = (unsigned long long)(unsigned)max((int)(unsigned)b, (int)(unsigned)part[1][w]);
          } else {
            a = mm_merge(a, part[0][w], true);
            b = mm_merge(b, part[1][w], false);
          }
        }
        if (o.kind == OP_MINMAX) {
          slot[off] = (uint32_t)a;
          slot[off + 1] = (uint32_t)b;
        } else {
          slot[off] = (uint32_t)a;
          slot[off + 1] = (uint32_t)(a >> 32);
          slot[off + 2] = (uint32_t)b;
          slot[off + 3] = (uint32_t)(b >> 32);
        }
      }
      __syncthreads();
    }
    off += red_block_words(o.kind, o.p0);
    ++k;
  }
}

// One tile of a generic program.  `lds` holds P.lds_words words.  RED: the
// program holds global operators, reduced into `red`.
// (Inlined into its kernels: as a called function it would receive the I/O
// table through a copy in scratch memory.)
template <int NT, bool NL, bool RED>
__device__ __forceinline__ void generic_tile(const GProg& P, const IOTable& io, int tile, int32_t* lds, RedState* red) {
  TileCtx t;
  t.P = &P;
  t.io = &io;
  t.lds = lds;
  t.tx0 = (tile % P.tiles_x) * P.tw;
  t.ty0 = (tile / P.tiles_x) * P.th;
  const int W = P.w, H = P.h;
  for (int vi = 0; vi < P.nvals; ++vi) {
    const GVal& v = P.vals[vi];
    if (!v.input || v.lds < 0) continue;
    const int e = v.ext, rw = P.tw + 2 * e;
    const int x0 = t.tx0 - e, y0 = t.ty0 - e;
    const int cx0 = max(x0, 0), cy0 = max(y0, 0);
    const int cx1 = min(x0 + rw, W), cy1 = min(y0 + P.th + 2 * e, H);
    const int cw = cx1 - cx0, ch = cy1 - cy0;
    if (cw <= 0 || ch <= 0) continue;
    const void* base = io.ptr[v.io];
    const int64_t pitch = io.pitch[v.io];
    if (v.wrap) {  // the whole extent, positions outside the image taken periodically
      for (int yy = y0 + (int)(threadIdx.x >> 6); yy < y0 + P.th + 2 * e; yy += NT / 64)
        for (int xx = x0 + (int)(threadIdx.x & 63); xx < x0 + rw; xx += 64)
          lds[v.lds + (yy - y0) * rw + (xx - x0)] = gload(v.df, base, pitch, repeat_pos(xx, W), repeat_pos(yy, H));
      continue;
    }
    // rows spread over groups of 64 threads, columns over the lanes
    for (int yy = cy0 + (int)(threadIdx.x >> 6); yy < cy1; yy += NT / 64)
      for (int xx = cx0 + (int)(threadIdx.x & 63); xx < cx1; xx += 64)
        lds[v.lds + (yy - y0) * rw + (xx - x0)] = gload(v.df, base, pitch, xx, yy);
  }
  __syncthreads();
  int slot = 0;
  for (int oi = 0; oi < P.nops; ++oi) {
    const GOp& o = P.ops[oi];
    if constexpr (RED) {
      if (is_reduce_op(o.kind)) {
        // the tile's own pixels of the input, read from its LDS tile
        const int x1 = min(t.tx0 + P.tw, W), y1 = min(t.ty0 + P.th, H);
        for (int yy = t.ty0 + (int)(threadIdx.x >> 6); yy < y1; yy += NT / 64)
          for (int xx = t.tx0 + (int)(threadIdx.x & 63); xx < x1; xx += 64)
            red_add(*red, slot, o, rd(t, o, o.in[0], xx, yy));
        ++slot;
        // the LDS the input occupies may be reused by the next operator's
        // output or the next tile's loads: every thread must be done reading
        __syncthreads();
        continue;
      }
    }
    const GVal& ov = P.vals[o.out];
    const int e = ov.lds >= 0 ? ov.ext : 0;
    const int rw = P.tw + 2 * e;
    const int x0 = t.tx0 - e, y0 = t.ty0 - e;
    const int cx0 = max(x0, 0), cy0 = max(y0, 0);
    const int cx1 = min(x0 + rw, W), cy1 = min(y0 + P.th + 2 * e, H);
    const int cw = cx1 - cx0, ch = cy1 - cy0;
    int32_t* dst = ov.lds >= 0 ? (int32_t*)lds + ov.lds : nullptr;
    void* gbase = ov.store ? io.ptr[ov.io] : nullptr;
    const int64_t gpitch = ov.store ? io.pitch[ov.io] : 0;
    if (cw > 0 && ch > 0) {
      for (int yy = cy0 + (int)(threadIdx.x >> 6); yy < cy1; yy += NT / 64)
        for (int xx = cx0 + (int)(threadIdx.x & 63); xx < cx1; xx += 64) {
          const int r = eval_op<NL>(t, o, xx, yy);
          if (dst) dst[(yy - y0) * rw + (xx - x0)] = r;
          if (gbase && xx >= t.tx0 && xx < t.tx0 + P.tw && yy >= t.ty0 && yy < t.ty0 + P.th)
            gstore(ov.df, gbase, gpitch, xx, yy, r);
        }
    }
    __syncthreads();
  }
}

// ---- one point operator over a whole image ----------------------------------
// A group that is a single point operator needs no tile or halo: each thread
// reads four consecutive pixels of each input with one vector load, applies
// the operator, and writes four pixels with one vector store (per-element
// accesses only in the last, partial group of a row).

__device__ __forceinline__ void load4(int df, const uint8_t* row, int x, int W, int v[4]) {
  if (x + 3 < W) {
    switch (df) {
      case DF_U8: {
        const uint32_t r = *(const uint32_t*)(row + x);
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = (r >> (8 * k)) & 0xFF;
        return;
      }
      case DF_S16: {
        const uint2 r = *(const uint2*)(row + 2 * x);
        v[0] = (int)(int16_t)(r.x & 0xFFFF);
        v[1] = ((int)r.x) >> 16;
        v[2] = (int)(int16_t)(r.y & 0xFFFF);
        v[3] = ((int)r.y) >> 16;
        return;
      }
      case DF_UYVY: {
        const uint2 r = *(const uint2*)(row + 2 * x);
        v[0] = r.x & 0xFFFF;
        v[1] = r.x >> 16;
        v[2] = r.y & 0xFFFF;
        v[3] = r.y >> 16;
        return;
      }
      default: {
        const uint4 r = *(const uint4*)(row + 4 * x);
        v[0] = (int)r.x;
        v[1] = (int)r.y;
        v[2] = (int)r.z;
        v[3] = (int)r.w;
        return;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = x + k < W ? gload(df, row, 0, x + k, 0) : 0;
}

// NT: a non-temporal store, for outputs that no later kernel of the graph
// reads (they stream past the caches instead of waiting there to be
// written back while the next kernels read)
template <bool NT, class T>
__device__ __forceinline__ void put(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <bool NT = false>
__device__ __forceinline__ void store4(int df, uint8_t* row, int x, int W, const int v[4]) {
  typedef uint32_t u2v __attribute__((ext_vector_type(2)));
  typedef uint32_t u4v __attribute__((ext_vector_type(4)));
  if (x + 3 < W) {
    switch (df) {
      case DF_U8:
        put<NT>((uint32_t*)(row + x), (uint32_t)(v[0] & 0xFF) | (uint32_t)(v[1] & 0xFF) << 8 |
                                          (uint32_t)(v[2] & 0xFF) << 16 | (uint32_t)(v[3] & 0xFF) << 24);
        return;
      case DF_S16:
        put<NT>((u2v*)(row + 2 * x), u2v{(uint32_t)(v[0] & 0xFFFF) | (uint32_t)v[1] << 16,
                                          (uint32_t)(v[2] & 0xFFFF) | (uint32_t)v[3] << 16});
        return;
      default:
        put<NT>((u4v*)(row + 4 * x), u4v{(uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2], (uint32_t)v[3]});
        return;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (x + k < W) gstore(df, row, 0, x + k, 0, v[k]);
}

// 256 threads cover 1024 pixels of one row; block b handles row b / bx of
// the ceil(W / 1024) = bx blocks per row.
__device__ __forceinline__ void point_image(const GProg& P, const IOTable& io) {
  const GOp& o = P.ops[0];
  const int W = P.w, H = P.h;
  const int bx = (W + 1023) >> 10;
  const int y = blockIdx.x / bx;
  const int x = ((blockIdx.x - y * bx) * 256 + (int)threadIdx.x) * 4;
  if (y >= H || x >= W) return;
  int a[4][4] = {};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (o.in[i] < 0) continue;
    const GVal& v = P.vals[o.in[i]];
    if (v.df == DF_BUF) continue;  // a table (OP_LUT), read below
    load4(v.df, (const uint8_t*)io.ptr[v.io] + (size_t)y * io.pitch[v.io], x, W, a[i]);
  }
  const GVal& ov = P.vals[o.out];
  const bool in_f32 = P.vals[o.in[0]].df == DF_F32;
  int r[4];
  if (o.kind == OP_LUT) {
    const uint8_t* tab = lut_table(P, io, o);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = tab[a[0][k] & 0xFF];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = point_eval(o, ov.df, in_f32, a[0][k], a[1][k], a[2][k]);
  }
  store4(ov.df, (uint8_t*)io.ptr[ov.io] + (size_t)y * io.pitch[ov.io], x, W, r);
}

// ---- one local operator over a whole image ----------------------------------
// A group that is a single local operator reads its input straight from
// global memory: each thread produces four consecutive pixels of one row
// from a window of (2R+1) rows x 12 columns (the aligned 4-pixel groups left
// of, at and right of its own), fetched with three vector loads per row;
// neighbouring threads' windows overlap in the caches, so HBM sees each input
// row about once.  Windows that leave the image take the border rule per
// element.

// reads the window of local_image around output pixel x0 + K: every index
// is a compile-time constant once inlined, so the window stays in VGPRs
template <int R, int K>
struct WinRd {
  const int (*w)[12];
  __device__ __forceinline__ int operator()(int dx, int dy) const { return w[R + dy][4 + K + dx]; }
};

template <int R, bool F32, bool NL>
__device__ __forceinline__ void local_image(const GProg& P, const IOTable& io) {
  const GOp& o = P.ops[0];
  const int W = P.w, H = P.h;
  const int bx = (W + 1023) >> 10;
  const int y = blockIdx.x / bx;
  const int x0 = ((blockIdx.x - y * bx) * 256 + (int)threadIdx.x) * 4;
  if (y >= H || x0 >= W) return;
  const GVal& iv = P.vals[o.in[0]];
  const GVal& ov = P.vals[o.out];
  const uint8_t* base = (const uint8_t*)io.ptr[iv.io];
  const int64_t pitch = io.pitch[iv.io];
  int win[2 * R + 1][12];  // columns x0-4 .. x0+7
  const bool inside = x0 >= 4 && x0 + 8 <= W && y >= R && y + R < H;
  if (inside) {
#pragma unroll
    for (int j = 0; j < 2 * R + 1; ++j) {
      const uint8_t* row = base + (size_t)(y - R + j) * pitch;
      if (F32) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const uint4 v = *(const uint4*)(row + 4 * (x0 - 4 + 4 * q));
          win[j][4 * q] = (int)v.x;
          win[j][4 * q + 1] = (int)v.y;
          win[j][4 * q + 2] = (int)v.z;
          win[j][4 * q + 3] = (int)v.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const uint32_t v = *(const uint32_t*)(row + x0 - 4 + 4 * q);
#pragma unroll
          for (int k = 0; k < 4; ++k) win[j][4 * q + k] = (v >> (8 * k)) & 0xFF;
        }
      }
    }
  } else {
    const bool cst = o.border == B_CONSTANT;
    const int cval = F32 ? __float_as_int(o.cf) : o.cint;
#pragma unroll
    for (int j = 0; j < 2 * R + 1; ++j)
#pragma unroll
      for (int k = 4 - R; k < 8 + R; ++k) {
        int xx = x0 - 4 + k, yy = y - R + j;
        const bool out = xx < 0 || yy < 0 || xx >= W || yy >= H;
        if (out && o.border == B_MIRROR) {
          xx = (xx < 0 || xx >= W) ? mirror_pos(xx, W) : xx;
          yy = (yy < 0 || yy >= H) ? mirror_pos(yy, H) : yy;
        }
        if (out && o.border == B_REPEAT) {
          xx = repeat_pos(xx, W);
          yy = repeat_pos(yy, H);
        }
        xx = min(max(xx, 0), W - 1);
        yy = min(max(yy, 0), H - 1);
        const int v = gload(iv.df, base, pitch, xx, yy);
        win[j][k] = (out && cst) ? cval : v;
      }
  }
  int r[4];
  r[0] = local_eval<NL>(o, ov.df, WinRd<R, 0>{win});
  r[1] = local_eval<NL>(o, ov.df, WinRd<R, 1>{win});
  r[2] = local_eval<NL>(o, ov.df, WinRd<R, 2>{win});
  r[3] = local_eval<NL>(o, ov.df, WinRd<R, 3>{win});
  store4(ov.df, (uint8_t*)io.ptr[ov.io] + (size_t)y * io.pitch[ov.io], x0, W, r);
}

}  // namespace hvx
