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
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_phase.hpp"

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
  const int32_t* lds;
  int tx0, ty0;
};

// Read value `vi` at (x, y) as seen by operator `o` (border applied).
__device__ __forceinline__ int rd(const TileCtx& t, const GOp& o, int vi, int x, int y) {
  const GProg& P = *t.P;
  const GVal& v = P.vals[vi];
  if (x < 0 || y < 0 || x >= P.w || y >= P.h) {
    if (o.border == B_CONSTANT) return v.df == DF_F32 ? __float_as_int(o.cf) : o.cint;
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

// Evaluate operator `o` at (x, y).  Returns the output element as int bits
// (F32 outputs as their bit pattern).
__device__ __forceinline__ int eval_op(const TileCtx& t, const GOp& o, int x, int y) {
  const GProg& P = *t.P;
  switch (o.kind) {
    case OP_CHANNEL_Y: return (rd(t, o, o.in[0], x, y) >> 8) & 0xFF;
    case OP_GAUSS3: {
      int s = 0;
#pragma unroll
      for (int j = -1; j <= 1; ++j) {
        const int wj = j == 0 ? 2 : 1;
        int r = rd(t, o, o.in[0], x - 1, y + j) + 2 * rd(t, o, o.in[0], x, y + j) + rd(t, o, o.in[0], x + 1, y + j);
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
        for (int i = -2; i <= 2; ++i) r += wt[i + 2] * rd(t, o, o.in[0], x + i, y + j);
        s += wt[j + 2] * r;
      }
      return s >> 8;
    }
    case OP_BOX3: {
      int s = 0;
#pragma unroll
      for (int j = -1; j <= 1; ++j)
#pragma unroll
        for (int i = -1; i <= 1; ++i) s += rd(t, o, o.in[0], x + i, y + j);
      return s / 9;
    }
    case OP_BOX5F: {
      // fixed order: each row left to right, rows top to bottom
      float s = 0.f;
#pragma unroll
      for (int j = -2; j <= 2; ++j) {
        float r = 0.f;
#pragma unroll
        for (int i = -2; i <= 2; ++i) r += rdf(t, o, o.in[0], x + i, y + j);
        s += r;
      }
      return __float_as_int(s);
    }
    case OP_SOBEL_X: {
      int s = 0;
#pragma unroll
      for (int j = -1; j <= 1; ++j) {
        const int wj = j == 0 ? 2 : 1;
        s += wj * (rd(t, o, o.in[0], x + 1, y + j) - rd(t, o, o.in[0], x - 1, y + j));
      }
      return s;
    }
    case OP_SOBEL_Y: {
      int s = 0;
#pragma unroll
      for (int i = -1; i <= 1; ++i) {
        const int wi = i == 0 ? 2 : 1;
        s += wi * (rd(t, o, o.in[0], x + i, y + 1) - rd(t, o, o.in[0], x + i, y - 1));
      }
      return s;
    }
    case OP_MAGNITUDE: {
      int a = rd(t, o, o.in[0], x, y), b = rd(t, o, o.in[1], x, y);
      uint32_t s = (uint32_t)(a * a) + (uint32_t)(b * b);
      uint32_t q = isqrt_u32(s);
      uint32_t m = q + ((s - q * q) > q ? 1u : 0u);
      return (int)min(m, 32767u);
    }
    case OP_PHASE: {
      // the fused kernels' phase function; S16 gradients beyond 1023 are
      // first scaled down by a common power of two (the angle depends on
      // their ratio only; the truncation moves it by under 0.1 level)
      int a = rd(t, o, o.in[0], x, y), b = rd(t, o, o.in[1], x, y);
      const int ua = a < 0 ? -a : a, ub = b < 0 ? -b : b;
      const int m = ua > ub ? ua : ub;
      const int sh = m >= 1024 ? 22 - __clz(m) : 0;
      const int sa = ua >> sh, sb = ub >> sh;
      const uint32_t ga = (uint32_t)(uint16_t)(a < 0 ? -sa : sa), gb = (uint32_t)(uint16_t)(b < 0 ? -sb : sb);
      return (int)(phase_pair(ga, gb) & 0xFF);
    }
    case OP_THRESHOLD: {
      const GVal& iv = P.vals[o.in[0]];
      int v = rd(t, o, o.in[0], x, y);
      bool hit = iv.df == DF_F32 ? (__int_as_float(v) > o.pf) : (v >= o.p2);
      return hit ? o.p0 : o.p1;
    }
    case OP_ADD: {
      int s = rd(t, o, o.in[0], x, y) + rd(t, o, o.in[1], x, y);
      int odf = P.vals[o.out].df;
      if (odf == DF_U8) return o.p0 == 0 ? sat_u8(s) : (s & 0xFF);
      return o.p0 == 0 ? sat_s16(s) : (int)(int16_t)(uint16_t)(s & 0xFFFF);
    }
    case OP_MULF: {
      float a = (float)rd(t, o, o.in[0], x, y), b = (float)rd(t, o, o.in[1], x, y);
      return __float_as_int(a * b);
    }
    case OP_HARRIS: {
      float sxx = rdf(t, o, o.in[0], x, y), syy = rdf(t, o, o.in[1], x, y), sxy = rdf(t, o, o.in[2], x, y);
      float det = sxx * syy - sxy * sxy;
      float tr = sxx + syy;
      return __float_as_int(det - o.pf * tr * tr);
    }
    case OP_CONVOLVE: {
      const int cols = o.p0, rows = o.p1, rx = cols / 2, ry = rows / 2;
      int s = 0;
      for (int j = -ry; j <= ry; ++j)
        for (int i = -rx; i <= rx; ++i) s += o.mask[(j + ry) * cols + (i + rx)] * rd(t, o, o.in[0], x - i, y - j);
      int q = s >= 0 ? (s >> o.p2) : -((-s) >> o.p2);  // divide by 2^p2 toward zero
      return P.vals[o.out].df == DF_U8 ? sat_u8(q) : sat_s16(q);
    }
  }
  return 0;
}

// One tile of a generic program.  `lds` holds P.lds_words words.
template <int NT>
__device__ void generic_tile(const GProg& P, const IOTable& io, int tile, int32_t* lds) {
  TileCtx t;
  t.P = &P;
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
    for (int i = threadIdx.x; i < cw * ch; i += NT) {
      const int yy = cy0 + i / cw, xx = cx0 + i % cw;
      lds[v.lds + (yy - y0) * rw + (xx - x0)] = gload(v.df, base, pitch, xx, yy);
    }
  }
  __syncthreads();
  for (int oi = 0; oi < P.nops; ++oi) {
    const GOp& o = P.ops[oi];
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
      for (int i = threadIdx.x; i < cw * ch; i += NT) {
        const int yy = cy0 + i / cw, xx = cx0 + i % cw;
        const int r = eval_op(t, o, xx, yy);
        if (dst) dst[(yy - y0) * rw + (xx - x0)] = r;
        if (gbase && xx >= t.tx0 && xx < t.tx0 + P.tw && yy >= t.ty0 && yy < t.ty0 + P.th)
          gstore(ov.df, gbase, gpitch, xx, yy, r);
      }
    }
    __syncthreads();
  }
}

}  // namespace hvx
