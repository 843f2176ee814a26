// Device helpers shared by the global-operator kernels and the fused
// kernels that reduce a global operator over their tiles: merging the
// (value, count) pairs of the smallest and largest pixel across a wave and
// into the 64-bit keys of the result (hvx_desc.h: mm_key, mm_merge).
#pragma once
// hipRTC (kernels generated at run time) provides the HIP and integer types itself
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "hvx_desc.h"

namespace hvx {

// Merges a (value, count) key into *dst with a compare-and-swap loop;
// skipped when the key can change nothing (no pixel, or a value that
// neither improves nor ties the current one).
__device__ __forceinline__ void merge_key(unsigned long long* dst, unsigned long long k, bool want_min) {
  if ((unsigned)k == 0) return;
  unsigned long long old = __atomic_load_n(dst, __ATOMIC_RELAXED);
  while (true) {
    const unsigned long long nw = mm_merge(old, k, want_min);
    if (nw == old) return;
    const unsigned long long seen = atomicCAS(dst, old, nw);
    if (seen == old) return;
    old = seen;
  }
}

// (value, count) pairs of both extremes merged across the wave: both lanes
// of each exchange compute the same merged pair, so every lane ends with the
// wave's result.
__device__ __forceinline__ void wave_merge_extremes(int& mn, uint32_t& cmn, int& mx, uint32_t& cmx) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int omn = __shfl_xor(mn, off), omx = __shfl_xor(mx, off);
    const uint32_t ocn = (uint32_t)__shfl_xor((int)cmn, off), ocx = (uint32_t)__shfl_xor((int)cmx, off);
    cmn = omn < mn ? ocn : (omn == mn ? cmn + ocn : cmn);
    cmx = omx > mx ? ocx : (omx == mx ? cmx + ocx : cmx);
    mn = min(mn, omn);
    mx = max(mx, omx);
  }
}

}  // namespace hvx
