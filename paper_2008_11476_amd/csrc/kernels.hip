// Kernel entry points and their host-side launchers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dev_fast.hpp"
#include "dev_generic.hpp"
#include "kernels.h"

namespace hvx {

// Work items are spread so that each of the 8 XCDs (each with its own L2)
// receives a contiguous range: blocks are dispatched to XCDs round-robin, so
// block b runs on XCD b % 8.  Adjacent bands then share halo rows in one L2.
__device__ __forceinline__ int xcd_item(int b, int n) {
  const int x = b & 7, i = b >> 3;
  const int q = n >> 3, r = n & 7;
  return x * q + min(x, r) + i;
}

// The program lives in device memory: the interpreter indexes its value and
// operator tables with wave-uniform indices (scalar loads), which a by-value
// kernel argument would turn into a private (scratch) copy.
// NL: the program holds a NonLinearFilter (its evaluation is compiled only
// into these variants, which carry its registers)
// RED: the program reduces global operators; the groups then loop over the
// tiles (fewer groups than tiles, so each merges its partial results once)
// and the LDS after the tiles holds the group's histogram.
static_assert(kExprThreads == 256, "user kernels run in 256-thread groups");

template <bool NL, bool RED>
__global__ __launch_bounds__(256) void k_generic(const GProg* __restrict__ P, const IOTable io) {
  extern __shared__ int32_t lds[];
  if constexpr (!RED) {
    generic_tile<256, NL, false>(*P, io, blockIdx.x, lds, nullptr);
  } else {
    RedState rs;
    red_begin<256>(rs, (uint32_t*)(lds + P->lds_words));
    const int ntiles = P->tiles_x * P->tiles_y;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      generic_tile<256, NL, true>(*P, io, tile, lds, &rs);
      __syncthreads();  // the tile's LDS is free for the next tile's loads
    }
    red_end<256>(*P, io, rs);
  }
}

__global__ __launch_bounds__(256) void k_point(const GProg* __restrict__ P, const IOTable io) {
  point_image(*P, io);
}

template <int R, bool F32, bool NL>
__global__ __launch_bounds__(256) void k_local(const GProg* __restrict__ P, const IOTable io) {
  local_image<R, F32, NL>(*P, io);
}

template <bool PHASE>
__global__ __launch_bounds__(64) void k_edge(const EdgeDesc d, int xcd) {
  __shared__ u32x4 lds[kEdgeLds];
  const int item = xcd ? xcd_item(blockIdx.x, gridDim.x) : blockIdx.x;
  edge_item<PHASE>(d, item % d.g.nstrips, item / d.g.nstrips, lds);
}

__global__ __launch_bounds__(64) void k_corner(const CornerDesc d, int xcd) {
  __shared__ u32x4 lds[kCornerLds];
  const int item = xcd ? xcd_item(blockIdx.x, gridDim.x) : blockIdx.x;
  corner_item(d, item % d.g.nstrips, item / d.g.nstrips, lds);
}

template <bool UYVY>
__global__ __launch_bounds__(64) void k_gauss5(const Gauss5Desc d, int xcd) {
  __shared__ u32x4 lds[kGauss5Lds<UYVY>];
  const int item = xcd ? xcd_item(blockIdx.x, gridDim.x) : blockIdx.x;
  gauss5_item<UYVY>(d, item % d.g.nstrips, item / d.g.nstrips, lds);
}

// Persistent batch kernel.  The flat work list is cut into 8 contiguous
// ranges, one per XCD group of waves (block b belongs to group b % 8, the
// XCD the hardware dispatches it to), so that the atomics of different
// groups hit different counters and neighbouring items share an L2.  Within
// a group, waves take `chunk` consecutive items per atomic fetch until the
// range is exhausted; the next fetch is issued before the current chunk is
// processed.  Every wave's last fetch is the one past the end of its range,
// so every wave exits.  The last wave of a group to finish resets that
// group's counters, so the next launch (or graph replay) starts from zero.
constexpr int kCtrStride = 32;  // counters 128 bytes apart

// KS: the set of kinds a batch holds (bit 1 edge, 2 corner, 4 Gaussian5x5,
// 8 edge with phase, 16 Gaussian5x5 of UYVY luma); only those bodies are
// compiled into the batch kernel, so a batch of one kind keeps that kind's
// register budget and occupancy.
// LDS of a batch kernel: the largest need among its kinds (one item at a time)
constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <int KS>
constexpr int kBatchLds = cmax(cmax((KS & 9) ? kEdgeLds : 1, (KS & 2) ? kCornerLds : 1),
                               cmax((KS & 4) ? kGauss5Lds<false> : 1, (KS & 16) ? kGauss5Lds<true> : 1));

template <int KS>
__device__ __forceinline__ void run_item(const BatchImage& bi, int local, u32x4* lds) {
  if ((KS & 9) && bi.kind == FK_EDGE) {
    const EdgeDesc& d = bi.d.e;
    if ((KS & 8) && d.phase) edge_item<true>(d, local % d.g.nstrips, local / d.g.nstrips, lds);
    else if (KS & 1) edge_item<false>(d, local % d.g.nstrips, local / d.g.nstrips, lds);
  } else if ((KS & 2) && bi.kind == FK_CORNER) {
    const CornerDesc& d = bi.d.c;
    corner_item(d, local % d.g.nstrips, local / d.g.nstrips, lds);
  } else if ((KS & 20) && bi.kind == FK_GAUSS5) {
    const Gauss5Desc& d = bi.d.g5;
    if ((KS & 16) && d.uyvy) gauss5_item<true>(d, local % d.g.nstrips, local / d.g.nstrips, lds);
    else if (KS & 4) gauss5_item<false>(d, local % d.g.nstrips, local / d.g.nstrips, lds);
  }
}

template <int KS>
__device__ __forceinline__ void run_flat(const BatchImage* __restrict__ imgs, const uint16_t* __restrict__ item_img,
                                         int item, u32x4* lds) {
  const int im = item_img[item];
  const BatchImage& bi = imgs[im];
  run_item<KS>(bi, item - bi.first_item, lds);
}

template <int KS>
__global__ __launch_bounds__(64, 4) void k_batch(const BatchImage* __restrict__ imgs,
                                              const uint16_t* __restrict__ item_img, int total, int chunk,
                                              unsigned* __restrict__ counter) {
  __shared__ u32x4 lds[kBatchLds<KS>];
  const int lane = threadIdx.x & 63;
  const int grp = blockIdx.x & 7;
  const int begin = (int)((long long)total * grp / 8), end = (int)((long long)total * (grp + 1) / 8);
  unsigned* next = counter + grp * kCtrStride;
  unsigned* done = counter + (8 + grp) * kCtrStride;
  unsigned got = 0;
  if (lane == 0) got = atomicAdd(next, (unsigned)chunk);
  int base = begin + __builtin_amdgcn_readfirstlane((int)got);
  while (base < end) {
    unsigned nxt = 0;
    if (lane == 0) nxt = atomicAdd(next, (unsigned)chunk);
    const int stop = min(base + chunk, end);
    for (int item = base; item < stop; ++item) run_flat<KS>(imgs, item_img, item, lds);
    base = begin + __builtin_amdgcn_readfirstlane((int)nxt);
  }
  if (lane == 0) {
    const unsigned waves = (gridDim.x - grp + 7) / 8;  // blocks of this group
    const unsigned d = atomicAdd(done, 1u);
    if (d == waves - 1) {
      atomicExch(next, 0u);
      atomicExch(done, 0u);
    }
  }
}

// One wave per work item, no counter; items mapped XCD-contiguously.
template <int KS>
__global__ __launch_bounds__(64) void k_batch_direct(const BatchImage* __restrict__ imgs,
                                                     const uint16_t* __restrict__ item_img, int total) {
  __shared__ u32x4 lds[kBatchLds<KS>];
  const int item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= total) return;
  run_flat<KS>(imgs, item_img, item, lds);
}

// ---- host launchers ---------------------------------------------------------

hipError_t launch_generic(const GProg& P, const GProg* dev_prog, const IOTable& io, int num_cus, hipStream_t s) {
  if (P.nops == 1 && is_point_op(P.ops[0].kind)) {
    const long long blocks = (long long)((P.w + 1023) >> 10) * P.h;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_point, dim3((unsigned)blocks), dim3(256), 0, s, dev_prog, io);
    return hipGetLastError();
  }
  const int in_df = P.nops == 1 && P.ops[0].in[0] >= 0 ? P.vals[P.ops[0].in[0]].df : -1;
  // a user local kernel reads its window at run-time offsets: tile path only
  if (P.nops == 1 && (in_df == DF_U8 || in_df == DF_F32) && P.ops[0].kind != OP_EXPR_LOCAL) {
    const GOp& o = P.ops[0];
    const long long blocks = (long long)((P.w + 1023) >> 10) * P.h;
    if (blocks <= 0) return hipSuccess;
    const bool f32 = in_df == DF_F32;
    const dim3 g((unsigned)blocks), b(256);
    if (o.kind == OP_NONLINEAR) {  // U8 only, mask up to 5x5
      hipLaunchKernelGGL((k_local<2, false, true>), g, b, 0, s, dev_prog, io);
    } else if (local_radius(o.kind) == 1) {
      if (f32) hipLaunchKernelGGL((k_local<1, true, false>), g, b, 0, s, dev_prog, io);
      else hipLaunchKernelGGL((k_local<1, false, false>), g, b, 0, s, dev_prog, io);
    } else {
      if (f32) hipLaunchKernelGGL((k_local<2, true, false>), g, b, 0, s, dev_prog, io);
      else hipLaunchKernelGGL((k_local<2, false, false>), g, b, 0, s, dev_prog, io);
    }
    return hipGetLastError();
  }
  const int tiles = P.tiles_x * P.tiles_y;
  if (tiles <= 0) return hipSuccess;
  bool nl = false;
  for (int i = 0; i < P.nops; ++i) nl |= P.ops[i].kind == OP_NONLINEAR;
  if (P.nred > 0) {
    // four groups per CU at most, each merging its results once
    const dim3 g((unsigned)std::min(tiles, 4 * num_cus));
    const size_t lds = (size_t)(P.lds_words + kHistWords) * 4;
    if (nl) hipLaunchKernelGGL((k_generic<true, true>), g, dim3(256), lds, s, dev_prog, io);
    else hipLaunchKernelGGL((k_generic<false, true>), g, dim3(256), lds, s, dev_prog, io);
    return hipGetLastError();
  }
  if (nl) hipLaunchKernelGGL((k_generic<true, false>), dim3(tiles), dim3(256), (size_t)P.lds_words * 4, s, dev_prog, io);
  else hipLaunchKernelGGL((k_generic<false, false>), dim3(tiles), dim3(256), (size_t)P.lds_words * 4, s, dev_prog, io);
  return hipGetLastError();
}

hipError_t launch_edge(const EdgeDesc& d, bool xcd, hipStream_t s) {
  const int n = d.g.nstrips * d.g.nbands;
  if (n <= 0) return hipSuccess;
  if (d.phase) hipLaunchKernelGGL(k_edge<true>, dim3(n), dim3(64), 0, s, d, xcd ? 1 : 0);
  else hipLaunchKernelGGL(k_edge<false>, dim3(n), dim3(64), 0, s, d, xcd ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_gauss5(const Gauss5Desc& d, bool xcd, hipStream_t s) {
  const int n = d.g.nstrips * d.g.nbands;
  if (n <= 0) return hipSuccess;
  if (d.uyvy) hipLaunchKernelGGL(k_gauss5<true>, dim3(n), dim3(64), 0, s, d, xcd ? 1 : 0);
  else hipLaunchKernelGGL(k_gauss5<false>, dim3(n), dim3(64), 0, s, d, xcd ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_corner(const CornerDesc& d, bool xcd, hipStream_t s) {
  const int n = d.g.nstrips * d.g.nbands;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_corner, dim3(n), dim3(64), 0, s, d, xcd ? 1 : 0);
  return hipGetLastError();
}

template <int KS>
static void launch_batch_ks(const BatchImage* imgs, const uint16_t* item_img, int total, unsigned* counter, int grid,
                            bool persistent, hipStream_t s) {
  if (persistent) {
    grid = max(grid, 8);  // every group of the 8 ranges needs at least one wave
    const int per_group_waves = max(1, grid / 8);
    const int chunk = max(1, (total / 8) / (per_group_waves * 4));
    hipLaunchKernelGGL(k_batch<KS>, dim3(grid), dim3(64), 0, s, imgs, item_img, total, chunk, counter);
  } else {
    hipLaunchKernelGGL(k_batch_direct<KS>, dim3(total), dim3(64), 0, s, imgs, item_img, total);
  }
}

hipError_t launch_batch(const BatchImage* imgs, const uint16_t* item_img, int total, unsigned* counter, int grid,
                        bool persistent, int kinds, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  switch (kinds) {
    case 1: launch_batch_ks<1>(imgs, item_img, total, counter, grid, persistent, s); break;
    case 2: launch_batch_ks<2>(imgs, item_img, total, counter, grid, persistent, s); break;
    case 4: launch_batch_ks<4>(imgs, item_img, total, counter, grid, persistent, s); break;
    case 8: launch_batch_ks<8>(imgs, item_img, total, counter, grid, persistent, s); break;
    case 16: launch_batch_ks<16>(imgs, item_img, total, counter, grid, persistent, s); break;
    case 7: launch_batch_ks<7>(imgs, item_img, total, counter, grid, persistent, s); break;
    case 19: launch_batch_ks<19>(imgs, item_img, total, counter, grid, persistent, s); break;
    default: launch_batch_ks<31>(imgs, item_img, total, counter, grid, persistent, s); break;
  }
  return hipGetLastError();
}

int kind_bit(const BatchImage& bi) {
  switch (bi.kind) {
    case FK_EDGE: return bi.d.e.phase ? 8 : 1;
    case FK_CORNER: return 2;
    case FK_GAUSS5: return bi.d.g5.uyvy ? 16 : 4;
    default: return 0;
  }
}

size_t batch_counter_bytes() { return 16 * kCtrStride * sizeof(unsigned); }

int batch_waves_per_cu(int kinds) {
  int blocks = 0;
  hipError_t e;
  switch (kinds) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<1>, 64, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<2>, 64, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<4>, 64, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<8>, 64, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<16>, 64, 0); break;
    case 7: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<7>, 64, 0); break;
    case 19: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<19>, 64, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<31>, 64, 0); break;
  }
  if (e != hipSuccess || blocks <= 0) blocks = 8;
  return blocks;
}

}  // namespace hvx
