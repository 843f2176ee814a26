// Kernel entry points and their host-side launchers.
#include <hip/hip_runtime.h>

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

__global__ __launch_bounds__(256) void k_generic(const GProg P, const IOTable io) {
  extern __shared__ int32_t lds[];
  generic_tile<256>(P, io, blockIdx.x, lds);
}

template <bool PHASE>
__global__ __launch_bounds__(64) void k_edge(const EdgeDesc d, int xcd) {
  const int item = xcd ? xcd_item(blockIdx.x, gridDim.x) : blockIdx.x;
  edge_item<PHASE>(d, item % d.g.nstrips, item / d.g.nstrips);
}

template <bool UYVY>
__global__ __launch_bounds__(64) void k_gauss5(const Gauss5Desc d, int xcd) {
  const int item = xcd ? xcd_item(blockIdx.x, gridDim.x) : blockIdx.x;
  gauss5_item<UYVY>(d, item % d.g.nstrips, item / d.g.nstrips);
}

// Persistent batch kernel: every wave takes work items from one atomic
// counter until the flat list is exhausted (each wave's last fetch is the one
// that fails, so every wave reaches the exit).  The next fetch is issued
// before the current item is processed to hide the atomic's latency.  The
// wave that finishes last resets both counters, so the next launch on the
// stream (or the next replay of a captured graph) starts from zero.
__device__ __forceinline__ void run_item(const BatchImage& bi, int local) {
  switch (bi.kind) {
    case FK_EDGE: {
      const EdgeDesc& d = bi.d.e;
      if (d.phase) edge_item<true>(d, local % d.g.nstrips, local / d.g.nstrips);
      else edge_item<false>(d, local % d.g.nstrips, local / d.g.nstrips);
      break;
    }
    case FK_GAUSS5: {
      const Gauss5Desc& d = bi.d.g5;
      if (d.uyvy) gauss5_item<true>(d, local % d.g.nstrips, local / d.g.nstrips);
      else gauss5_item<false>(d, local % d.g.nstrips, local / d.g.nstrips);
      break;
    }
    default: break;
  }
}

__global__ __launch_bounds__(64) void k_batch(const BatchImage* __restrict__ imgs,
                                              const uint16_t* __restrict__ item_img, int total,
                                              unsigned* __restrict__ counter) {
  const int lane = threadIdx.x & 63;
  unsigned got = 0;
  if (lane == 0) got = atomicAdd(&counter[0], 1u);
  int item = __builtin_amdgcn_readfirstlane((int)got);
  while (item < total) {
    unsigned nxt = 0;
    if (lane == 0) nxt = atomicAdd(&counter[0], 1u);
    const int im = item_img[item];
    const BatchImage& bi = imgs[im];
    run_item(bi, item - bi.first_item);
    item = __builtin_amdgcn_readfirstlane((int)nxt);
  }
  if (lane == 0) {
    unsigned done = atomicAdd(&counter[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counter[0], 0u);
      atomicExch(&counter[1], 0u);
    }
  }
}

// One work item per wave, no counter (used when the tuner finds it faster).
__global__ __launch_bounds__(64) void k_batch_direct(const BatchImage* __restrict__ imgs,
                                                     const uint16_t* __restrict__ item_img, int total) {
  const int item = blockIdx.x;
  if (item >= total) return;
  const BatchImage& bi = imgs[item_img[item]];
  run_item(bi, item - bi.first_item);
}

// ---- host launchers ---------------------------------------------------------

hipError_t launch_generic(const GProg& P, const IOTable& io, hipStream_t s) {
  const int tiles = P.tiles_x * P.tiles_y;
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_generic, dim3(tiles), dim3(256), (size_t)P.lds_words * 4, s, P, io);
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

hipError_t launch_batch(const BatchImage* imgs, const uint16_t* item_img, int total, unsigned* counter, int grid,
                        bool persistent, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  if (persistent) hipLaunchKernelGGL(k_batch, dim3(grid), dim3(64), 0, s, imgs, item_img, total, counter);
  else hipLaunchKernelGGL(k_batch_direct, dim3(total), dim3(64), 0, s, imgs, item_img, total);
  return hipGetLastError();
}

int batch_waves_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch, 64, 0) != hipSuccess || blocks <= 0) blocks = 8;
  return blocks;
}

}  // namespace hvx
