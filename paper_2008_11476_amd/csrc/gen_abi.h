// Arguments shared by the host and the kernels generated at run time beyond
// the interpreter's own (hvx_desc.h): plain data, no pointers to host memory.
#pragma once
#include "hvx_desc.h"

namespace hvx {

// One image of a batch run by one generated kernel: its I/O table, its size
// and the first work-group of the launch that works on it.
struct GenBatchImage {
  IOTable io;
  int32_t w, h;
  int32_t block0;
  int32_t pad;
};

// Partial results of one work-group of a generated kernel that reduces
// global operators: for each of its reduce operators in program order, a
// block of 32-bit words (even-sized, so 64-bit values stay aligned):
// HISTOGRAM / EQHIST the p0 counts, MINMAX {min, max}, MMCOUNT the two
// (value, count) keys of the extremes, SUMS the 64-bit sums of v and v^2.
__host__ __device__ inline int red_block_words(int kind, int p0) {
  switch (kind) {
    case OP_HISTOGRAM:
    case OP_EQHIST: return (p0 + 1) & ~1;
    case OP_MINMAX: return 2;
    default: return 4;  // MMCOUNT, SUMS
  }
}

__host__ __device__ inline int red_slot_words(const GProg& P) {
  int w = 0;
  for (int i = 0; i < P.nops; ++i)
    if (is_reduce_op(P.ops[i].kind)) w += red_block_words(P.ops[i].kind, P.ops[i].p0);
  return w;
}

}  // namespace hvx
