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

}  // namespace hvx
