// Kernels generated for one fused group and compiled at run time.
//
// The tile interpreter (k_generic) runs any verified group but decides every
// operator, format, border and window offset per pixel.  The source-to-source
// step of Section 6 instead emits a kernel per fused group in which all of
// these are constants: here the group's program is written out as HIP
// source, compiled by hipRTC for the device's architecture and cached per
// process, so a graph structure is compiled once however often it is
// verified.  The generated kernel takes the same arguments as the
// interpreter (the device copy of the program, for the image size and the
// reduction epilogue, and the I/O table).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "gen_abi.h"
#include "hvx_desc.h"

namespace hvx {

struct GenKernel;

// Launch shape of a generated kernel.
enum GenForm : int32_t {
  GEN_POINTS = 1,  // point operators only: four pixels of one row per thread, no LDS
  GEN_TILES = 2,   // LDS tiles with halos; work-groups loop over tiles when the group reduces
};

struct GenSource {
  std::string text;
  int form = 0;
  int tw = 0, th = 0;  // output tile (GEN_TILES)
  bool red = false;    // reduces global operators over the image
  int lds_words = 0;   // static LDS of one work-group
};

// Whether a program is run by a generated kernel: everything except the
// single operators that the interpreter's own one-operator kernels already
// run with constant operators (a built-in point operator; a built-in local
// operator on U8 or F32 other than Convolve and NonLinearFilter, whose masks
// that kernel reads at run time).
bool gen_wanted(const GProg& P);

// Emit the kernel of program P with an output tile of tw x th (0: the
// largest that fits the LDS budget).  Bit i of `stream` marks value i as an
// output that no later kernel reads (written with non-temporal stores).
// False, with the reason, if P cannot be generated at that tile.
bool gen_source(const GProg& P, int tw, int th, uint32_t stream, GenSource* out, std::string* why);

// Compile (or find in the process cache) the kernel for `src`.  Null, with
// the compiler's log, on failure.  Compiling needs no device.
const GenKernel* gen_compile(const GenSource& src, std::string* why);

// Load the kernel's code object on the current device (once per device).
hipError_t gen_load(const GenKernel* k, int device);

// Launch on stream s (gen_load must have succeeded on the current device).
// A kernel that reduces global operators (not gen_batchable) writes one slot
// of red_slot_words(P) words per work-group, gen_blocks of them, to `ws`.
hipError_t gen_launch(const GenKernel* k, int device, const GProg& P, const GProg* dev_prog, const IOTable& io,
                      int num_cus, hipStream_t s, uint32_t* ws);

// Tile of a generated kernel (0 x 0 for the point form).
void gen_tile(const GenKernel* k, int* tw, int* th);

// Work-groups the kernel launches for one w x h image when run over a batch
// (one per tile, or one per 1024 pixels of a row for the point form).
long long gen_blocks(const GenKernel* k, int w, int h);

// Whether one launch can run the kernel over a batch of images (a kernel
// that reduces global operators cannot: each image has its own result).
bool gen_batchable(const GenKernel* k);

// One launch over n images: `imgs` in device memory, image i's work-groups
// starting at imgs[i].block0, `blocks` in all.
hipError_t gen_launch_batch(const GenKernel* k, int device, const GenBatchImage* imgs, int n, long long blocks,
                            hipStream_t s);

}  // namespace hvx
