// Host-side launchers of the global-operator kernels (global.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hvx_desc.h"

namespace hvx {

// One image as the global kernels read it: rows of `pitch` bytes (a multiple
// of 64) from a 16-byte aligned base; `bpp` bytes per element (1 or 2).
struct GlobalImg {
  const uint8_t* base;
  int64_t pitch;
  int32_t w, h, bpp;
};

hipError_t launch_histogram(const GlobalImg& im, int num_bins, int offset, int range, uint32_t* counts,
                            hipStream_t s);
hipError_t launch_min_max(const GlobalImg& im, int32_t* min_max, hipStream_t s);
// min_max plus the counts of pixels equal to each: result[0..3]
hipError_t launch_min_max_count(const GlobalImg& im, int32_t* result, hipStream_t s);
// min_max_count plus up to `cap` (x, y) locations of each extreme
hipError_t launch_min_max_loc(const GlobalImg& im, int32_t* result, uint32_t* lmin, uint32_t* lmax, uint32_t cap,
                              hipStream_t s);
// histogram equalisation into `out` (same size, U8); workspace: 1280 bytes
hipError_t launch_equalize_hist(const GlobalImg& im, uint8_t* out, int64_t out_pitch, void* workspace,
                                hipStream_t s);
hipError_t launch_mean_std_dev(const GlobalImg& im, void* result, hipStream_t s);
// the location pass of min_max_loc alone, after a min_max_count into `result`
hipError_t launch_extreme_locs(const GlobalImg& im, int32_t* result, uint32_t* lmin, uint32_t* lmax, uint32_t cap,
                               hipStream_t s);
// result[4..5] := min(result[4..5], cap): the locations each list holds
hipError_t launch_clamp_slots(int32_t* result, uint32_t cap, hipStream_t s);
// histogram and EqualizeHist mapping into `workspace` (counts, then the table)
hipError_t launch_equalize_mapping(const GlobalImg& im, void* workspace, hipStream_t s);
// starting value and final step of a global operator (OP_*) that fused
// kernels reduce into `result`
hipError_t launch_reduce_init(int kind, void* result, int num_bins, hipStream_t s);
hipError_t launch_reduce_finish(int kind, void* result, long long npix, hipStream_t s);
// The partial results a generated reducing kernel left in `ws` (nslots
// slots of slot_words words, red_slot_words) merged into the results of the
// program's reduce operators (between launch_reduce_init and _finish).
hipError_t launch_merge_partials(const GProg* dev_prog, const IOTable& io, const uint32_t* ws, int nslots,
                                 int slot_words, hipStream_t s);
// n uint32 words of device memory set to zero
hipError_t launch_zero_words(void* p, int n, hipStream_t s);

// Bytes of the fixed device array that replaces the EqualizeHist workspace
// (256 uint32 counts, then the 256-byte mapping).
constexpr size_t kEqualizeScratchBytes = 1280;
// Device address of that array on `device`, which must be the current
// device; resolved on the first call per device, then cached.
hipError_t equalize_scratch(int device, void** ptr);

}  // namespace hvx
