// Host-side launchers of the kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "hvx_desc.h"

namespace hvx {

// P: host copy (launch shape); dev_prog: the same program in device memory;
// num_cus sizes the grid of programs that reduce global operators
hipError_t launch_generic(const GProg& P, const GProg* dev_prog, const IOTable& io, int num_cus, hipStream_t s);
hipError_t launch_edge(const EdgeDesc& d, bool xcd, hipStream_t s);
hipError_t launch_corner(const CornerDesc& d, bool xcd, hipStream_t s);
hipError_t launch_gauss5(const Gauss5Desc& d, bool xcd, hipStream_t s);
// persistent: grid waves pull items from counter[0..1] (must start at zero);
// otherwise one wave per item.
// kinds: bit set of the kinds present (kind_bit); selects the compiled body set.
hipError_t launch_batch(const BatchImage* imgs, const uint16_t* item_img, int total, unsigned* counter, int grid,
                        bool persistent, int kinds, hipStream_t s);
int batch_waves_per_cu(int kinds);
int kind_bit(const BatchImage& bi);
// bytes of the zero-initialised counter block the persistent batch kernel needs
size_t batch_counter_bytes();

}  // namespace hvx
