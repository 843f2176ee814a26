// Host-side launchers of the kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "hvx_desc.h"

namespace hvx {

hipError_t launch_generic(const GProg& P, const IOTable& io, hipStream_t s);
hipError_t launch_edge(const EdgeDesc& d, bool xcd, hipStream_t s);
hipError_t launch_gauss5(const Gauss5Desc& d, bool xcd, hipStream_t s);
// persistent: grid waves pull items from counter[0..1] (must start at zero);
// otherwise one wave per item.
hipError_t launch_batch(const BatchImage* imgs, const uint16_t* item_img, int total, unsigned* counter, int grid,
                        bool persistent, hipStream_t s);
int batch_waves_per_cu();

}  // namespace hvx
