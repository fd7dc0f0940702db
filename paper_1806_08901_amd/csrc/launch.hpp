// Host-visible launch interface between the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace szsel {

// Enqueues the three kernels of one request on stream s.
hipError_t launch_request(const ReqDesc &r, hipStream_t s);

}  // namespace szsel
