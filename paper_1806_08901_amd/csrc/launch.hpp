// Host-visible launch interface between the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace szsel {

// Enqueues the kernels of one request on stream s.  When ev is not NULL,
// ev[0..3] are recorded before the range pass, after it, after the ZFP pass
// and after the SZ pass (phase timers).
hipError_t launch_request(const ReqDesc &r, hipStream_t s, const hipEvent_t *ev = nullptr);

}  // namespace szsel
