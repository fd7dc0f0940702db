// The allocation-free entry point's workspace: a static device array per GPU.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace szsel {

// Size of the array (the largest workspace one allocation-free request may
// use: about 4.8 MB of fixed workspace plus 2 bytes per sampled value).
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;

// Looks up the device address of the array on `device` (which must be the
// current device) and zeroes it, once per device; later calls return at
// once.  Thread-safe.
hipError_t noalloc_setup(int device);

// Device address of the array on `device`, or NULL before noalloc_setup.
char *noalloc_scratch(int device);

}  // namespace szsel
