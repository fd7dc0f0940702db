// Batched execution of many requests (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "device.hpp"

namespace szsel {

struct BatchState;

// Runs every request of `descs` (already planned) on stream s and copies the
// results to out[0..n).  `bs` is created or grown on demand.
int batch_run(BatchState *&bs, int device, int ncu, size_t budget, std::vector<ReqDesc> &descs,
              szsel_result *out, hipStream_t s, std::string &msg);

void batch_destroy(BatchState *bs);

}  // namespace szsel
