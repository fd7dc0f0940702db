// Host-visible launch interface between the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace szsel {

// Enqueues the kernels of one request on stream s.  When ev is not NULL,
// ev[0..3] are recorded before the range pass, after it, after the ZFP pass
// and after the SZ pass (phase timers).
hipError_t launch_request(const ReqDesc &r, hipStream_t s, const hipEvent_t *ev = nullptr);

// Device bytes of one request's workspace (state, per-workgroup partials of
// the three passes, 65536-bin histogram, result) for the given pass sizes,
// and the binding of a zero-initialised region of that size to r.
size_t request_workspace_bytes(int nrange, int nzfp, int nsz, int64_t ovf_cap);

// Overflow-region capacity of a planned request (sblk * 4^d codes per SZ
// workgroup) and its total workspace size.
inline int64_t request_ovf_capacity(const ReqDesc &r) {
  return ((int64_t)r.nsz * r.sblk) << (2 * r.nd);
}
inline size_t request_bytes(const ReqDesc &r) {
  return request_workspace_bytes(r.nrange, r.nzfp, r.nsz, request_ovf_capacity(r));
}
void bind_request_workspace(ReqDesc &r, char *base, int nrange, int nzfp, int nsz,
                            int64_t ovf_cap);

}  // namespace szsel
