// Workspace of the allocation-free entry point (szsel_select_noalloc): one
// request's fixed and variable workspace carved out of a static device
// array of fixed size, instead of memory the context allocates.
//
// Every GPU the library runs on holds its own copy of the array until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy (in host code it names a host-side stand-in): the device address of
// each GPU's copy is looked up once, at context creation with that device
// current, and kept here per device.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "noalloc.hpp"

static __device__ __align__(256) unsigned char scratch[szsel::kNoallocScratchBytes];

namespace szsel {
namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
char *g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// Zero fill of n 16-byte words (a kernel, not a memset node, so that the
// clearing is safe wherever it is enqueued).
__global__ __launch_bounds__(256) void k_scratch_clear(uint4 *p, size_t n) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

hipError_t noalloc_setup(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p || (uintptr_t)p % 256) return hipErrorInvalidSymbol;
  // the kernels keep the fixed part of a workspace clean from one request
  // to the next; it starts out zero
  hipLaunchKernelGGL(k_scratch_clear, dim3(1024), dim3(256), 0, nullptr, (uint4 *)p,
                     kNoallocScratchBytes / sizeof(uint4));
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return e;
  g_scratch[device] = (char *)p;
  return hipSuccess;
}

char *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (device < 0 || device >= kMaxDevices) return nullptr;
  return g_scratch[device];
}

}  // namespace szsel
