// Batched execution: every request gets its own workspace region so that all
// of them can be in flight at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "batch.hpp"
#include "launch.hpp"

namespace szsel {

struct BatchState {
  char *mem = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }



void batch_destroy(BatchState *bs) {
  if (!bs) return;
  if (bs->mem) (void)hipFree(bs->mem);
  if (bs->done) (void)hipEventDestroy(bs->done);
  delete bs;
}

int batch_run(BatchState *&bs, int device, int ncu, size_t budget, std::vector<ReqDesc> &descs,
              szsel_result *out, hipStream_t s, std::string &msg) {
  (void)ncu;
  const size_t n = descs.size();
  // layout: results first (one contiguous copy back), then one workspace
  // region per request
  size_t off = align_up(sizeof(szsel_result) * n, 256);
  std::vector<size_t> base(n);
  for (size_t i = 0; i < n; i++) {
    const ReqDesc &r = descs[i];
    base[i] = off;
    off = align_up(off + request_bytes(r), 256);
  }
  const size_t need = off;
  if (!bs) {
    bs = new BatchState();
    if (hipEventCreateWithFlags(&bs->done, hipEventDisableTiming) != hipSuccess) {
      msg = "hipEventCreate failed";
      return SZSEL_EHIP;
    }
  }
  if (need > bs->cap) {
    if (need > budget) {
      msg = "batch workspace of " + std::to_string(need) + " bytes exceeds the budget";
      return SZSEL_ENOMEM;
    }
    if (bs->mem) {
      (void)hipDeviceSynchronize();
      (void)hipFree(bs->mem);
      bs->mem = nullptr;
      bs->cap = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e == hipSuccess) e = hipMemset(p, 0, need);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      if (p) (void)hipFree(p);
      msg = std::string("batch workspace: ") + hipGetErrorString(e);
      return SZSEL_ENOMEM;
    }
    bs->mem = (char *)p;
    bs->cap = need;
    bs->used = false;
  }
  hipError_t e = hipSuccess;
  if (bs->used) e = hipStreamWaitEvent(s, bs->done, 0);
  szsel_result *res = (szsel_result *)bs->mem;
  for (size_t i = 0; i < n && e == hipSuccess; i++) {
    ReqDesc &r = descs[i];
    bind_request_workspace(r, bs->mem + base[i], r.nrange, r.nzfp, r.nsz, request_ovf_capacity(r));
    r.res = res + i;
    e = launch_request(r, s);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, res, sizeof(szsel_result) * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(bs->done, s);
  if (e != hipSuccess) {
    msg = std::string("batch launch: ") + hipGetErrorString(e);
    return SZSEL_EHIP;
  }
  bs->used = true;
  (void)device;
  return SZSEL_OK;
}

}  // namespace szsel
