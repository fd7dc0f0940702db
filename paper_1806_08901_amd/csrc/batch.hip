// Batched execution: every request gets its own workspace region so that all
// of them can be in flight at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "batch.hpp"
#include "launch.hpp"

namespace szsel {

struct BatchState {
  char *fixed = nullptr;  // request_fixed_bytes() per request index, zeroed on allocation
  size_t nfixed = 0;      // request indices the fixed buffer holds
  char *var = nullptr;
  size_t var_cap = 0;
  szsel_result *res = nullptr;  // contiguous results for one copy back
  size_t nres = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void batch_destroy(BatchState *bs) {
  if (!bs) return;
  if (bs->fixed) (void)hipFree(bs->fixed);
  if (bs->var) (void)hipFree(bs->var);
  if (bs->res) (void)hipFree(bs->res);
  if (bs->done) (void)hipEventDestroy(bs->done);
  delete bs;
}

static hipError_t grow(char *&buf, size_t &have, size_t want, bool zero) {
  (void)hipDeviceSynchronize();
  if (buf) (void)hipFree(buf);
  buf = nullptr;
  have = 0;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e == hipSuccess && zero) e = hipMemset(p, 0, want);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (p) (void)hipFree(p);
    return e;
  }
  buf = (char *)p;
  have = want;
  return hipSuccess;
}

int batch_run(BatchState *&bs, int device, int ncu, size_t budget, std::vector<ReqDesc> &descs,
              szsel_result *out, hipStream_t s, std::string &msg) {
  (void)ncu;
  (void)device;
  const size_t n = descs.size();
  const size_t fixed = request_fixed_bytes();
  std::vector<size_t> voff(n);
  size_t var = 0;
  for (size_t i = 0; i < n; i++) {
    voff[i] = var;
    var = align_up(var + request_var_bytes(descs[i]), 256);
  }
  if (!bs) {
    bs = new BatchState();
    if (hipEventCreateWithFlags(&bs->done, hipEventDisableTiming) != hipSuccess) {
      msg = "hipEventCreate failed";
      return SZSEL_EHIP;
    }
  }
  const size_t want_fixed = n > bs->nfixed ? n : bs->nfixed;
  const size_t total = want_fixed * fixed + (var > bs->var_cap ? var : bs->var_cap) +
                       sizeof(szsel_result) * (n > bs->nres ? n : bs->nres);
  if (total > budget) {
    msg = "batch workspace of " + std::to_string(total) + " bytes exceeds the budget";
    return SZSEL_ENOMEM;
  }
  hipError_t e = hipSuccess;
  if (n > bs->nfixed) {
    size_t have = 0;
    e = grow(bs->fixed, have, n * fixed, true);
    bs->nfixed = e == hipSuccess ? n : 0;
    bs->used = false;
  }
  if (e == hipSuccess && var > bs->var_cap) e = grow(bs->var, bs->var_cap, var, false);
  if (e == hipSuccess && n > bs->nres) {
    char *p = (char *)bs->res;
    size_t have = 0;
    e = grow(p, have, sizeof(szsel_result) * n, false);
    bs->res = (szsel_result *)p;
    bs->nres = e == hipSuccess ? n : 0;
  }
  if (e != hipSuccess) {
    msg = std::string("batch workspace: ") + hipGetErrorString(e);
    return SZSEL_ENOMEM;
  }
  if (bs->used) e = hipStreamWaitEvent(s, bs->done, 0);
  for (size_t i = 0; i < n && e == hipSuccess; i++) {
    ReqDesc &r = descs[i];
    bind_request_workspace(r, bs->fixed + i * fixed, bs->var + voff[i]);
    r.res = bs->res + i;
    e = launch_request(r, s);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, bs->res, sizeof(szsel_result) * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(bs->done, s);
  if (e != hipSuccess) {
    msg = std::string("batch launch: ") + hipGetErrorString(e);
    return SZSEL_EHIP;
  }
  bs->used = true;
  return SZSEL_OK;
}

}  // namespace szsel
