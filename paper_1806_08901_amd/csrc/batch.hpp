// Batched execution of many requests (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "device.hpp"
#include "launch.hpp"

struct szsel_ctx;

namespace szsel {

struct BatchState;

// Phase timer of batched launches: an event pair around every launch,
// tagged 2 * pass + dtype (pass numbering of BatchLaunch, dtype SZSEL_F32 /
// SZSEL_F64).  Events are created on demand and reused after a drain.
struct LaunchTimer {
  std::vector<hipEvent_t> ev;  // 2 per recorded launch
  std::vector<int> tag;
  size_t used = 0;             // launches recorded since the last drain
};

struct BatchOptions {
  bool autotune = false;  // time launch-shape candidates per batch shape, keep the fastest
  bool graph = true;      // capture the launches as a HIP graph and replay it
  Tune fixed;             // the schedule used without autotuning
  LaunchTimer *timer = nullptr;  // non-NULL: time every launch (eager launches, no graph)
};

// Plans and runs the n requests on stream s and copies the results to
// out[0..n) (asynchronously).  `bs` is created or grown on demand; it is
// reused only after its previous batch has finished.  `budget` caps its
// device memory.
int batch_run(szsel_ctx *ctx, int ncu, BatchState *&bs, size_t budget, const szsel_request *reqs, int n,
              szsel_result *out, hipStream_t s, const BatchOptions &opt, std::string &msg);

// Creates `bs` if needed and grows its buffers to hold nreq requests and
// var_bytes of variable workspace, so that later batches within that size
// allocate nothing (an allocation or release synchronises the device).
// Then enqueues one kernel launch, one host-to-device and one
// device-to-host transfer on stream s (the caller waits for them): the
// runtime sets up a stream's queues at its first launch and transfers, and
// more copy queues when transfers first run on several streams at once,
// which takes milliseconds.  Waits for the state's previous batch.
int batch_reserve(BatchState *&bs, int nreq, size_t var_bytes, hipStream_t s, std::string &msg);

void batch_destroy(BatchState *bs);

// CU count of the context's device.
int ctx_ncu(const szsel_ctx *ctx);

// Architecture name of the context's device (gcnArchName).
const char *ctx_arch(const szsel_ctx *ctx);

// The argument checks of one request (no device, no context): SZSEL_OK or a
// negative code with the reason in `why`.
int check_request(int op, const void *field, const int64_t *dims, int nd, int dtype, double eb,
                  int eb_mode, const int32_t *stride, std::string &why);

// Plans one request (checks it, then sets its launch shape from `tu`);
// errors go to the context's last error.
int plan_request(szsel_ctx *ctx, int op, const void *field, const int64_t *dims, int nd, int dtype,
                 double eb, int eb_mode, const int32_t *stride, const Tune &tu, ReqDesc &r);

// Device bytes a batch state needs per request of plan r (its share of
// the fixed and variable workspace, result, table entry and prefix counts;
// what batch_run checks against its budget, rounded up).
size_t batch_request_bytes(const ReqDesc &r);

// Device bytes held by a batch state (0 for NULL).
size_t batch_state_bytes(const BatchState *bs);

}  // namespace szsel
