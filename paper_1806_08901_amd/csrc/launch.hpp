// Host-visible launch interface between the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace szsel {

// Enqueues the kernels of one request on stream s.  When ev is not NULL,
// ev[0..5] are recorded before the range pass and after the range, ZFP, SZ,
// overflow-count and entropy passes (phase timers).
hipError_t launch_request(const ReqDesc &r, hipStream_t s, const hipEvent_t *ev = nullptr);

// Workspace of one request: a fixed part that must stay at the same place
// from one request to the next (state and counters, the self-cleaning
// histogram, result, chunk sums, overflow counts; zero-initialised once) and
// a variable part (per-workgroup partials, overflow regions).
size_t request_fixed_bytes();
size_t request_var_bytes(int nrange, int nzfp, int nsz, int64_t ovf_cap);
void bind_request_workspace(ReqDesc &r, char *fixed, char *var);

// Overflow-region capacity of a planned request (sblk * 4^d codes per SZ
// workgroup) and its variable workspace size.
inline int64_t request_ovf_capacity(const ReqDesc &r) {
  return ((int64_t)r.nsz * r.sblk) << (2 * r.nd);
}
inline size_t request_var_bytes(const ReqDesc &r) {
  return request_var_bytes(r.nrange, r.nzfp, r.nsz, request_ovf_capacity(r));
}

// One launch of a batched pass over table entries [c0, c1) (see
// batch_kernels.hip); `items` workgroups in total.
enum { kBatchRange = 0, kBatchZfp, kBatchSz, kBatchOvf, kBatchEnt, kBatchHuff, kBatchPasses };
struct BatchLaunch {
  int group, pass, dtype, nd, vec, ec;
  const ReqDesc *tab;
  const uint32_t *first;
  int c0, c1;
  uint32_t items;  // work items
  uint32_t grid;   // workgroups (the overflow and entropy passes loop over their items)
  int lane = 0;    // launches after the range scans: stream lane (0: the caller's stream, 1: the side stream)
};
hipError_t launch_batch_pass(const BatchLaunch &a, hipStream_t s);

// Launch shape knobs of the planner.  Any choice gives bit-identical
// results (every reduction is an aligned subtree of the same fixed tree);
// they only move the balance between parallelism and per-workgroup
// overheads, which the batch autotuner measures.
struct Tune {
  int sz_wgs_q = 8;          // SZ workgroups per request, in quarters of the CU count
  int zfp_chunk = 16;        // smallest ZFP chunk (sampled blocks per one-wave workgroup;
                             // layouts of one block per lane take at least 64)
  int zfp_waves = 64;        // ZFP waves aimed at per CU, for a request (single calls) or a
                             // launch class (batches); chunks grow until they are about that many
  int range_wgs_q = 4;       // range workgroups (scan chunks) per request, in quarters of the CU count
  int range_grid = 0;        // batches: 0 = one workgroup per range chunk; k > 0 = k workgroups
                             // per CU that loop over all the launch's chunks (a resident scan
                             // that leaves the other wave slots to the sampled passes)
  int groups = 1;            // batches: request groups pipelined on parallel streams
  int lanes = 2;             // batches of one request group: 1 = one stream; 2 = two stream
                             // lanes for the passes after the scans, launch classes dealt
                             // in turn (one class: cut at half the work); 3 = two lanes
                             // cut at half the work
  int ovf_slice = kOvfPerSlice;  // overflow codes per slice of the overflow pass
  int share = 0;             // batches: 0 = SZ and range counts per request, 1 = the SZ
                             // count is the batch's, 2 = both are the batch's, 3 = the SZ
                             // count is each launch class's (batches always deal the
                             // ZFP waves within each launch class)
  // set by the batch planner for one request from the batch's counts above
  // (never tuned or cached): nonzero = SZ workgroups, range workgroups, ZFP
  // waves aimed at
  int sz_target = 0;
  int range_target = 0;
  int zfp_target = 0;
};



}  // namespace szsel
