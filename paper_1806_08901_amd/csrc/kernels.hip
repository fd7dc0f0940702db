// Per-request kernels of the estimator and their host-side launchers.
//   k_range : value range over all N values (Algorithm 1, line 2)
//   k_zfp   : ZFP bits and decoded error of the sampled blocks (Section 5.2)
//   k_sz    : Lorenzo/quantization codes and their histogram (Section 5.1)
// Each ends in a last-workgroup finalizer, so one request is three launches
// with no host round trip.
#include "estimator.hpp"
#include "launch.hpp"

namespace szsel {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_range(ReqDesc r) {
  __shared__ double s_lo[kWaves], s_hi[kWaves];
  __shared__ uint32_t s_bad[kWaves];
  __shared__ int s_last;
  RangeAcc<T> acc;
  range_scan<T>((const T *)r.field, 0, r.n, (int64_t)blockIdx.x * kThreads + threadIdx.x,
                (int64_t)gridDim.x * kThreads, acc);
  const RangePart p = range_reduce_wg<T>(acc, s_lo, s_hi, s_bad);
  if (threadIdx.x == 0) r.rpart[blockIdx.x] = p;
  if (!last_to_finish(&r.st->range_done, gridDim.x, &s_last)) return;
  RangeAcc<double> tot;
  for (int k = threadIdx.x; k < (int)gridDim.x; k += kThreads) {
    const RangePart q = r.rpart[k];
    tot.lo = fmin(tot.lo, q.lo);
    tot.hi = fmax(tot.hi, q.hi);
    tot.bad |= q.bad != 0;
  }
  const RangePart all = range_reduce_wg<double>(tot, s_lo, s_hi, s_bad);
  if (threadIdx.x == 0) {
    range_finalize_one(r, all.lo, all.hi, all.bad != 0);
    r.st->range_done = 0;
  }
}

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_zfp(ReqDesc r) {
  __shared__ TileLds L;
  __shared__ int s_last;
  if (skip_request(r.st)) return;
  const int minexp = r.st->minexp;
  for (int t = blockIdx.x; t < r.ntiles; t += gridDim.x) zfp_tile<T, D>(r, t, minexp, L);
  if (!last_to_finish(&r.st->zfp_done, gridDim.x, &s_last)) return;
  zfp_finalize<T, D>(r, L.red);
}

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_sz(ReqDesc r) {
  __shared__ TileLds L;
  __shared__ uint32_t s_hist[kHistWin];
  __shared__ int s_last;
  if (skip_request(r.st)) return;
  const double delta = r.st->delta, inv = r.st->inv, ebsz = r.st->eb_sz;
  hist_clear(s_hist);
  __syncthreads();
  for (int t = blockIdx.x; t < r.ntiles; t += gridDim.x)
    sz_tile<T, D>(r, t, delta, inv, ebsz, L, s_hist);
  __syncthreads();
  hist_flush(s_hist, r.hist);
  if (!last_to_finish(&r.st->sz_done, gridDim.x, &s_last)) return;
  sz_finalize<T, D>(r, L.red);
}

static hipError_t mark(const hipEvent_t *ev, int k, hipStream_t s) {
  return ev ? hipEventRecord(ev[k], s) : hipSuccess;
}

template <typename T, int D>
static hipError_t launch_tiles(const ReqDesc &r, hipStream_t s, const hipEvent_t *ev) {
  hipError_t e = hipSuccess;
  if (r.op != SZSEL_OP_SZ) {
    hipLaunchKernelGGL((k_zfp<T, D>), dim3(r.nzfp), dim3(kThreads), 0, s, r);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if ((e = mark(ev, 2, s)) != hipSuccess) return e;
  if (r.op != SZSEL_OP_ZFP) {
    hipLaunchKernelGGL((k_sz<T, D>), dim3(r.nsz), dim3(kThreads), 0, s, r);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return mark(ev, 3, s);
}

template <typename T>
static hipError_t launch_typed(const ReqDesc &r, hipStream_t s, const hipEvent_t *ev) {
  hipError_t e = mark(ev, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_range<T>), dim3(r.nrange), dim3(kThreads), 0, s, r);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = mark(ev, 1, s)) != hipSuccess) return e;
  switch (r.nd) {
    case 1: return launch_tiles<T, 1>(r, s, ev);
    case 2: return launch_tiles<T, 2>(r, s, ev);
    default: return launch_tiles<T, 3>(r, s, ev);
  }
}

hipError_t launch_request(const ReqDesc &r, hipStream_t s, const hipEvent_t *ev) {
  return r.dtype == SZSEL_F32 ? launch_typed<float>(r, s, ev) : launch_typed<double>(r, s, ev);
}

}  // namespace szsel
