// Batched passes: one launch per pass (and request class) covers every
// request of a batch.  The requests sit in a device table ordered so that
// each launch covers a contiguous range [c0, c1); first[i] is the first work
// item (workgroup) of table entry i in this pass, first[c1] the end.
#include "estimator.hpp"
#include "launch.hpp"

namespace szsel {

// Table entry of this workgroup's work item and the item's index within
// its request: the prefix counts are staged in LDS and searched (entries
// with no items are skipped by taking the last entry whose start is <= g).
__device__ inline int batch_item(const uint32_t *first, int c0, int c1, uint32_t *s_first, int &local) {
  const int n = c1 - c0;
  for (int k = threadIdx.x; k <= n; k += blockDim.x) s_first[k] = first[c0 + k];
  __syncthreads();
  const uint32_t g = s_first[0] + blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_first[mid] <= g) lo = mid; else hi = mid - 1;
  }
  local = (int)(g - s_first[lo]);
  __syncthreads();
  return c0 + lo;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void kb_range(const ReqDesc *tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const int i = batch_item(first, c0, c1, s_first, local);
  range_wg<T>(tab[i], local, L);
}

template <typename T, int D, bool VEC>
__global__ __launch_bounds__(kWave, 2) void kb_zfp(const ReqDesc *tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const int i = batch_item(first, c0, c1, s_first, local);
  const ReqDesc &r = tab[i];
  if (skip_request(r.st)) return;
  zfp_wg<T, D, VEC>(r, local, L);
}

template <typename T, int D, bool VEC>
__global__ __launch_bounds__(kThreads) void kb_sz(const ReqDesc *tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_hist[kHistWin];
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const int i = batch_item(first, c0, c1, s_first, local);
  const ReqDesc &r = tab[i];
  if (skip_request(r.st)) return;
  sz_wg<T, D, VEC>(r, local, L, s_hist);
}

template <int D>
__global__ __launch_bounds__(kThreads) void kb_ovf(const ReqDesc *tab, const uint32_t *first, int c0, int c1) {
  __shared__ uint32_t s_cnt[kOvfBins];
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const int i = batch_item(first, c0, c1, s_first, local);
  const ReqDesc &r = tab[i];
  if (skip_request(r.st)) return;
  ovf_wg<D>(r, local, s_cnt);
}

template <typename T, int D>
__global__ __launch_bounds__(kThreads) void kb_ent(const ReqDesc *tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const int i = batch_item(first, c0, c1, s_first, local);
  const ReqDesc &r = tab[i];
  if (skip_request(r.st)) return;
  ent_wg<T, D>(r, local, L);
}

template <typename T, int D>
static hipError_t launch_typed(const BatchLaunch &a, hipStream_t s) {
  const dim3 grid(a.items);
  switch (a.pass) {
    case kBatchRange:
      hipLaunchKernelGGL((kb_range<T>), grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      break;
    case kBatchZfp:
      if (a.vec)
        hipLaunchKernelGGL((kb_zfp<T, D, true>), grid, dim3(kWave), 0, s, a.tab, a.first, a.c0, a.c1);
      else
        hipLaunchKernelGGL((kb_zfp<T, D, false>), grid, dim3(kWave), 0, s, a.tab, a.first, a.c0, a.c1);
      break;
    case kBatchSz:
      if (a.vec)
        hipLaunchKernelGGL((kb_sz<T, D, true>), grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      else
        hipLaunchKernelGGL((kb_sz<T, D, false>), grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      break;
    case kBatchOvf:
      hipLaunchKernelGGL((kb_ovf<D>), grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      break;
    default:
      hipLaunchKernelGGL((kb_ent<T, D>), grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_pass(const BatchLaunch &a, hipStream_t s) {
  if (a.items == 0) return hipSuccess;
  if (a.dtype == SZSEL_F32) {
    switch (a.nd) {
      case 1: return launch_typed<float, 1>(a, s);
      case 2: return launch_typed<float, 2>(a, s);
      default: return launch_typed<float, 3>(a, s);
    }
  }
  switch (a.nd) {
    case 1: return launch_typed<double, 1>(a, s);
    case 2: return launch_typed<double, 2>(a, s);
    default: return launch_typed<double, 3>(a, s);
  }
}

}  // namespace szsel
