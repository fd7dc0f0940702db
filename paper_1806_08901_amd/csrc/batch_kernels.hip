// Batched passes: one launch per pass covers every request of a batch (of
// a request group; the ZFP and SZ passes, whose kernels are templates of
// the dtype and rank, one launch per request class, and on two stream
// lanes every pass after the range scans one launch per class and lane).  The requests sit in a device table ordered so that
// each launch covers a contiguous range [c0, c1); first[i] is the first work
// item (workgroup) of table entry i in this pass, first[c1] the end.
#include "estimator.hpp"
#include "launch.hpp"

namespace szsel {

// Stages the prefix counts first[c0..c1] of a launch in LDS.
__device__ inline void batch_stage(const uint32_t *first, int c0, int c1, uint32_t *s_first) {
  for (int k = threadIdx.x; k <= c1 - c0; k += blockDim.x) s_first[k] = first[c0 + k];
  __syncthreads();
}

// Table entry of work item g (counted from the launch's first item) and the
// item's index within its request: the last entry whose start is <= g
// (entries with no items are skipped that way).
__device__ inline int batch_find(const uint32_t *s_first, int c0, int c1, uint32_t g, int &local) {
  const uint32_t a = s_first[0] + g;
  int lo = 0, hi = c1 - c0 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_first[mid] <= a) lo = mid; else hi = mid - 1;
  }
  local = (int)(a - s_first[lo]);
  return c0 + lo;
}

// One work item per workgroup.
// Both are the same in every thread; saying so keeps the request's fields
// in scalar registers (one copy per wave, not per lane).
__device__ inline int batch_item(const uint32_t *first, int c0, int c1, uint32_t *s_first, int &local) {
  batch_stage(first, c0, c1, s_first);
  const int i = batch_find(s_first, c0, c1, blockIdx.x, local);
  local = __builtin_amdgcn_readfirstlane(local);
  return __builtin_amdgcn_readfirstlane(i);
}

// Range chunks of fields of either dtype: one per workgroup, or (a grid
// smaller than the chunk count) every workgroup loops over chunks
// blockIdx.x, + gridDim.x, ... in table order, so that a few resident
// workgroups per CU scan the whole launch.
__global__ __launch_bounds__(kThreads) void kb_range(const ReqDesc *__restrict__ tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_first[kMaxBatch + 1];
  batch_stage(first, c0, c1, s_first);
  const uint32_t items = s_first[c1 - c0] - s_first[0];
  for (uint32_t g = blockIdx.x; g < items; g += gridDim.x) {
    int local;
    const int i = __builtin_amdgcn_readfirstlane(batch_find(s_first, c0, c1, g, local));
    local = __builtin_amdgcn_readfirstlane(local);
    // (either dtype: one launch scans every field of the request group)
    if (tab[i].dtype == SZSEL_F32)
      range_wg<float>(tab[i], local, L);
    else
      range_wg<double>(tab[i], local, L);
    __syncthreads();
  }
}

template <typename T, int D, bool VEC, bool EC>
__global__ __launch_bounds__(kWave, (kZfpWavesPerSimd<T, D, EC>)) void kb_zfp(const ReqDesc *__restrict__ tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const int i = batch_item(first, c0, c1, s_first, local);
  const ReqDesc &r = tab[i];
  if (skip_request(r.st)) return;
  zfp_wg<T, D, VEC, EC>(r, local, L);
}

template <typename T, int D, bool VEC>
__global__ __launch_bounds__(kThreads, (kSzWavesPerSimd<T, D>)) void kb_sz(const ReqDesc *__restrict__ tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_hist[kHistWin];
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const int i = batch_item(first, c0, c1, s_first, local);
  const ReqDesc &r = tab[i];
  if (skip_request(r.st)) return;
  sz_wg<T, D, VEC>(r, local, L, s_hist);
}

// The overflow and entropy passes have many small items, and how many a
// request has is known only on the device (overflow slices, chunks with
// codes): a grid of a few workgroups per CU first numbers the items of the
// launch's requests (every workgroup reads the counts and scans them) and
// then loops over them.  Requests without items in this pass (first[i + 1]
// == first[i]) and skipped requests count 0.  s_pre[i] is request c0 + i's
// first item, s_pre[c1 - c0] the total.
template <int NT, typename F>
__device__ inline uint32_t batch_device_items(const ReqDesc *tab, const uint32_t *first, int c0, int c1,
                                              uint32_t *s_pre, uint32_t *s_wave, F count) {
  const int n = c1 - c0, t = threadIdx.x;
  constexpr int kPer = (kMaxBatch + NT - 1) / NT;  // requests per thread
  uint32_t cnt[kPer], sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const int i = t * kPer + k;
    cnt[k] = 0;
    if (i < n && first[c0 + i + 1] != first[c0 + i]) {
      const ReqDesc &r = tab[c0 + i];
      if (!skip_request(r.st)) cnt[k] = count(r);
    }
    sum += cnt[k];
  }
  uint32_t inc = sum;
  const int lane = t & (kWave - 1), wv = t / kWave;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == kWave - 1) s_wave[wv] = inc;
  __syncthreads();
  uint32_t base = inc - sum;
  for (int q = 0; q < wv; q++) base += s_wave[q];
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const int i = t * kPer + k;
    if (i <= n) s_pre[i] = base;
    base += cnt[k];
  }
  if (t == NT - 1 && n == kMaxBatch) s_pre[n] = base;
  __syncthreads();
  return s_pre[n];
}

// The request (index from c0) whose items hold item g: the last one whose
// first item is <= g.
__device__ inline int batch_owner(const uint32_t *s_pre, int n, uint32_t g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_pre[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);  // the same in every thread
}

__global__ __launch_bounds__(kOvfThreads) void kb_ovf(const ReqDesc *__restrict__ tab, const uint32_t *first, int c0, int c1) {
  __shared__ uint32_t s_cnt[kOvfBins];
  __shared__ uint32_t s_pre[kMaxBatch + 1];
  __shared__ uint32_t s_wave[kOvfThreads / kWave];
  const uint32_t items = batch_device_items<kOvfThreads>(tab, first, c0, c1, s_pre, s_wave, [](const ReqDesc &r) {
    return get_u32(&r.st->ovf_slices) * (uint32_t)kOvfRanges;
  });
  for (uint32_t g = blockIdx.x; g < items; g += gridDim.x) {
    const int lo = batch_owner(s_pre, c1 - c0, g);
    ovf_wg(tab[c0 + lo], (int)(g - s_pre[lo]), s_cnt);
    __syncthreads();
  }
}

// Items: the chunks the entropy pass works on (ent_chunks), in bit order.
__global__ __launch_bounds__(kThreads) void kb_ent(const ReqDesc *__restrict__ tab, const uint32_t *first, int c0, int c1) {
  __shared__ TileLds L;
  __shared__ uint32_t s_pre[kMaxBatch + 1];
  __shared__ uint32_t s_wave[kWaves];
  const uint32_t items = batch_device_items<kThreads>(tab, first, c0, c1, s_pre, s_wave, [](const ReqDesc &r) {
    return (uint32_t)__popcll(ent_chunks(r));
  });
  for (uint32_t g = blockIdx.x; g < items; g += gridDim.x) {
    const int lo = batch_owner(s_pre, c1 - c0, g);
    const ReqDesc &r = tab[c0 + lo];
    const uint64_t chunks = ent_chunks(r);
    uint64_t m = chunks;
    for (uint32_t k = g - s_pre[lo]; k > 0; k--) m &= m - 1;  // drop the lower chunks
    ent_wg(r, __ffsll((long long)m) - 1, chunks, L);
    __syncthreads();
  }
}

template <typename T, int D>
__global__ __launch_bounds__(kHuffThreads) void kb_huff(const ReqDesc *__restrict__ tab, const uint32_t *first, int c0, int c1) {
  __shared__ HuffLds S;
  __shared__ uint32_t s_first[kMaxBatch + 1];
  int local;
  const ReqDesc &r = tab[batch_item(first, c0, c1, s_first, local)];
  if (!skip_request(r.st)) huff_wg<T, D>(r, S);
}

template <typename T, int D>
static hipError_t launch_typed(const BatchLaunch &a, hipStream_t s) {
  const dim3 grid(a.grid ? a.grid : a.items);
  switch (a.pass) {
    case kBatchZfp:
      if (a.ec) {
        if (a.vec)
          hipLaunchKernelGGL((kb_zfp<T, D, true, true>), grid, dim3(kWave), 0, s, a.tab, a.first, a.c0, a.c1);
        else
          hipLaunchKernelGGL((kb_zfp<T, D, false, true>), grid, dim3(kWave), 0, s, a.tab, a.first, a.c0, a.c1);
      } else if (a.vec) {
        hipLaunchKernelGGL((kb_zfp<T, D, true, false>), grid, dim3(kWave), 0, s, a.tab, a.first, a.c0, a.c1);
      } else {
        hipLaunchKernelGGL((kb_zfp<T, D, false, false>), grid, dim3(kWave), 0, s, a.tab, a.first, a.c0, a.c1);
      }
      break;
    case kBatchSz:
      if (a.vec)
        hipLaunchKernelGGL((kb_sz<T, D, true>), grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      else
        hipLaunchKernelGGL((kb_sz<T, D, false>), grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      break;
    default:
      hipLaunchKernelGGL((kb_huff<T, D>), grid, dim3(kHuffThreads), 0, s, a.tab, a.first, a.c0, a.c1);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_pass(const BatchLaunch &a, hipStream_t s) {
  if (a.items == 0) return hipSuccess;
  // the range, overflow and entropy passes serve every dtype and rank in
  // one launch
  if (a.pass == kBatchRange || a.pass == kBatchOvf || a.pass == kBatchEnt) {
    const dim3 grid(a.grid ? a.grid : a.items);
    if (a.pass == kBatchRange)
      hipLaunchKernelGGL(kb_range, grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
    else if (a.pass == kBatchOvf)
      hipLaunchKernelGGL(kb_ovf, grid, dim3(kOvfThreads), 0, s, a.tab, a.first, a.c0, a.c1);
    else
      hipLaunchKernelGGL(kb_ent, grid, dim3(kThreads), 0, s, a.tab, a.first, a.c0, a.c1);
    return hipGetLastError();
  }
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
