// Per-request kernels of the estimator and their host-side launchers.
//   k_range : value range over all N values (Algorithm 1's error bound)
//   k_zfp   : ZFP bits and decoded error of the sampled blocks (Section 5.2)
//   k_sz    : Lorenzo/quantization codes and their histogram (Section 5.1)
//   k_ovf   : counts the codes that fell outside the SZ pass's LDS window
//   k_ent   : entropy of the histogram, SZ bit-rate, selection (Eq. 5, Alg. 1)
//   k_huff  : exact Huffman cost of the histogram (when asked for)
// Passes with a cross-workgroup total end in a last-workgroup finalizer; a
// request is a chain of launches on one stream with no host round trip.
#include "estimator.hpp"
#include "launch.hpp"

namespace szsel {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_range(ReqDesc r) {
  __shared__ TileLds L;
  range_wg<T>(r, blockIdx.x, L);
}

// Two waves per SIMD (at most 256 registers each) so that every wave of a
// request's ZFP pass is resident at once; binary64 3-D blocks (64 64-bit
// coefficients) get one wave per SIMD and 512 registers instead, which
// spills a third as much and runs 1.8x faster.
// VEC: rows of 4 values start 16-byte aligned and are read as vectors.
// EC: the paper's point sub-sampling estimate instead of the exact one.
template <typename T, int D, bool VEC, bool EC>
__global__ __launch_bounds__(kWave, (kZfpWavesPerSimd<T, D, EC>)) void k_zfp(ReqDesc r) {
  __shared__ TileLds L;
  if (skip_request(r.st)) return;
  zfp_wg<T, D, VEC, EC>(r, blockIdx.x, L);
}

template <typename T, int D, bool VEC>
__global__ __launch_bounds__(kThreads, (kSzWavesPerSimd<T, D>)) void k_sz(ReqDesc r) {
  __shared__ TileLds L;
  __shared__ uint32_t s_hist[kHistWin];
  if (skip_request(r.st)) return;
  sz_wg<T, D, VEC>(r, blockIdx.x, L, s_hist);
}

__global__ __launch_bounds__(kOvfThreads) void k_ovf(ReqDesc r) {
  __shared__ uint32_t s_cnt[kOvfBins];
  if (skip_request(r.st)) return;
  ovf_wg(r, blockIdx.x, s_cnt);
}

__global__ __launch_bounds__(kThreads) void k_ent(ReqDesc r) {
  __shared__ TileLds L;
  if (skip_request(r.st)) return;
  const uint64_t chunks = ent_chunks(r);
  if ((chunks >> blockIdx.x) & 1u) ent_wg(r, blockIdx.x, chunks, L);
}

template <typename T, int D>
__global__ __launch_bounds__(kHuffThreads) void k_huff(ReqDesc r) {
  __shared__ HuffLds S;
  if (skip_request(r.st)) return;
  huff_wg<T, D>(r, S);
}

static hipError_t mark(const hipEvent_t *ev, int k, hipStream_t s) {
  return ev ? hipEventRecord(ev[k], s) : hipSuccess;
}

template <typename T, int D>
static hipError_t launch_tiles(const ReqDesc &r, hipStream_t s, const hipEvent_t *ev) {
  hipError_t e = hipSuccess;
  if (r.op != SZSEL_OP_SZ) {
    if (r.ec) {
      if (r.vec)
        hipLaunchKernelGGL((k_zfp<T, D, true, true>), dim3(r.nzfp), dim3(kWave), 0, s, r);
      else
        hipLaunchKernelGGL((k_zfp<T, D, false, true>), dim3(r.nzfp), dim3(kWave), 0, s, r);
    } else if (r.vec) {
      hipLaunchKernelGGL((k_zfp<T, D, true, false>), dim3(r.nzfp), dim3(kWave), 0, s, r);
    } else {
      hipLaunchKernelGGL((k_zfp<T, D, false, false>), dim3(r.nzfp), dim3(kWave), 0, s, r);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if ((e = mark(ev, 2, s)) != hipSuccess) return e;
  if (r.op != SZSEL_OP_ZFP) {
    if (r.vec)
      hipLaunchKernelGGL((k_sz<T, D, true>), dim3(r.nsz), dim3(kThreads), 0, s, r);
    else
      hipLaunchKernelGGL((k_sz<T, D, false>), dim3(r.nsz), dim3(kThreads), 0, s, r);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if ((e = mark(ev, 3, s)) != hipSuccess) return e;
  if (r.op != SZSEL_OP_ZFP) {
    hipLaunchKernelGGL(k_ovf, dim3(kOvfSlices * kOvfRanges), dim3(kOvfThreads), 0, s, r);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if ((e = mark(ev, 4, s)) != hipSuccess) return e;
  if (r.op != SZSEL_OP_ZFP) {
    hipLaunchKernelGGL(k_ent, dim3(kEntWgs), dim3(kThreads), 0, s, r);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (r.huff) {
      hipLaunchKernelGGL((k_huff<T, D>), dim3(1), dim3(kHuffThreads), 0, s, r);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return mark(ev, 5, s);
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

// ---------------------------------------------------------------------------
// Workspace of one request
// ---------------------------------------------------------------------------
static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static size_t parts_bytes(int n) { return align_up((size_t)(n > 0 ? n : 1) * 8, 256) * 4; }


// Fixed part: what must persist between requests at the same place (state,
// the completion counters, the self-cleaning histogram) and the fixed-size
// buffers.  Variable part: per-workgroup partials and overflow regions,
// fully rewritten by every request.
static size_t group_parts_bytes() { return align_up((size_t)kMaxGroups * 8, 256) * 4; }

size_t request_fixed_bytes() {
  return align_up(sizeof(ReqState), 256) + align_up(sizeof(PassSync) * kPasses, 256) +
         align_up(sizeof(uint32_t) * kBins * kHistCopies, 256) + align_up(sizeof(szsel_result), 256) +
         parts_bytes(kEntWgs) + group_parts_bytes() * kPasses +
         align_up(sizeof(uint32_t) * kBins, 256) + align_up(sizeof(uint32_t) * kBins, 256);
}

size_t request_var_bytes(int nrange, int nzfp, int nsz, int64_t ovf_cap) {
  return parts_bytes(nrange) + parts_bytes(nzfp) + parts_bytes(nsz) +
         align_up(sizeof(uint16_t) * (size_t)(ovf_cap > 0 ? ovf_cap : 1), 256);
}

static Parts bind_parts(char *&p, int n) {
  const size_t one = align_up((size_t)(n > 0 ? n : 1) * 8, 256);
  Parts q;
  q.sse = (double *)p;
  q.err = (double *)(p + one);
  q.a = (uint64_t *)(p + 2 * one);
  q.b = (uint64_t *)(p + 3 * one);
  p += 4 * one;
  return q;
}

void bind_request_workspace(ReqDesc &r, char *fixed, char *var) {
  char *p = fixed;
  r.st = (ReqState *)p;
  p += align_up(sizeof(ReqState), 256);
  r.sync = (PassSync *)p;
  p += align_up(sizeof(PassSync) * kPasses, 256);
  r.hist = (uint32_t *)p;
  p += align_up(sizeof(uint32_t) * kBins * kHistCopies, 256);
  r.res = (szsel_result *)p;
  p += align_up(sizeof(szsel_result), 256);
  r.ep = bind_parts(p, kEntWgs);
  for (int k = 0; k < kPasses; k++) r.grp[k] = bind_parts(p, kMaxGroups);
  r.ovf_hist = (uint32_t *)p;
  p += align_up(sizeof(uint32_t) * kBins, 256);
  r.hfinal = (uint32_t *)p;
  p = var;
  r.rp = bind_parts(p, r.nrange);
  r.zp = bind_parts(p, r.nzfp);
  r.sp = bind_parts(p, r.nsz);
  r.ovf = (uint16_t *)p;
}

}  // namespace szsel
