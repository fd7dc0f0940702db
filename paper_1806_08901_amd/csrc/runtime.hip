// Host runtime behind the C ABI of include/szsel.h: argument checking,
// request planning (tiles, grid sizes), workspace slots, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "batch.hpp"
#include "compress.hpp"
#include "launch.hpp"
#include "noalloc.hpp"
#include "szsel.h"

using namespace szsel;

namespace {

constexpr int kSlots = 4;
constexpr int kBatchSlots = 4;  // batch states in rotation (batches in flight)
constexpr int kPhases = 5;  // range, ZFP, SZ, overflow count, entropy
constexpr int kEv = kPhases + 1;

struct Slot {
  char *mem = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};

}  // namespace

struct szsel_ctx {
  int device = 0;
  int ncu = 256;
  std::string arch;  // gcnArchName of the device
  size_t budget = 0;
  size_t used_bytes = 0;
  Slot slots[kSlots];
  int next = 0;
  double sz_offset = 0.5;
  int huffman = 0;
  int ec = 0;
  char *zc_ws = nullptr;  // Step 4 workspace (grown on demand)
  size_t zc_ws_bytes = 0;
  szsel_debug dbg{};
  bool dbg_armed = false;
  std::string err;
  BatchState *batch[kBatchSlots] = {};
  size_t batch_bytes[kBatchSlots] = {};
  int bnext = 0;
  BatchOptions bopt;
  // phase timers
  bool prof = false;
  std::vector<hipEvent_t> prof_events;  // kPhases + 1 per recorded call
  std::vector<int> prof_dtype;          // dtype of each recorded call
  size_t prof_used = 0;                 // events in use
  LaunchTimer batch_timer;              // batched launches
  double prof_ms[kPhases][2] = {};      // per phase and dtype
  uint64_t prof_calls[kPhases][2] = {};
};

namespace {

int fail(szsel_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(szsel_ctx *c, hipError_t e, const char *what) {
  return fail(c, SZSEL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace szsel {

int ctx_ncu(const szsel_ctx *ctx) { return ctx ? ctx->ncu : 256; }

const char *ctx_arch(const szsel_ctx *ctx) { return ctx ? ctx->arch.c_str() : ""; }

int check_request(int op, const void *field, const int64_t *dims, int nd, int dtype, double eb,
                  int eb_mode, const int32_t *stride, std::string &why) {
  auto bad = [&](int code, const char *m) {
    why = m;
    return code;
  };
  if (!field) return bad(SZSEL_EINVAL, "field is NULL");
  if (!dims) return bad(SZSEL_EINVAL, "dims is NULL");
  if (nd < 1 || nd > 3) return bad(SZSEL_EINVAL, "ndims must be 1, 2 or 3");
  if (dtype != SZSEL_F32 && dtype != SZSEL_F64) return bad(SZSEL_EDTYPE, "dtype must be SZSEL_F32 or SZSEL_F64");
  if (op < SZSEL_OP_SZ || op > SZSEL_OP_FIXED_EB) return bad(SZSEL_EINVAL, "bad op");
  if (!(eb > 0.0) || !std::isfinite(eb)) return bad(SZSEL_EINVAL, "eb must be > 0 and finite");
  if (eb_mode != SZSEL_EB_ABS && eb_mode != SZSEL_EB_REL)
    return bad(SZSEL_EINVAL, "eb_mode must be SZSEL_EB_ABS or SZSEL_EB_REL");
  const size_t esz = dtype == SZSEL_F32 ? 4 : 8;
  if ((uintptr_t)field % esz) return bad(SZSEL_EINVAL, "field is not aligned to its element size");
  int64_t n = 1;
  uint64_t nblk = 1;
  for (int k = 0; k < nd; k++) {
    if (dims[k] < 1) return bad(SZSEL_EINVAL, "every extent must be >= 1");
    const int32_t st = stride ? stride[k] : 1;
    if (st < 1) return bad(SZSEL_EINVAL, "every stride must be >= 1");
    if (n > INT64_MAX / dims[k]) return bad(SZSEL_EINVAL, "field too large");
    n *= dims[k];
    const int64_t ns = (dims[k] / 4 + st - 1) / st;
    if (ns > 0xFFFFFFFFll) return bad(SZSEL_EINVAL, "too many blocks along an axis");
    nblk *= (uint64_t)ns;
    if (nblk > 0xFFFFFFFFull) return bad(SZSEL_EINVAL, "more than 2^32 sampled blocks; use a larger stride");
  }
  return SZSEL_OK;
}

int plan_request(szsel_ctx *ctx, int op, const void *field, const int64_t *dims, int nd,
                 int dtype, double eb, int eb_mode, const int32_t *stride, const Tune &tu,
                 ReqDesc &r) {
  if (!ctx) return SZSEL_EINVAL;
  {
    std::string why;
    const int rc = check_request(op, field, dims, nd, dtype, eb, eb_mode, stride, why);
    if (rc != SZSEL_OK) return fail(ctx, rc, why);
  }
  const size_t esz = dtype == SZSEL_F32 ? 4 : 8;
  std::memset(&r, 0, sizeof(r));
  r.field = field;
  r.nd = nd;
  r.dtype = dtype;
  r.op = op;
  r.eb_mode = eb_mode;
  r.eb = eb;
  r.sz_offset = ctx->sz_offset;
  r.huff = ctx->huffman;
  r.ec = ctx->ec;
  r.ovf_per_slice = tu.ovf_slice > 0 ? tu.ovf_slice : kOvfPerSlice;
  int64_t n = 1;
  uint64_t nblk = 1;
  for (int k = 0; k < nd; k++) {  // (the bounds were checked above)
    const int32_t s = stride ? stride[k] : 1;
    n *= dims[k];
    r.dims[k] = dims[k];
    r.stride[k] = s;
    const int64_t nb = dims[k] / 4;
    const int64_t ns = (nb + s - 1) / s;
    r.nsel[k] = (uint32_t)ns;
    // multiply-shift constants for dividing block indices by nsel[k]
    // (Granlund and Montgomery, PLDI 1994): l = ceil(log2 d),
    // m = floor(2^32 (2^l - d) / d) + 1, shifts min(l, 1) and max(l - 1, 0)
    {
      const uint64_t d = ns > 0 ? (uint64_t)ns : 1;
      int l = 0;
      while ((1ull << l) < d) l++;
      const uint64_t m = (((uint64_t)1 << 32) * ((1ull << l) - d)) / d + 1;
      r.dmul[k] = (uint32_t)m;
      r.dsh[k] = (uint32_t)(l < 1 ? l : 1) | ((uint32_t)(l > 1 ? l - 1 : 0) << 8);
    }
    nblk *= (uint64_t)ns;
  }
  r.n = n;
  r.nblk = (int64_t)nblk;
  // element offsets of the Lorenzo neighbours p - e_S, subsets in the
  // predictor's term order (single axes slowest first, then pairs, then all)
  {
    int64_t st[3] = {0, 0, 0};
    int64_t acc = 1;
    for (int k = nd - 1; k >= 0; k--) {
      st[k] = acc;
      acc *= dims[k];
    }
    static const int kS1[1] = {1}, kS2[3] = {1, 2, 3}, kS3[7] = {1, 2, 4, 3, 5, 6, 7};
    const int *sub = nd == 1 ? kS1 : (nd == 2 ? kS2 : kS3);
    for (int t = 0; t < (1 << nd) - 1; t++) {
      int64_t off = 0;
      for (int k = 0; k < nd; k++)
        if (sub[t] & (1 << k)) off += st[k];
      r.nboff[t] = off;
    }
  }
  // ZFP and SZ passes: every workgroup owns an aligned power-of-two chunk of
  // consecutive sampled blocks, and a pass has at most kMaxParts workgroups.
  // ZFP: one wave per workgroup, rounds of 64 blocks (one block per lane)
  // or, for 3-D blocks without sub-sampling, of 16 (four lanes per block),
  // about tu.zfp_waves waves per CU (default 64, about 16 per SIMD: several
  // rounds of the resident waves, so that the last round's tail is short
  // while each wave still does a few rounds of blocks), or the batch
  // planner's share of them.  SZ: at least one round of 4 waves.
  auto chunk_for = [&](uint64_t min_chunk, uint64_t target_wgs, uint64_t max_wgs) {
    const uint64_t want = (nblk + target_wgs - 1) / target_wgs;
    uint64_t c = min_chunk;
    while (c < want) c <<= 1;
    while ((nblk + c - 1) / c > max_wgs) c <<= 1;
    return c;
  };
  const uint64_t zround = (nd == 3 && !r.ec) ? (uint64_t)(kWave / 4) : (uint64_t)kWave;
  const uint64_t zfp_target = tu.zfp_target > 0 ? (uint64_t)tu.zfp_target
                                                 : (uint64_t)std::max(1, tu.zfp_waves) * (uint64_t)ctx->ncu;
  const uint64_t zc = chunk_for(std::max<uint64_t>((uint64_t)tu.zfp_chunk, zround), zfp_target, kMaxParts);
  // SZ: one lane per two rows of 4 points (one row in 1-D); by
  // default 2 workgroups per CU, all of them resident at once
  const uint64_t sz_target = tu.sz_target > 0 ? (uint64_t)tu.sz_target
                                               : std::max<uint64_t>(1, (uint64_t)tu.sz_wgs_q * (uint64_t)ctx->ncu / 4);
  const uint64_t sc = chunk_for((uint64_t)kWaves * sz_blocks_per_wave(nd), sz_target, kMaxParts);
  if (zc > (1u << 30) || sc > (1u << 30)) return fail(ctx, SZSEL_EINVAL, "too many sampled blocks");
  r.zblk = (int32_t)zc;
  r.sblk = (int32_t)sc;
  r.nzfp = (int32_t)std::max<uint64_t>(1, (nblk + zc - 1) / zc);
  r.nsz = (int32_t)std::max<uint64_t>(1, (nblk + sc - 1) / sc);
  // global histogram copies: about 128 SZ workgroups flush into each
  r.nhc = 1;
  while (r.nhc < kHistCopies && (int64_t)r.nhc * 128 < r.nsz) r.nhc <<= 1;
  // rows of 4 values start on 16-byte boundaries: aligned field, row
  // length a multiple of 16 bytes / element size (blocks start at x = 4 b s)
  r.vec = ((uintptr_t)field % 16 == 0 && (dims[nd - 1] * (int64_t)esz) % 16 == 0) ? 1 : 0;
  // range pass: contiguous chunks of whole 16-byte vectors, about
  // range_wgs_q quarters of the CU count of them, at least 8 vectors per thread
  const int64_t vn = 16 / (int64_t)esz;
  const int64_t quantum = (int64_t)kThreads * vn;
  const int64_t rw = std::min<int64_t>(kMaxParts, tu.range_target > 0 ? (int64_t)tu.range_target
                                                                     : std::max<int64_t>(1, (int64_t)tu.range_wgs_q * ctx->ncu / 4));
  int64_t chunk = (n + rw - 1) / rw;
  chunk = std::max<int64_t>(chunk, 8 * quantum);
  chunk = (chunk + quantum - 1) / quantum * quantum;
  r.rchunk = chunk;
  r.nrange = (int32_t)((n + chunk - 1) / chunk);
  if (r.nrange > kMaxParts) return fail(ctx, SZSEL_EINVAL, "field too large for one request");
  return SZSEL_OK;
}

}  // namespace szsel

namespace {

constexpr size_t kProfEvents = kEv * 1024;

// Accumulates the elapsed times of the recorded phase events and frees them.
int profile_drain(szsel_ctx *c) {
  for (size_t k = 0; k + kEv <= c->prof_used; k += kEv) {
    hipEvent_t *ev = &c->prof_events[k];
    const int dt = c->prof_dtype[k / kEv];
    hipError_t e = hipEventSynchronize(ev[kPhases]);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    for (int ph = 0; ph < kPhases; ph++) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[ph], ev[ph + 1]);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
      c->prof_ms[ph][dt] += ms;
      c->prof_calls[ph][dt] += 1;
    }
  }
  c->prof_used = 0;
  // batched launches: one event pair per launch; the Huffman pass counts
  // with the entropy pass, as in single calls
  LaunchTimer &lt = c->batch_timer;
  for (size_t k = 0; k < lt.used; k++) {
    hipError_t e = hipEventSynchronize(lt.ev[2 * k + 1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, lt.ev[2 * k], lt.ev[2 * k + 1]);
    if (e != hipSuccess) return hip_fail(c, e, "batch phase timer");
    const int ph = std::min(lt.tag[k] / 2, kPhases - 1), dt = lt.tag[k] & 1;
    c->prof_ms[ph][dt] += ms;
    c->prof_calls[ph][dt] += 1;
  }
  lt.used = 0;
  return SZSEL_OK;
}

int run_single(szsel_ctx *ctx, int op, const void *field, const int64_t *dims, int nd, int dtype,
               double eb, int eb_mode, const int32_t *stride, szsel_result *out, void *stream) {
  if (!ctx) return SZSEL_EINVAL;
  if (!out) return fail(ctx, SZSEL_EINVAL, "out is NULL");
  ReqDesc r;
  int rc = plan_request(ctx, op, field, dims, nd, dtype, eb, eb_mode, stride, ctx->bopt.fixed, r);
  if (rc != SZSEL_OK) return rc;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t fixed = request_fixed_bytes();
  const size_t need = fixed + request_var_bytes(r);
  Slot &sl = ctx->slots[ctx->next];
  ctx->next = (ctx->next + 1) % kSlots;
  if (need > sl.bytes) {  // grow the slot (waits for the device)
    if (ctx->used_bytes - sl.bytes + need > ctx->budget)
      return fail(ctx, SZSEL_ENOMEM, "request workspace exceeds the context's budget");
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    if (sl.mem) (void)hipFree(sl.mem);
    ctx->used_bytes -= sl.bytes;
    sl.mem = nullptr;
    sl.bytes = 0;
    sl.used = false;
    void *p = nullptr;
    e = hipMalloc(&p, need);
    if (e == hipSuccess) e = hipMemset(p, 0, need);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      if (p) (void)hipFree(p);
      return hip_fail(ctx, e, "workspace allocation");
    }
    sl.mem = (char *)p;
    sl.bytes = need;
    ctx->used_bytes += need;
  }
  if (sl.used) {
    e = hipStreamWaitEvent(s, sl.done, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamWaitEvent");
  }
  bind_request_workspace(r, sl.mem, sl.mem + fixed);
  if (ctx->dbg_armed) {
    r.dbg_codes = ctx->dbg.codes;
    r.dbg_zbits = ctx->dbg.zfp_bits;
    r.dbg_zsse = ctx->dbg.zfp_sse;
    r.dbg_zemax = ctx->dbg.zfp_emax;
    r.dbg_ssse = ctx->dbg.sz_sse;
    r.dbg_hist = ctx->dbg.hist;
    ctx->dbg_armed = false;
  }
  const hipEvent_t *ev = nullptr;
  if (ctx->prof) {
    if (ctx->prof_used + kEv > ctx->prof_events.size()) {
      int rc2 = profile_drain(ctx);
      if (rc2 != SZSEL_OK) return rc2;
    }
    ev = &ctx->prof_events[ctx->prof_used];
    ctx->prof_dtype[ctx->prof_used / kEv] = dtype;
    ctx->prof_used += kEv;
  }
  e = launch_request(r, s, ev);
  if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
  e = hipMemcpyAsync(out, r.res, sizeof(szsel_result), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(result)");
  e = hipEventRecord(sl.done, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
  sl.used = true;
  ctx->err.clear();
  return SZSEL_OK;
}

}  // namespace

extern "C" {

int szsel_create(szsel_ctx **out, int hip_device, size_t budget) {
  if (!out) return SZSEL_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return SZSEL_EINVAL;
  szsel_ctx *c = new (std::nothrow) szsel_ctx();
  if (!c) return SZSEL_ENOMEM;
  c->device = hip_device;
  c->budget = budget ? budget : ((size_t)16 << 30);
  hipError_t e = hipSetDevice(hip_device);
  int ncu = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, hip_device);
  if (e != hipSuccess) {
    delete c;
    return SZSEL_EHIP;
  }
  c->ncu = ncu > 0 ? ncu : 256;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) c->arch = prop.gcnArchName;
  }
  // slots are allocated on first use and grow with the requests they serve
  for (int k = 0; k < kSlots; k++) {
    e = hipEventCreateWithFlags(&c->slots[k].done, hipEventDisableTiming);
    if (e != hipSuccess) {
      szsel_destroy(c);
      return SZSEL_EHIP;
    }
  }
  // the allocation-free entry point's workspace on this device (once per
  // device and process)
  e = noalloc_setup(hip_device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    szsel_destroy(c);
    return SZSEL_EHIP;
  }
  *out = c;
  return SZSEL_OK;
}

void szsel_destroy(szsel_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (int k = 0; k < kSlots; k++) {
    if (c->slots[k].mem) (void)hipFree(c->slots[k].mem);
    if (c->slots[k].done) (void)hipEventDestroy(c->slots[k].done);
  }
  for (int k = 0; k < kBatchSlots; k++) batch_destroy(c->batch[k]);
  if (c->zc_ws) (void)hipFree(c->zc_ws);
  for (auto &ev : c->prof_events)
    if (ev) (void)hipEventDestroy(ev);
  for (auto &ev : c->batch_timer.ev)
    if (ev) (void)hipEventDestroy(ev);
  delete c;
}

int szsel_estimate_sz(szsel_ctx *c, const void *f, const int64_t *d, int nd, int dt, double eb,
                      int m, const int32_t *s, szsel_result *o, void *st) {
  return run_single(c, SZSEL_OP_SZ, f, d, nd, dt, eb, m, s, o, st);
}

int szsel_estimate_zfp(szsel_ctx *c, const void *f, const int64_t *d, int nd, int dt, double eb,
                       int m, const int32_t *s, szsel_result *o, void *st) {
  return run_single(c, SZSEL_OP_ZFP, f, d, nd, dt, eb, m, s, o, st);
}

int szsel_select(szsel_ctx *c, const void *f, const int64_t *d, int nd, int dt, double eb, int m,
                 const int32_t *s, szsel_result *o, void *st) {
  return run_single(c, SZSEL_OP_SELECT, f, d, nd, dt, eb, m, s, o, st);
}

int szsel_select_fixed_eb(szsel_ctx *c, const void *f, const int64_t *d, int nd, int dt, double eb,
                          int m, const int32_t *s, szsel_result *o, void *st) {
  return run_single(c, SZSEL_OP_FIXED_EB, f, d, nd, dt, eb, m, s, o, st);
}

int szsel_select_noalloc(szsel_ctx *c, const void *f, const int64_t *d, int nd, int dt, double eb,
                         int m, const int32_t *s, szsel_result *o, void *st) {
  // szsel_select with the request's workspace in the device's static array:
  // no allocation, no event, no profiling; ordering between calls is the
  // caller's (they share the array)
  if (!c) return SZSEL_EINVAL;
  if (!o) return fail(c, SZSEL_EINVAL, "out is NULL");
  ReqDesc r;
  int rc = plan_request(c, SZSEL_OP_SELECT, f, d, nd, dt, eb, m, s, c->bopt.fixed, r);
  if (rc != SZSEL_OK) return rc;
  char *ws = noalloc_scratch(c->device);
  if (!ws) return fail(c, SZSEL_EHIP, "the allocation-free workspace is not set up on this device");
  const size_t fixed = request_fixed_bytes();
  const size_t need = fixed + request_var_bytes(r);
  if (need > kNoallocScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "request needs %zu bytes of workspace; szsel_select_noalloc has %zu "
                  "(use a larger stride, or szsel_select)",
                  need, kNoallocScratchBytes);
    return fail(c, SZSEL_ENOMEM, msg);
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const hipStream_t hs = (hipStream_t)st;
  bind_request_workspace(r, ws, ws + fixed);
  e = launch_request(r, hs, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  e = hipMemcpyAsync(o, r.res, sizeof(szsel_result), hipMemcpyDeviceToHost, hs);
  if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync(result)");
  c->err.clear();
  return SZSEL_OK;
}

int szsel_select_batch(szsel_ctx *c, const szsel_request *reqs, int n, szsel_result *out,
                       void *stream) {
  if (!c) return SZSEL_EINVAL;
  if (n < 0 || (n > 0 && (!reqs || !out))) return fail(c, SZSEL_EINVAL, "bad batch arguments");
  if (n == 0) return SZSEL_OK;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  const int k = c->bnext;
  c->bnext = (c->bnext + 1) % kBatchSlots;
  // the batch states share the context's budget with the single-request slots
  size_t others = c->used_bytes;
  for (int q = 0; q < kBatchSlots; q++)
    if (q != k) others += c->batch_bytes[q];
  const size_t budget = c->budget > others ? c->budget - others : 0;
  std::string msg;
  c->err.clear();
  BatchOptions opt = c->bopt;
  opt.timer = c->prof ? &c->batch_timer : nullptr;
  const int rc = batch_run(c, c->ncu, c->batch[k], budget, reqs, n, out, (hipStream_t)stream, opt, msg);
  c->batch_bytes[k] = batch_state_bytes(c->batch[k]);
  if (rc != SZSEL_OK) return fail(c, rc, msg + c->err);
  c->err.clear();
  return SZSEL_OK;
}

const char *szsel_last_error(const szsel_ctx *c) { return c ? c->err.c_str() : "no context"; }

int szsel_stride_for_rate(double r_sp, int nd, const int64_t *dims, int32_t *out) {
  if (!(r_sp > 0.0) || r_sp > 1.0 || nd < 1 || nd > 3 || !dims || !out) return SZSEL_EINVAL;
  int64_t nb[3];
  for (int k = 0; k < nd; k++) {
    if (dims[k] < 4) return SZSEL_EINVAL;
    nb[k] = dims[k] / 4;
  }
  // stride 1 on the fastest axis (contiguous rows of blocks); search the
  // slower axes for the fraction closest to r_sp in log ratio, with a small
  // penalty on unbalanced strides (an even spread of samples), then the
  // larger stride on the slowest axis
  double best = INFINITY;
  int32_t bs[3] = {1, 1, 1};
  const int slow = nd - 1;
  const int64_t lim0 = slow >= 1 ? nb[0] : 1, lim1 = slow >= 2 ? nb[1] : 1;
  for (int64_t s0 = 1; s0 <= lim0; s0++) {
    for (int64_t s1 = 1; s1 <= lim1; s1++) {
      double frac = 1.0;
      if (slow >= 1) frac *= (double)((nb[0] + s0 - 1) / s0) / (double)nb[0];
      if (slow >= 2) frac *= (double)((nb[1] + s1 - 1) / s1) / (double)nb[1];
      const double balance = slow >= 2 ? std::fabs(std::log((double)s0 / (double)s1)) : 0.0;
      const double cost = std::fabs(std::log(frac / r_sp)) + 0.05 * balance - 1e-12 * (double)s0;
      if (cost < best) {
        best = cost;
        bs[0] = (int32_t)s0;
        bs[1] = (int32_t)s1;
      }
    }
  }
  for (int k = 0; k < nd; k++) out[k] = 1;
  if (slow >= 1) out[0] = bs[0];
  if (slow >= 2) out[1] = bs[1];
  return SZSEL_OK;
}

int szsel_set_option(szsel_ctx *c, int option, double value) {
  if (!c) return SZSEL_EINVAL;
  if (option == SZSEL_OPT_SZ_OFFSET) {
    if (!std::isfinite(value)) return fail(c, SZSEL_EINVAL, "offset must be finite");
    c->sz_offset = value;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_HUFFMAN) {
    if (value != 0.0 && value != 1.0 && value != 2.0) return fail(c, SZSEL_EINVAL, "Huffman option: 0, 1 or 2");
    c->huffman = (int)value;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_EC_SAMPLING) {
    if (value != 0.0 && value != 1.0 && value != 2.0) return fail(c, SZSEL_EINVAL, "EC sampling option: 0, 1 or 2");
    c->ec = (int)value;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_AUTOTUNE) {
    c->bopt.autotune = value != 0.0;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_BATCH_GRAPH) {
    c->bopt.graph = value != 0.0;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_BATCH_SHARE) {
    const int v = (int)value;
    if (value != (double)v || v < 0 || v > 3) return fail(c, SZSEL_EINVAL, "batch share: 0, 1, 2 or 3");
    c->bopt.fixed.share = v;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_RANGE_GRID) {
    const int v = (int)value;
    if (value != (double)v || v < 0 || v > 64) return fail(c, SZSEL_EINVAL, "range grid: 0 to 64 workgroups per CU");
    c->bopt.fixed.range_grid = v;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_BATCH_LANES) {
    const int v = (int)value;
    if (value != (double)v || v < 0 || v > 3) return fail(c, SZSEL_EINVAL, "batch lanes: 0 to 3");
    c->bopt.fixed.lanes = v ? v : Tune().lanes;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_BATCH_GROUPS) {
    const int v = (int)value;
    if (value != (double)v || v < 0 || v > 8) return fail(c, SZSEL_EINVAL, "request groups: 0 to 8");
    c->bopt.fixed.groups = v ? v : Tune().groups;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_RANGE_WGS) {
    const double q = value * 4.0;
    if (!(q >= 0.0) || q != std::floor(q) || q > 256.0)
      return fail(c, SZSEL_EINVAL, "range workgroups per CU: a multiple of 0.25, at most 64");
    c->bopt.fixed.range_wgs_q = q > 0.0 ? (int)q : Tune().range_wgs_q;
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_SZ_WGS || option == SZSEL_OPT_ZFP_CHUNK) {
    const Tune dflt;
    const int v = (int)value;
    if (value != (double)v || v < 0) return fail(c, SZSEL_EINVAL, "launch-shape values are non-negative integers");
    if (option == SZSEL_OPT_SZ_WGS) {
      if (v > 256) return fail(c, SZSEL_EINVAL, "SZ workgroups: at most 256 quarters of the CU count");
      c->bopt.fixed.sz_wgs_q = v ? v : dflt.sz_wgs_q;
    } else {
      if (v && (v < 16 || v > 65536 || (v & (v - 1))))
        return fail(c, SZSEL_EINVAL, "ZFP chunk: a power of two from 16 to 65536");
      c->bopt.fixed.zfp_chunk = v ? v : dflt.zfp_chunk;
    }
    return SZSEL_OK;
  }
  if (option == SZSEL_OPT_PROFILE) {
    const bool on = value != 0.0;
    if (on && c->prof_events.empty()) {
      (void)hipSetDevice(c->device);
      c->prof_events.resize(kProfEvents, nullptr);
      c->prof_dtype.resize(kProfEvents / kEv, 0);
      for (auto &ev : c->prof_events) {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
      }
    }
    if (!on && c->prof) {
      int rc = profile_drain(c);
      if (rc != SZSEL_OK) return rc;
    }
    c->prof = on;
    return SZSEL_OK;
  }
  return fail(c, SZSEL_EINVAL, "unknown option");
}

int szsel_profile_read(szsel_ctx *c, double *ms, uint64_t *calls) {
  if (!c || !ms || !calls) return SZSEL_EINVAL;
  double m[2 * kPhases];
  uint64_t n[2 * kPhases];
  const int rc = szsel_profile_read_split(c, m, n);
  if (rc != SZSEL_OK) return rc;
  for (int k = 0; k < kPhases; k++) {
    ms[k] = m[2 * k] + m[2 * k + 1];
    calls[k] = n[2 * k] + n[2 * k + 1];
  }
  return SZSEL_OK;
}

int szsel_profile_read_split(szsel_ctx *c, double *ms, uint64_t *calls) {
  if (!c || !ms || !calls) return SZSEL_EINVAL;
  int rc = profile_drain(c);
  if (rc != SZSEL_OK) return rc;
  for (int k = 0; k < kPhases; k++)
    for (int d = 0; d < 2; d++) {
      ms[2 * k + d] = c->prof_ms[k][d];
      calls[2 * k + d] = c->prof_calls[k][d];
      c->prof_ms[k][d] = 0.0;
      c->prof_calls[k][d] = 0;
    }
  return SZSEL_OK;
}

int szsel_set_debug(szsel_ctx *c, const szsel_debug *d) {
  if (!c) return SZSEL_EINVAL;
  if (d) {
    c->dbg = *d;
    c->dbg_armed = true;
  } else {
    c->dbg_armed = false;
  }
  return SZSEL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Step 4 (Section 3; Algorithm 1's ZFP branch): ZFP compression of the whole field
// ---------------------------------------------------------------------------

static int64_t zc_num_blocks(const int64_t *dims, int nd) {
  int64_t nb = 1;
  for (int k = 0; k < nd; k++) nb *= (dims[k] + 3) / 4;
  return nb;
}

size_t szsel_zfp_stream_bytes(const int64_t *dims, int ndims, int dtype) {
  if (!dims || ndims < 1 || ndims > 3 || (dtype != SZSEL_F32 && dtype != SZSEL_F64)) return 0;
  for (int k = 0; k < ndims; k++)
    if (dims[k] < 1) return 0;
  return szsel::zc_stream_words(zc_num_blocks(dims, ndims), ndims, dtype) * 8;
}

static uint64_t unordered_bits(uint64_t b) { return (b >> 63) ? (b & ~(1ull << 63)) : ~b; }
static double bits_double(uint64_t b) {
  double v;
  std::memcpy(&v, &b, sizeof(v));
  return v;
}

int szsel_zfp_compress(szsel_ctx *c, const void *field, const int64_t *dims, int ndims, int dtype,
                       double eb_abs, void *stream_buf, size_t stream_bytes, void *decoded,
                       szsel_compressed *out, void *stream) {
  if (!c) return SZSEL_EINVAL;
  if (!field || !dims || !stream_buf || !out) return fail(c, SZSEL_EINVAL, "null argument");
  if (ndims < 1 || ndims > 3) return fail(c, SZSEL_EINVAL, "ndims must be 1, 2 or 3");
  if (dtype != SZSEL_F32 && dtype != SZSEL_F64) return fail(c, SZSEL_EINVAL, "dtype must be SZSEL_F32 or SZSEL_F64");
  if (!(eb_abs > 0.0) || !std::isfinite(eb_abs)) return fail(c, SZSEL_EINVAL, "eb_abs must be > 0 and finite");
  int64_t n = 1;
  for (int k = 0; k < ndims; k++) {
    if (dims[k] < 1) return fail(c, SZSEL_EINVAL, "every extent must be >= 1");
    if (n > INT64_MAX / dims[k]) return fail(c, SZSEL_EINVAL, "field too large");
    n *= dims[k];
  }
  const size_t esz = dtype == SZSEL_F32 ? 4 : 8;
  if ((uintptr_t)field % esz || (decoded && (uintptr_t)decoded % esz))
    return fail(c, SZSEL_EINVAL, "field and decoded must be aligned to their element size");
  if ((uintptr_t)stream_buf % 8) return fail(c, SZSEL_EINVAL, "stream buffer must be 8-byte aligned");
  const size_t need = szsel_zfp_stream_bytes(dims, ndims, dtype);
  if (stream_bytes < need) return fail(c, SZSEL_EINVAL, "stream buffer smaller than szsel_zfp_stream_bytes()");
  (void)hipSetDevice(c->device);
  hipStream_t s = (hipStream_t)stream;
  const int64_t nblocks = zc_num_blocks(dims, ndims);
  if (nblocks > (int64_t)INT32_MAX * 64) return fail(c, SZSEL_EINVAL, "too many blocks");
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t red_half = szsel::zc_red_half(nblocks), nchunks = szsel::zc_chunks(nblocks);
  const size_t b_counts = al(4 * (size_t)nblocks), b_offsets = al(8 * (size_t)nblocks), b_sse = al(8 * (size_t)nblocks);
  const size_t b_chunk = al(8 * nchunks), b_red = al(16 * red_half), b_res = al(sizeof(szsel::ZcResult));
  const size_t total = b_counts + b_offsets + b_sse + b_chunk + b_red + b_res;
  if (total > c->zc_ws_bytes) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    if (c->zc_ws) (void)hipFree(c->zc_ws);
    c->zc_ws = nullptr;
    c->zc_ws_bytes = 0;
    e = hipMalloc((void **)&c->zc_ws, total);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc (compression workspace)");
    c->zc_ws_bytes = total;
  }
  char *p = c->zc_ws;
  szsel::ZcArgs a{};
  a.field = field;
  for (int k = 0; k < ndims; k++) {
    a.dims[k] = dims[k];
    a.nb[k] = (dims[k] + 3) / 4;
  }
  a.nd = ndims;
  a.dtype = dtype;
  {
    int e2;
    (void)std::frexp(eb_abs, &e2);
    a.minexp = e2 - 1;  // floor(log2(eb_abs))
  }
  a.nblocks = nblocks;
  a.counts = (uint32_t *)p;
  p += b_counts;
  a.offsets = (uint64_t *)p;
  p += b_offsets;
  a.bsse = (double *)p;
  p += b_sse;
  a.chunk = (uint64_t *)p;
  p += b_chunk;
  a.red = (double *)p;
  a.red_half = (int64_t)red_half;
  p += b_red;
  a.res = (szsel::ZcResult *)p;
  a.stream = (uint64_t *)stream_buf;
  a.stream_words = (int64_t)(need / 8);
  a.decoded = decoded;
  hipError_t e = szsel::zc_launch(a, s);
  if (e != hipSuccess) return hip_fail(c, e, "ZFP compression launch");
  szsel::ZcResult h{};
  e = hipMemcpyAsync(&h, a.res, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "ZFP compression");
  std::memset(out, 0, sizeof(*out));
  out->bits = h.bits;
  out->values = (uint64_t)n;
  out->blocks = (uint64_t)nblocks;
  out->bitrate = (double)h.bits / (double)n;
  out->sse = h.sse;
  out->mse = h.sse / (double)n;
  out->maxerr = bits_double(unordered_bits(h.maxerr_bits));
  const double vmin = bits_double(unordered_bits(h.vmin_bits)), vmax = bits_double(unordered_bits(h.vmax_bits));
  out->vr = vmax - vmin;
  out->eb_abs = eb_abs;
  out->psnr = out->mse > 0.0 ? 20.0 * std::log10(out->vr) - 10.0 * std::log10(out->mse) : INFINITY;
  if (h.nonfinite) out->flags |= SZSEL_FLAG_NONFINITE;
  return SZSEL_OK;
}

int szsel_sz_compress(szsel_ctx *c, const void *field, const int64_t *dims, int ndims, int dtype,
                      double eb_abs, void *symbols, void *decoded, szsel_compressed *out, void *stream) {
  if (!c) return SZSEL_EINVAL;
  if (!field || !dims || !out) return fail(c, SZSEL_EINVAL, "null argument");
  if (ndims < 1 || ndims > 3) return fail(c, SZSEL_EINVAL, "ndims must be 1, 2 or 3");
  if (dtype != SZSEL_F32 && dtype != SZSEL_F64) return fail(c, SZSEL_EINVAL, "dtype must be SZSEL_F32 or SZSEL_F64");
  if (!(eb_abs > 0.0) || !std::isfinite(eb_abs)) return fail(c, SZSEL_EINVAL, "eb_abs must be > 0 and finite");
  int64_t n = 1;
  for (int k = 0; k < ndims; k++) {
    if (dims[k] < 1) return fail(c, SZSEL_EINVAL, "every extent must be >= 1");
    if (n > INT64_MAX / dims[k]) return fail(c, SZSEL_EINVAL, "field too large");
    n *= dims[k];
  }
  const size_t esz = dtype == SZSEL_F32 ? 4 : 8;
  if ((uintptr_t)field % esz || (decoded && (uintptr_t)decoded % esz) || ((uintptr_t)symbols % 2))
    return fail(c, SZSEL_EINVAL, "buffers must be aligned to their element size");
  const double delta = 2.0 * eb_abs;
  if (!std::isfinite(delta)) return fail(c, SZSEL_EINVAL, "2 eb_abs overflows");
  (void)hipSetDevice(c->device);
  hipStream_t s = (hipStream_t)stream;
  const size_t nchunks = szsel::sz4_chunks(n);
  if (nchunks > (size_t)INT32_MAX) return fail(c, SZSEL_EINVAL, "field too large");
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t red_half = szsel::zc_red_half((int64_t)nchunks);
  const size_t b_hist = al(sizeof(uint32_t) * (size_t)szsel::kSzCopies * 65536), b_hfinal = al(sizeof(uint32_t) * 65536);
  const size_t b_chunk = al(8 * nchunks), b_red = al(16 * red_half), b_res = al(sizeof(szsel::SzResult));
  const size_t total = b_hist + b_hfinal + b_chunk + b_red + b_res;
  if (total > c->zc_ws_bytes) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    if (c->zc_ws) (void)hipFree(c->zc_ws);
    c->zc_ws = nullptr;
    c->zc_ws_bytes = 0;
    e = hipMalloc((void **)&c->zc_ws, total);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc (compression workspace)");
    c->zc_ws_bytes = total;
  }
  char *p = c->zc_ws;
  szsel::SzArgs a{};
  a.field = field;
  for (int k = 0; k < ndims; k++) a.dims[k] = dims[k];
  a.nd = ndims;
  a.dtype = dtype;
  a.n = n;
  a.delta = delta;
  a.inv = 1.0 / delta;
  a.eb = eb_abs;
  a.hist = (uint32_t *)p;
  p += b_hist;
  a.hfinal = (uint32_t *)p;
  p += b_hfinal;
  a.chunk_sse = (double *)p;
  a.nchunks = (int64_t)nchunks;
  p += b_chunk;
  a.red = (double *)p;
  a.red_half = (int64_t)red_half;
  p += b_red;
  a.res = (szsel::SzResult *)p;
  a.decoded = decoded;
  a.symbols = (uint16_t *)symbols;
  hipError_t e = szsel::sz4_launch(a, s);
  if (e != hipSuccess) return hip_fail(c, e, "SZ compression launch");
  szsel::SzResult h{};
  e = hipMemcpyAsync(&h, a.res, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "SZ compression");
  const int W = dtype == SZSEL_F32 ? 32 : 64;
  std::memset(out, 0, sizeof(*out));
  out->values = (uint64_t)n;
  out->unpredictable = h.escapes;
  out->symbols = h.symbols;
  out->code_bits = h.code_bits;
  out->code_entropy = std::log2((double)n) - h.hsum / (double)n;
  const uint64_t side = (uint64_t)W * h.escapes + 32ull * h.symbols;
  if (h.huff_ok) {
    out->bits = h.code_bits + side;
    out->bitrate = (double)out->bits / (double)n;
  } else {
    out->flags |= SZSEL_FLAG_NO_HUFFMAN;
    out->bitrate = out->code_entropy + (double)side / (double)n;
  }
  out->sse = h.sse;
  out->mse = h.sse / (double)n;
  out->maxerr = bits_double(unordered_bits(h.maxerr_bits));
  const double vmin = bits_double(unordered_bits(h.vmin_bits)), vmax = bits_double(unordered_bits(h.vmax_bits));
  out->vr = vmax - vmin;
  out->eb_abs = eb_abs;
  out->psnr = out->mse > 0.0 ? 20.0 * std::log10(out->vr) - 10.0 * std::log10(out->mse) : INFINITY;
  if (h.nonfinite) out->flags |= SZSEL_FLAG_NONFINITE;
  return SZSEL_OK;
}
