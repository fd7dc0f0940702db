// Serving engine: continuous batching of snapshots of fields.
//
// The caller (the producer loop) owns a device pool.  A snapshot is admitted
// by reserving its bytes in the pool (first-fit arena over 256-byte
// granules); the producer writes its fields there and submits its requests.
// Admitted requests wait in one FIFO.  The engine has L lanes, each a stream
// with its own batch workspace: whenever a lane is free and requests are
// waiting, the lane takes up to kServeBatch of them (from any number of
// snapshots) as one batch.  Lanes run concurrently, so requests that arrive
// while others are on the GPU start as soon as a lane frees up and overlap
// them.  A snapshot completes when all of its requests have; its pool range
// is then released, which may admit the next snapshot.
//
// Requests are checked when they are submitted (the planner's argument
// checks, and that one request fits a lane's workspace), and a lane batch
// never holds more requests than its workspace budget takes.  A batch that
// still fails to launch is put back in the queue and retried in halves; a
// single request that fails alone completes with SZSEL_FLAG_FAILED, so that
// no snapshot waits forever and every pool range is released.
//
// Single-threaded: every call comes from the same host thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "batch.hpp"
#include "launch.hpp"
#include "szsel.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kGranule = 256;
constexpr int kServeBatch = 64;  // requests per lane batch (bounds a lane's workspace)

// First-fit allocator over [0, size) in granules, coalescing on release.
struct Arena {
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t bytes) {
    size = bytes / kGranule * kGranule;
    used = 0;
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t &off) {
    const size_t want = (bytes + kGranule - 1) / kGranule * kGranule;
    if (want == 0) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < want) continue;
      off = it->first;
      const size_t rest = it->second - want;
      free_.erase(it);
      if (rest) free_[off + want] = rest;
      used += want;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    const size_t len = (bytes + kGranule - 1) / kGranule * kGranule;
    used -= len;
    auto next = free_.lower_bound(off);
    size_t o = off, l = len;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == o) {
        o = prev->first;
        l += prev->second;
        free_.erase(prev);
      }
    }
    next = free_.lower_bound(o + l);
    if (next != free_.end() && next->first == o + l) {
      l += next->second;
      free_.erase(next);
    }
    free_[o] = l;
  }
  size_t largest() const {
    size_t m = 0;
    for (auto &f : free_) m = std::max(m, f.second);
    return m;
  }
};

struct Snapshot {
  size_t off = 0, bytes = 0;
  bool submitted = false, done = false;
  int remaining = 0;
  szsel_result *out = nullptr;
  hipEvent_t ready = nullptr;  // producer's writes are complete
  double t_submit = 0.0, t_done = 0.0;
};

struct Pending {
  uint64_t ticket;
  int index;  // request index within its snapshot
  szsel_request req;
  size_t bytes;  // lane workspace it needs
};

struct Lane {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  szsel::BatchState *bs = nullptr;
  szsel_result *res = nullptr;  // pinned, kServeBatch results
  std::vector<std::pair<uint64_t, int>> parts;  // (ticket, index) of each request of the batch
  uint64_t seq = 0;  // launch order
  bool busy = false;
};

}  // namespace

struct szsel_server {
  szsel_ctx *ctx = nullptr;
  int ncu = 256;
  char *pool = nullptr;
  Arena arena;
  std::vector<Lane> lanes;
  std::deque<Pending> queue;
  std::map<uint64_t, Snapshot> snaps;
  uint64_t next_ticket = 1;
  std::string err;
  szsel::BatchOptions bopt;  // eager launches: served batches rarely repeat a shape
  size_t lane_budget = (size_t)4 << 30;
  int fail_batches = 0;  // test hook: the next this many lane batches fail before launching
  // statistics
  uint64_t batches = 0, batched_requests = 0, snapshots_done = 0, launches = 0, failed_requests = 0;
};

namespace {

int sfail(szsel_server *s, int code, const std::string &m) {
  s->err = m;
  return code;
}

// One request of snapshot `sn` has its result: completes the snapshot
// (releasing its pool range) when it was the last.  Returns 1 then.
int finish_one(szsel_server *s, Snapshot &sn, double t) {
  if (--sn.remaining) return 0;
  sn.done = true;
  sn.t_done = t;
  s->arena.release(sn.off, sn.bytes);
  if (sn.ready) (void)hipEventDestroy(sn.ready);
  sn.ready = nullptr;
  s->snapshots_done++;
  return 1;
}

// Retires finished lanes: distributes their results, completes snapshots
// and releases their pool ranges.  Returns the number of snapshots
// completed.
int retire(szsel_server *s, bool wait_one) {
  int completed = 0;
  if (wait_one) {  // the busy lane launched first
    Lane *old = nullptr;
    for (Lane &l : s->lanes)
      if (l.busy && (!old || l.seq < old->seq)) old = &l;
    if (old) (void)hipEventSynchronize(old->done);
  }
  for (Lane &l : s->lanes) {
    if (!l.busy || hipEventQuery(l.done) != hipSuccess) continue;
    const double t = now_ms();
    for (size_t k = 0; k < l.parts.size(); k++) {
      auto it = s->snaps.find(l.parts[k].first);
      if (it == s->snaps.end()) continue;
      Snapshot &sn = it->second;
      sn.out[l.parts[k].second] = l.res[k];
      completed += finish_one(s, sn, t);
    }
    l.parts.clear();
    l.busy = false;
  }
  return completed;
}

// Packs waiting requests onto free lanes: up to kServeBatch of them, and no
// more than the lane's workspace budget takes.  A batch that fails to
// launch goes back to the front of the queue and is retried in halves; a
// request that fails alone gets a result with SZSEL_FLAG_FAILED.
int dispatch(szsel_server *s) {
  int cap = kServeBatch;
  for (Lane &l : s->lanes) {
    while (!l.busy && !s->queue.empty()) {
      std::vector<szsel_request> reqs;
      std::vector<Pending> taken;
      std::vector<hipEvent_t> waits;
      size_t bytes = 0;
      while (!s->queue.empty() && (int)reqs.size() < cap) {
        Pending &p = s->queue.front();
        if (!reqs.empty() && bytes + p.bytes > s->lane_budget) break;
        bytes += p.bytes;
        Snapshot &sn = s->snaps[p.ticket];
        if (sn.ready && (waits.empty() || waits.back() != sn.ready)) waits.push_back(sn.ready);
        reqs.push_back(p.req);
        taken.push_back(p);
        s->queue.pop_front();
      }
      hipError_t e = hipSuccess;
      for (hipEvent_t ev : waits)
        if (e == hipSuccess) e = hipStreamWaitEvent(l.s, ev, 0);
      std::string msg;
      int rc = SZSEL_OK;
      if (e != hipSuccess) {
        rc = SZSEL_EHIP;
        msg = std::string("lane wait: ") + hipGetErrorString(e);
      } else if (s->fail_batches > 0) {
        s->fail_batches--;
        rc = SZSEL_EHIP;
        msg = "failure injected by SZSEL_SERVER_FAIL_BATCHES";
      } else {
        rc = szsel::batch_run(s->ctx, s->ncu, l.bs, s->lane_budget, reqs.data(), (int)reqs.size(), l.res, l.s,
                              s->bopt, msg);
      }
      if (rc == SZSEL_OK) {
        e = hipEventRecord(l.done, l.s);
        if (e != hipSuccess) return sfail(s, SZSEL_EHIP, std::string("hipEventRecord: ") + hipGetErrorString(e));
        l.parts.clear();
        for (const Pending &p : taken) l.parts.emplace_back(p.ticket, p.index);
        l.busy = true;
        l.seq = ++s->launches;
        s->batches++;
        s->batched_requests += reqs.size();
        break;
      }
      s->err = "batch of " + std::to_string(reqs.size()) + " requests failed: " + msg;
      if (taken.size() > 1) {  // back to the front, in order; retry in halves
        for (size_t k = taken.size(); k-- > 0;) s->queue.push_front(taken[k]);
        cap = std::max<int>(1, (int)taken.size() / 2);
        continue;
      }
      auto it = s->snaps.find(taken[0].ticket);
      if (it != s->snaps.end()) {
        szsel_result r;
        std::memset(&r, 0, sizeof(r));
        r.flags = SZSEL_FLAG_FAILED;
        r.choice = -1;
        it->second.out[taken[0].index] = r;
        s->failed_requests++;
        finish_one(s, it->second, now_ms());
      }
    }
  }
  return SZSEL_OK;
}

}  // namespace

extern "C" {

int szsel_server_create(szsel_server **out, szsel_ctx *ctx, void *pool, size_t pool_bytes, int lanes,
                        size_t lane_workspace_bytes) {
  if (!out) return SZSEL_EINVAL;
  *out = nullptr;
  if (lanes < 0 || lanes > 16 || (ctx && (!pool || lanes < 1))) return SZSEL_EINVAL;
  if ((uintptr_t)pool % kGranule) return SZSEL_EINVAL;
  szsel_server *s = new (std::nothrow) szsel_server();
  if (!s) return SZSEL_ENOMEM;
  s->ctx = ctx;
  s->pool = (char *)pool;
  s->arena.init(pool_bytes);
  if (lane_workspace_bytes) s->lane_budget = lane_workspace_bytes;
  s->bopt.graph = false;
  // one stream per lane: launched one by one (no graph), the two-stream
  // batch layout measured slower than one stream, and the lanes already
  // overlap each other's batches
  s->bopt.fixed.lanes = 1;
  if (const char *v = std::getenv("SZSEL_SERVER_FAIL_BATCHES")) s->fail_batches = std::max(0, std::atoi(v));
  if (ctx) {
    s->ncu = szsel::ctx_ncu(ctx);
    s->lanes.resize((size_t)lanes);
    for (Lane &l : s->lanes) {
      void *h = nullptr;
      if (hipStreamCreateWithFlags(&l.s, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess ||
          hipHostMalloc(&h, sizeof(szsel_result) * kServeBatch, hipHostMallocDefault) != hipSuccess) {
        szsel_server_destroy(s);
        return SZSEL_EHIP;
      }
      l.res = (szsel_result *)h;
      // part of the lane's workspace, allocated now (the fixed workspace of
      // up to a full batch within half the budget, and a quarter of the
      // budget of variable workspace): growing it while serving would
      // synchronise the device and stall every lane; the reservation also
      // makes the lane stream's first launch and transfers, on all lanes at
      // once (waited for below)
      const size_t per = szsel::request_fixed_bytes();
      const int nres = (int)std::min<size_t>((size_t)kServeBatch, s->lane_budget / 2 / per);
      if (nres >= 1) {
        std::string msg;
        const int rc = szsel::batch_reserve(l.bs, nres, s->lane_budget / 4, l.s, msg);
        if (rc != SZSEL_OK) {
          szsel_server_destroy(s);
          return rc;
        }
      }
    }
  }
  for (Lane &l : s->lanes)
    if (hipStreamSynchronize(l.s) != hipSuccess) {
      szsel_server_destroy(s);
      return SZSEL_EHIP;
    }
  *out = s;
  return SZSEL_OK;
}

void szsel_server_destroy(szsel_server *s) {
  if (!s) return;
  if (s->ctx) (void)hipDeviceSynchronize();
  for (Lane &l : s->lanes) {
    if (l.bs) szsel::batch_destroy(l.bs);
    if (l.s) (void)hipStreamDestroy(l.s);
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.res) (void)hipHostFree(l.res);
  }
  for (auto &kv : s->snaps)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  delete s;
}

int szsel_server_reserve(szsel_server *s, size_t bytes, void **dev_ptr, uint64_t *ticket) {
  if (!s || !dev_ptr || !ticket || bytes == 0) return SZSEL_EINVAL;
  if (bytes > s->arena.size) return sfail(s, SZSEL_ENOMEM, "snapshot larger than the pool");
  size_t off = 0;
  if (!s->arena.alloc(bytes, off)) return sfail(s, SZSEL_EBUSY, "pool full: wait for running snapshots");
  const uint64_t t = s->next_ticket++;
  Snapshot &sn = s->snaps[t];
  sn.off = off;
  sn.bytes = bytes;
  *dev_ptr = s->pool + off;
  *ticket = t;
  return SZSEL_OK;
}

int szsel_server_cancel(szsel_server *s, uint64_t ticket) {
  if (!s) return SZSEL_EINVAL;
  auto it = s->snaps.find(ticket);
  if (it == s->snaps.end() || it->second.submitted) return sfail(s, SZSEL_EINVAL, "no reservation to cancel");
  s->arena.release(it->second.off, it->second.bytes);
  s->snaps.erase(it);
  return SZSEL_OK;
}

int szsel_server_submit(szsel_server *s, uint64_t ticket, const szsel_request *reqs, int n, szsel_result *out,
                        void *producer_stream) {
  if (!s || !s->ctx || n < 1 || !reqs || !out) return SZSEL_EINVAL;
  auto it = s->snaps.find(ticket);
  if (it == s->snaps.end() || it->second.submitted) return sfail(s, SZSEL_EINVAL, "unknown or already submitted ticket");
  Snapshot &sn = it->second;
  const char *lo = s->pool + sn.off, *hi = lo + sn.bytes;
  std::vector<size_t> need((size_t)n);
  for (int i = 0; i < n; i++) {
    const szsel_request &q = reqs[i];
    const std::string who = "request " + std::to_string(i) + ": ";
    int32_t st[3] = {1, 1, 1};
    for (int k = 0; k < 3; k++) st[k] = q.stride[k] ? q.stride[k] : 1;
    std::string why;
    int rc = szsel::check_request(q.op, q.field, q.dims, q.ndims, q.dtype, q.eb, q.eb_mode, st, why);
    if (rc != SZSEL_OK) return sfail(s, rc, who + why);
    size_t b = q.dtype == SZSEL_F64 ? 8 : 4;
    for (int k = 0; k < q.ndims; k++) b *= (size_t)q.dims[k];
    const char *f = (const char *)q.field;
    if (f < lo || f + b > hi) return sfail(s, SZSEL_EINVAL, who + "field outside the snapshot's reservation");
    szsel::ReqDesc r;
    rc = szsel::plan_request(s->ctx, q.op, q.field, q.dims, q.ndims, q.dtype, q.eb, q.eb_mode, st, s->bopt.fixed, r);
    if (rc != SZSEL_OK) return sfail(s, rc, who + szsel_last_error(s->ctx));
    need[(size_t)i] = szsel::batch_request_bytes(r);
    if (need[(size_t)i] > s->lane_budget)
      return sfail(s, SZSEL_ENOMEM, who + "needs " + std::to_string(need[(size_t)i]) +
                                        " bytes of lane workspace, more than the lane budget");
  }
  if (producer_stream) {
    hipError_t e = hipEventCreateWithFlags(&sn.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(sn.ready, (hipStream_t)producer_stream);
    if (e != hipSuccess) return sfail(s, SZSEL_EHIP, std::string("producer event: ") + hipGetErrorString(e));
  }
  sn.submitted = true;
  sn.remaining = n;
  sn.out = out;
  sn.t_submit = now_ms();
  for (int i = 0; i < n; i++) s->queue.push_back(Pending{ticket, i, reqs[i], need[(size_t)i]});
  return dispatch(s);
}

int szsel_server_progress(szsel_server *s, int wait) {
  if (!s || !s->ctx) return SZSEL_EINVAL;
  bool busy = false;
  for (Lane &l : s->lanes) busy = busy || l.busy;
  int done = retire(s, wait && busy);
  const int rc = dispatch(s);
  if (rc != SZSEL_OK) return rc;
  return done;
}

int szsel_server_status(szsel_server *s, uint64_t ticket, double *latency_ms) {
  if (!s) return SZSEL_EINVAL;
  auto it = s->snaps.find(ticket);
  if (it == s->snaps.end()) return sfail(s, SZSEL_EINVAL, "unknown ticket");
  if (!it->second.done) return 0;
  if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
  s->snaps.erase(it);
  return 1;
}

int szsel_server_stats(const szsel_server *s, uint64_t *stats) {
  if (!s || !stats) return SZSEL_EINVAL;
  size_t pending = s->queue.size(), busy = 0;
  for (const Lane &l : s->lanes) busy += l.busy ? 1 : 0;
  stats[0] = s->batches;
  stats[1] = s->batched_requests;
  stats[2] = s->snapshots_done;
  stats[3] = pending;
  stats[4] = busy;
  stats[5] = s->arena.used;
  stats[6] = s->arena.size;
  stats[7] = s->arena.largest();
  return SZSEL_OK;
}

const char *szsel_server_last_error(const szsel_server *s) { return s ? s->err.c_str() : "no server"; }

}  // extern "C"
