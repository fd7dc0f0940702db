// Batched execution: n requests of any shape, dtype, bound and op in one
// launch per pass (the ZFP and SZ passes one per request class), captured
// as a HIP graph and replayed while the batch keeps the same launch shape.
//
// Table order.  Requests are sorted by (group, dtype, ndims, vector
// alignment, field size, field, dims) so that every class of kernel
// template is a contiguous range of the device table, and requests on the
// same field are adjacent: the first of them scans the value range once for
// all (nshare), the others get no range work items.  Results are written at
// the caller's indices.
//
// Workspace.  Each table entry owns a fixed part (state, counters,
// histogram, ...; zeroed once, kept clean by the kernels) and a variable
// part (partials, overflow regions).  Each batch state also holds the table
// and the per-pass prefix counts (device), their pinned staging copy, and
// the captured graph.
//
// Autotuning.  The launch shape knobs (Tune) never change the results; the
// tuner times a few candidates per batch shape on the caller's stream and
// keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>

#include "batch.hpp"
#include "launch.hpp"

struct szsel_ctx;

namespace szsel {

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr int kMaxGroupsPerBatch = 8;
constexpr int kGraphCache = 8;         // captured graphs kept per batch state

struct Plan {
  std::vector<ReqDesc> tab;             // table order
  std::vector<int> orig;                // caller index of each table entry
  std::vector<uint32_t> first;          // kBatchPasses x (n + 1) prefix counts
  std::vector<BatchLaunch> launches;    // in pass order (tab/first pointers filled at bind time)
  std::vector<size_t> voff;             // variable workspace offset of each table entry
  size_t var = 0;                       // variable workspace bytes
  std::vector<uint64_t> sig;            // launch shape (graph reuse key)
  int groups = 1;                       // request groups (streams)
};

bool same_field(const ReqDesc &a, const ReqDesc &b) {
  if (a.field != b.field || a.dtype != b.dtype || a.nd != b.nd) return false;
  for (int k = 0; k < a.nd; k++)
    if (a.dims[k] != b.dims[k]) return false;
  return true;
}

// Plans every request with the knobs `tu` and lays out the table, prefix
// counts and launches.
int make_plan(szsel_ctx *ctx, int ncu, const szsel_request *reqs, int n, const Tune &tu, Plan &p,
              std::string &msg) {
  std::vector<ReqDesc> d((size_t)n);
  for (int i = 0; i < n; i++) {
    const szsel_request &q = reqs[i];
    int32_t st[3];
    for (int k = 0; k < 3; k++) st[k] = q.stride[k] > 0 ? q.stride[k] : 1;
    const int rc = plan_request(ctx, q.op, q.field, q.dims, q.ndims, q.dtype, q.eb, q.eb_mode, st, tu, d[i]);
    if (rc != SZSEL_OK) {
      msg = "request " + std::to_string(i) + ": ";
      return rc;
    }
  }
  // Workgroup counts.  tu.share >= 1: the schedule's SZ count is the
  // batch's, dealt to the requests in proportion to their sampled blocks,
  // and (tu.share == 2) its range count too, in proportion to the bytes of
  // their fields (a field scanned once for all its requests counts once),
  // so that the small fields of a large batch get a few long-running
  // workgroups instead of many whose time goes to their set-up, the SZ LDS
  // histogram's clearing and hand-over and the completion counters.  With
  // tu.share == 3 the SZ count is dealt within each launch class (dtype,
  // rank, alignment, point sub-sampling) instead: the classes run as
  // launches of their own (one after another, or two at a time on two
  // stream lanes), and each should fill the chip (a small binary64 class dealt its share of the whole batch's count
  // runs on a few long workgroups).  The ZFP waves (tu.zfp_waves per CU)
  // are dealt within each launch class in every mode.
  if (n > 1) {
    auto cls = [&](int i) { return (d[i].dtype * 8 + d[i].nd) * 4 + (d[i].vec ? 2 : 0) + (d[i].ec ? 1 : 0); };
    auto sz_class = [&](int i) { return tu.share == 3 ? cls(i) : 0; };
    std::map<int, double> sz_blocks, zfp_blocks;
    double scan_bytes = 0.0;
    for (int i = 0; i < n; i++) {
      if (d[i].op != SZSEL_OP_ZFP) sz_blocks[sz_class(i)] += (double)d[i].nblk;
      if (d[i].op != SZSEL_OP_SZ) zfp_blocks[cls(i)] += (double)d[i].nblk;
      bool first_on_field = true;
      for (int j = 0; j < i && first_on_field; j++) first_on_field = !same_field(d[i], d[j]);
      if (first_on_field) scan_bytes += (double)d[i].n * (d[i].dtype == SZSEL_F32 ? 4.0 : 8.0);
    }
    const double sz_want = std::max(1.0, (double)tu.sz_wgs_q * (double)ncu / 4.0);
    const double range_want = std::max(1.0, (double)tu.range_wgs_q * (double)ncu / 4.0);
    const double zfp_want = (double)std::max(1, tu.zfp_waves) * (double)ncu;
    auto share = [](double want, double part, double whole) {
      return (int)std::max(1.0, std::min(1e9, std::round(want * part / whole)));
    };
    for (int i = 0; i < n; i++) {
      const szsel_request &q = reqs[i];
      int32_t st[3];
      for (int k = 0; k < 3; k++) st[k] = q.stride[k] > 0 ? q.stride[k] : 1;
      Tune t = tu;
      const double sb = sz_blocks[sz_class(i)], zb = zfp_blocks[cls(i)];
      if (tu.share > 0 && d[i].op != SZSEL_OP_ZFP && d[i].nblk > 0 && sb > 0.0)
        t.sz_target = share(sz_want, (double)d[i].nblk, sb);
      if (d[i].op != SZSEL_OP_SZ && d[i].nblk > 0 && zb > 0.0) t.zfp_target = share(zfp_want, (double)d[i].nblk, zb);
      if (tu.share == 2 && scan_bytes > 0.0)
        t.range_target = share(range_want, (double)d[i].n * (d[i].dtype == SZSEL_F32 ? 4.0 : 8.0), scan_bytes);
      const int rc = plan_request(ctx, q.op, q.field, q.dims, q.ndims, q.dtype, q.eb, q.eb_mode, st, t, d[i]);
      if (rc != SZSEL_OK) {
        msg = "request " + std::to_string(i) + ": ";
        return rc;
      }
    }
  }
  // request groups: requests on one field stay together (they share the
  // scan); fields are dealt to the groups largest first, each to the group
  // with the least estimated work (range bytes plus 8 bytes per sampled value)
  const int G = std::max(1, std::min(tu.groups, kMaxGroupsPerBatch));
  std::vector<int> grp((size_t)n, 0);
  if (G > 1) {
    std::vector<int> unit((size_t)n, -1);
    std::vector<double> ucost;
    std::vector<int> urep;
    for (int i = 0; i < n; i++) {
      for (int j = 0; j < i && unit[i] < 0; j++)
        if (same_field(d[i], d[j])) unit[i] = unit[j];
      const double sampled = (double)d[i].nblk * (double)(1 << (2 * d[i].nd)) * 8.0;
      if (unit[i] < 0) {
        unit[i] = (int)ucost.size();
        ucost.push_back((double)d[i].n * (d[i].dtype == SZSEL_F32 ? 4.0 : 8.0) + sampled);
        urep.push_back(i);
      } else {
        ucost[unit[i]] += sampled;
      }
    }
    std::vector<int> uo(ucost.size());
    std::iota(uo.begin(), uo.end(), 0);
    std::stable_sort(uo.begin(), uo.end(), [&](int a, int b) { return ucost[a] > ucost[b]; });
    std::vector<double> load((size_t)G, 0.0);
    std::vector<int> ug(ucost.size(), 0);
    for (int u : uo) {
      const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      ug[u] = g;
      load[g] += ucost[u];
    }
    for (int i = 0; i < n; i++) grp[i] = ug[unit[i]];
  }
  std::vector<int> ord((size_t)n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    const ReqDesc &x = d[a], &y = d[b];
    if (grp[a] != grp[b]) return grp[a] < grp[b];
    if (x.dtype != y.dtype) return x.dtype < y.dtype;
    if (x.nd != y.nd) return x.nd < y.nd;
    if (x.vec != y.vec) return x.vec > y.vec;
    // larger fields first within a class: the range launch's last
    // workgroups are then the small fields' short chunks
    if (x.n != y.n) return x.n > y.n;
    if (x.field != y.field) return (uintptr_t)x.field < (uintptr_t)y.field;
    for (int k = 0; k < x.nd; k++)
      if (x.dims[k] != y.dims[k]) return x.dims[k] < y.dims[k];
    return false;
  });
  p.tab.resize((size_t)n);
  p.orig = ord;
  p.groups = G;
  std::vector<int> tg((size_t)n);
  for (int k = 0; k < n; k++) {
    p.tab[k] = d[ord[k]];
    tg[k] = grp[ord[k]];
  }
  // one request group and two lanes: the passes after the range scans run
  // on the caller's stream for the table entries of lane 0 and on a side
  // stream for those of lane 1, so that the passes of the two lanes
  // overlap.  tu.lanes == 2 deals the launch classes (dtype, rank,
  // alignment, point sub-sampling) to the lanes in turn when there are
  // several (one class's latency-bound pass then runs beside another's
  // VALU-bound one); with one class, or tu.lanes == 3, the table is cut
  // where half of the estimated sampled work lies before it (sampled
  // values, binary64 ones counted twice), a class cut in two getting
  // launches of its own on either side.
  const bool class_lanes = G == 1 && tu.lanes > 1;
  std::vector<int> lane((size_t)n, 0);
  auto class_of = [&](int k) {
    const ReqDesc &r = p.tab[k];
    return ((r.dtype * 8 + r.nd) * 2 + r.vec) * 2 + (r.ec ? 1 : 0);
  };
  int nclass = 0;
  for (int k = 0; k < n; k++) nclass += (k == 0 || class_of(k) != class_of(k - 1)) ? 1 : 0;
  if (class_lanes && tu.lanes == 2 && nclass > 1) {
    int ord = 0;
    for (int k = 0; k < n; k++) {
      if (k > 0 && class_of(k) != class_of(k - 1)) ord++;
      lane[k] = ord & 1;
    }
  } else if (class_lanes) {
    std::vector<double> w((size_t)n);
    double total = 0.0;
    for (int k = 0; k < n; k++) {
      const ReqDesc &r = p.tab[k];
      w[k] = (double)r.nblk * (double)(1 << (2 * r.nd)) * (r.dtype == SZSEL_F32 ? 1.0 : 2.0);
      total += w[k];
    }
    double before = 0.0;
    for (int k = 0; k < n; k++) {
      lane[k] = before + 0.5 * w[k] > 0.5 * total ? 1 : 0;
      before += w[k];
    }
  }
  // range scans shared by runs of requests on the same field
  std::vector<bool> owner((size_t)n, true);
  for (int k = 0; k < n;) {
    int e = k + 1;
    while (e < n && tg[e] == tg[k] && same_field(p.tab[k], p.tab[e])) e++;
    p.tab[k].nshare = e - k - 1;
    for (int m = k + 1; m < e; m++) {
      p.tab[m].nshare = 0;
      owner[m] = false;
    }
    k = e;
  }
  // prefix counts of work items per pass
  p.first.assign((size_t)kBatchPasses * (n + 1), 0);
  for (int ps = 0; ps < kBatchPasses; ps++) {
    uint32_t acc = 0;
    for (int k = 0; k < n; k++) {
      const ReqDesc &r = p.tab[k];
      uint32_t c = 0;
      switch (ps) {
        case kBatchRange: c = owner[k] ? (uint32_t)r.nrange : 0u; break;
        case kBatchZfp: c = r.op != SZSEL_OP_SZ ? (uint32_t)r.nzfp : 0u; break;
        case kBatchSz: c = r.op != SZSEL_OP_ZFP ? (uint32_t)r.nsz : 0u; break;
        case kBatchOvf: c = r.op != SZSEL_OP_ZFP ? (uint32_t)(kOvfSlices * kOvfRanges) : 0u; break;
        case kBatchEnt: c = r.op != SZSEL_OP_ZFP ? (uint32_t)kEntWgs : 0u; break;
        default: c = r.op != SZSEL_OP_ZFP && r.huff ? 1u : 0u; break;
      }
      p.first[(size_t)ps * (n + 1) + k] = acc;
      acc += c;
    }
    p.first[(size_t)ps * (n + 1) + n] = acc;
  }
  // launches: per pass, one per contiguous class and lane (the range pass,
  // whose kernel takes any class, one per request group; the overflow and
  // entropy passes likewise unless the batch runs on two lanes)
  p.launches.clear();
  for (int ps = 0; ps < kBatchPasses; ps++) {
    const uint32_t *f = &p.first[(size_t)ps * (n + 1)];
    for (int k = 0; k < n;) {
      int e = k + 1;
      auto same_class = [&](int a, int b) {
        if (tg[a] != tg[b]) return false;
        const ReqDesc &x = p.tab[a], &y = p.tab[b];
        if (ps == kBatchRange) return true;
        if (lane[a] != lane[b]) return false;
        if ((ps == kBatchOvf || ps == kBatchEnt) && !class_lanes) return true;
        return x.dtype == y.dtype && x.nd == y.nd && x.vec == y.vec && (x.ec != 0) == (y.ec != 0);
      };
      while (e < n && same_class(k, e)) e++;
      BatchLaunch L;
      L.group = tg[k];
      L.pass = ps;
      L.dtype = p.tab[k].dtype;
      L.nd = p.tab[k].nd;
      L.vec = p.tab[k].vec;
      L.ec = p.tab[k].ec != 0;
      L.tab = nullptr;
      L.first = nullptr;
      L.c0 = k;
      L.c1 = e;
      L.lane = ps == kBatchRange ? 0 : lane[k];
      L.items = f[e] - f[k];
      L.grid = L.items;
      if (ps == kBatchRange && tu.range_grid > 0)
        L.grid = std::min<uint32_t>(L.items, (uint32_t)tu.range_grid * (uint32_t)ncu);
      if (ps == kBatchOvf) L.grid = std::min<uint32_t>(L.items, 2u * (uint32_t)ncu);
      if (ps == kBatchEnt) L.grid = std::min<uint32_t>(L.items, 8u * (uint32_t)ncu);
      if (L.items) p.launches.push_back(L);
      k = e;
    }
  }
  // variable workspace
  p.voff.resize((size_t)n);
  p.var = 0;
  for (int k = 0; k < n; k++) {
    p.voff[k] = p.var;
    p.var = align_up(p.var + request_var_bytes(p.tab[k]), 256);
  }
  // launch shape: everything the captured graph depends on except the
  // table contents (field pointers and bounds are uploaded on every call)
  p.sig.clear();
  p.sig.push_back((uint64_t)n);
  p.sig.push_back((uint64_t)G);
  for (int k = 0; k < n; k++) p.sig.push_back((uint64_t)p.orig[k]);
  for (uint32_t v : p.first) p.sig.push_back(v);
  for (const BatchLaunch &L : p.launches)
    p.sig.push_back(((uint64_t)L.group << 59) | ((uint64_t)L.pass << 56) | ((uint64_t)L.dtype << 52) | ((uint64_t)L.nd << 48) |
                    ((uint64_t)L.vec << 47) | ((uint64_t)L.ec << 46) | ((uint64_t)L.grid << 24) |
                    ((uint64_t)L.c0 << 12) | (uint64_t)L.c1);
  for (const BatchLaunch &L : p.launches) p.sig.push_back((uint64_t)L.lane);
  for (size_t v : p.voff) p.sig.push_back(v);
  return SZSEL_OK;
}

// Shape of a batch independent of the knobs (the autotuner's cache key).
std::vector<uint64_t> shape_key(const szsel_request *reqs, int n) {
  std::vector<uint64_t> k;
  k.push_back((uint64_t)n);
  for (int i = 0; i < n; i++) {
    const szsel_request &q = reqs[i];
    k.push_back(((uint64_t)q.dtype << 8) | ((uint64_t)q.ndims << 4) | (uint64_t)q.op);
    for (int a = 0; a < 3; a++) k.push_back((uint64_t)(a < q.ndims ? q.dims[a] : 0));
    for (int a = 0; a < 3; a++) k.push_back((uint64_t)(a < q.ndims ? q.stride[a] : 0));
    k.push_back(((uintptr_t)q.field % 16) ? 1u : 0u);
    // requests on one field share a scan: record the first index using it
    int same = i;
    for (int j = 0; j < i; j++)
      if (reqs[j].field == q.field) {
        same = j;
        break;
      }
    k.push_back((uint64_t)same);
  }
  return k;
}

hipError_t dev_grow(char *&buf, size_t &have, size_t want, bool zero) {
  if (want <= have) return hipSuccess;
  hipError_t e = hipDeviceSynchronize();
  if (buf) (void)hipFree(buf);
  buf = nullptr;
  have = 0;
  void *q = nullptr;
  if (e == hipSuccess) e = hipMalloc(&q, want);
  if (e == hipSuccess && zero) e = hipMemset(q, 0, want);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (q) (void)hipFree(q);
    return e;
  }
  buf = (char *)q;
  have = want;
  return hipSuccess;
}

}  // namespace

struct BatchState {
  char *fixed = nullptr;  // request_fixed_bytes() per table entry, zeroed on allocation
  size_t fixed_cap = 0;
  char *var = nullptr;
  size_t var_cap = 0;
  char *res = nullptr;  // results at the caller's indices
  size_t res_cap = 0;
  char *meta = nullptr;  // device table + prefix counts
  size_t meta_cap = 0;
  char *stage = nullptr;  // pinned staging copy of meta
  size_t stage_cap = 0;
  std::vector<char> staged;  // what the staging buffer holds
  bool dirty = false;        // staging rewritten since the last upload to meta
  hipEvent_t done = nullptr;
  bool used = false;
  hipStream_t cap = nullptr;  // private capture stream
  hipStream_t scan = nullptr;  // side stream of the range scans (request groups)
  hipEvent_t fork = nullptr;
  hipEvent_t scanned[kMaxGroupsPerBatch] = {};    // group g's range scans are done
  struct Graph {
    std::vector<uint64_t> key;  // launch shape, result destination
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  std::vector<Graph> graphs;  // captured graphs, the least recently used replaced
  uint64_t clock = 0;
  std::vector<const void *> outs;  // result destinations of the last calls
  std::vector<uint64_t> last_key;  // last batch shape, and its knobs
  Tune last_tune;
  bool last_auto = false;
  bool have_last = false;
};

size_t batch_request_bytes(const ReqDesc &r) {
  return request_fixed_bytes() + align_up(request_var_bytes(r), 256) + sizeof(szsel_result) + sizeof(ReqDesc) +
         sizeof(uint32_t) * kBatchPasses + 512;
}

size_t batch_state_bytes(const BatchState *bs) {
  return bs ? bs->fixed_cap + bs->var_cap + bs->res_cap + bs->meta_cap : 0;
}

void batch_destroy(BatchState *bs) {
  if (!bs) return;
  (void)hipDeviceSynchronize();
  for (BatchState::Graph &g : bs->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (bs->cap) (void)hipStreamDestroy(bs->cap);
  if (bs->scan) (void)hipStreamDestroy(bs->scan);
  if (bs->fork) (void)hipEventDestroy(bs->fork);
  for (int g = 0; g < kMaxGroupsPerBatch; g++) {
    if (bs->scanned[g]) (void)hipEventDestroy(bs->scanned[g]);
  }
  if (bs->fixed) (void)hipFree(bs->fixed);
  if (bs->var) (void)hipFree(bs->var);
  if (bs->res) (void)hipFree(bs->res);
  if (bs->meta) (void)hipFree(bs->meta);
  if (bs->stage) (void)hipHostFree(bs->stage);
  if (bs->done) (void)hipEventDestroy(bs->done);
  delete bs;
}

namespace {

// Tuned schedules per (device architecture, batch shape), shared by the
// process's contexts.  With SZSEL_TUNE_CACHE naming a file, the schedules
// of earlier processes are read from it on first use, and every newly
// tuned one is appended, one JSON object per line:
//   {"build":"...","arch":"gfx950...","key":[...],"tune":{"sz_wgs_q":8,...}}
// Lines of another build of the library (the schedule's best value depends
// on the kernels) or that do not parse are skipped.
constexpr const char *kTuneBuild = __DATE__ " " __TIME__;

struct Tuner {
  std::map<std::pair<std::string, std::vector<uint64_t>>, Tune> best;
  std::mutex mu;
  bool loaded = false;
  std::string path;
};
Tuner &tuner() {
  static Tuner t;
  return t;
}

// The knobs of a schedule as (JSON name, member) pairs.
template <typename F>
void tune_fields(Tune &t, F f) {
  f("sz_wgs_q", t.sz_wgs_q);
  f("zfp_chunk", t.zfp_chunk);
  f("zfp_waves", t.zfp_waves);
  f("range_wgs_q", t.range_wgs_q);
  f("range_grid", t.range_grid);
  f("groups", t.groups);
  f("lanes", t.lanes);
  f("ovf_slice", t.ovf_slice);
  f("share", t.share);
}

// The string value of "name" in one line of the cache, or false.
bool json_str(const std::string &line, const char *name, std::string &out) {
  const std::string pat = std::string("\"") + name + "\":\"";
  const size_t a = line.find(pat);
  if (a == std::string::npos) return false;
  const size_t b = line.find('"', a + pat.size());
  if (b == std::string::npos) return false;
  out = line.substr(a + pat.size(), b - a - pat.size());
  return true;
}

// Parses one cache line; false if it is not a complete entry.
bool parse_tune_line(const std::string &line, std::string &build, std::string &arch,
                     std::vector<uint64_t> &key, Tune &t) {
  if (!json_str(line, "build", build) || !json_str(line, "arch", arch)) return false;
  const size_t k0 = line.find("\"key\":[");
  if (k0 == std::string::npos) return false;
  const char *p = line.c_str() + k0 + 7;
  key.clear();
  while (*p && *p != ']') {
    char *end = nullptr;
    const unsigned long long v = std::strtoull(p, &end, 10);
    if (end == p) return false;
    key.push_back((uint64_t)v);
    p = end;
    if (*p == ',') p++;
  }
  if (*p != ']' || key.empty()) return false;
  bool ok = true;
  tune_fields(t, [&](const char *name, int &v) {
    const std::string pat = std::string("\"") + name + "\":";
    const size_t a = line.find(pat);
    if (a == std::string::npos) {
      ok = false;
      return;
    }
    char *end = nullptr;
    const long x = std::strtol(line.c_str() + a + pat.size(), &end, 10);
    if (end == line.c_str() + a + pat.size() || x < 0 || x > (1l << 30)) ok = false;
    v = (int)x;
  });
  return ok && t.groups >= 1 && t.sz_wgs_q >= 1 && t.zfp_chunk >= 1 && t.zfp_waves >= 1 && t.range_wgs_q >= 1 &&
         t.range_grid >= 0 && t.lanes >= 1 && t.lanes <= 3 &&
         t.ovf_slice >= 1 && t.share <= 3;
}

// Reads the cache file once per process (the tuner's lock held).
void tune_cache_load(Tuner &T) {
  if (T.loaded) return;
  T.loaded = true;
  const char *env = std::getenv("SZSEL_TUNE_CACHE");
  if (!env || !*env) return;
  T.path = env;
  std::ifstream in(T.path);
  std::string line;
  while (std::getline(in, line)) {
    std::string build, arch;
    std::vector<uint64_t> key;
    Tune t;
    if (parse_tune_line(line, build, arch, key, t) && build == kTuneBuild)
      T.best[std::make_pair(arch, key)] = t;
  }
}

// Appends one tuned schedule to the cache file (the tuner's lock held).
void tune_cache_append(Tuner &T, const std::string &arch, const std::vector<uint64_t> &key, Tune t) {
  if (T.path.empty()) return;
  std::ostringstream o;
  o << "{\"build\":\"" << kTuneBuild << "\",\"arch\":\"" << arch << "\",\"key\":[";
  for (size_t i = 0; i < key.size(); i++) o << (i ? "," : "") << key[i];
  o << "],\"tune\":{";
  bool first = true;
  tune_fields(t, [&](const char *name, int &v) {
    o << (first ? "" : ",") << "\"" << name << "\":" << v;
    first = false;
  });
  o << "}}\n";
  std::ofstream out(T.path, std::ios::app);
  out << o.str();
}

// Waits until the state's last batch (and with it every copy from its
// staging buffer and every read of its workspace) is finished.
hipError_t batch_wait(BatchState *bs) {
  return bs->used ? hipEventSynchronize(bs->done) : hipSuccess;
}

// Makes the state's buffers large enough for plan p, binds every table
// entry to its workspace and result, and rewrites the staging copy when
// the table or the prefix counts differ from what it holds (after the
// state's last batch is finished; an unchanged plan waits for nothing, so
// the host can queue the next batch while one runs).
hipError_t bind_plan(BatchState *bs, Plan &p, size_t budget, std::string &msg) {
  const size_t n = p.tab.size();
  const size_t fixed = request_fixed_bytes();
  const size_t tab_bytes = align_up(sizeof(ReqDesc) * n, 256);
  const size_t meta = tab_bytes + sizeof(uint32_t) * p.first.size();
  const size_t need = fixed * n + p.var + sizeof(szsel_result) * n + meta;
  if (need > budget) {
    msg = "batch workspace of " + std::to_string(need) + " bytes exceeds the budget of " + std::to_string(budget);
    return hipErrorOutOfMemory;
  }
  hipError_t e = hipSuccess;
  const size_t total = std::max(bs->fixed_cap, fixed * n) + std::max(bs->var_cap, p.var) +
                       std::max(bs->res_cap, sizeof(szsel_result) * n) + std::max(bs->meta_cap, meta);
  if (total > budget) {
    // buffers grown by earlier batches of another shape: release them all
    // (and the graphs that point into them) and allocate what this one needs
    e = batch_wait(bs);
    if (e != hipSuccess) {
      msg = std::string("batch: ") + hipGetErrorString(e);
      return e;
    }
    for (BatchState::Graph &g : bs->graphs) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    bs->graphs.clear();
    for (char **b : {&bs->fixed, &bs->var, &bs->res, &bs->meta})
      if (*b) (void)hipFree(*b), *b = nullptr;
    bs->fixed_cap = bs->var_cap = bs->res_cap = bs->meta_cap = 0;
    bs->staged.clear();
  }
  if (fixed * n > bs->fixed_cap || p.var > bs->var_cap || sizeof(szsel_result) * n > bs->res_cap ||
      meta > bs->meta_cap || meta > bs->stage_cap)
    e = batch_wait(bs);
  if (e == hipSuccess && fixed * n > bs->fixed_cap) e = dev_grow(bs->fixed, bs->fixed_cap, fixed * n, true);
  if (e == hipSuccess) e = dev_grow(bs->var, bs->var_cap, p.var, false);
  if (e == hipSuccess) e = dev_grow(bs->res, bs->res_cap, sizeof(szsel_result) * n, false);
  if (e == hipSuccess && meta > bs->meta_cap) {
    bs->staged.clear();  // a new device table holds nothing yet
    e = dev_grow(bs->meta, bs->meta_cap, meta, false);
  }
  if (e == hipSuccess && meta > bs->stage_cap) {
    bs->staged.clear();
    if (bs->stage) (void)hipHostFree(bs->stage);
    bs->stage = nullptr;
    bs->stage_cap = 0;
    void *h = nullptr;
    e = hipHostMalloc(&h, meta, hipHostMallocDefault);
    if (e == hipSuccess) {
      bs->stage = (char *)h;
      bs->stage_cap = meta;
    }
  }
  if (e != hipSuccess) {
    msg = std::string("batch workspace: ") + hipGetErrorString(e);
    return e;
  }
  szsel_result *res = (szsel_result *)bs->res;
  for (size_t k = 0; k < n; k++) {
    ReqDesc &r = p.tab[k];
    bind_request_workspace(r, bs->fixed + k * fixed, bs->var + p.voff[k]);
    r.res = res + p.orig[k];
  }
  const ReqDesc *dtab = (const ReqDesc *)bs->meta;
  const uint32_t *dfirst = (const uint32_t *)(bs->meta + tab_bytes);
  for (BatchLaunch &L : p.launches) {
    L.tab = dtab;
    L.first = dfirst + (size_t)L.pass * (n + 1);
  }
  std::vector<char> img(meta, 0);
  std::memcpy(img.data(), p.tab.data(), sizeof(ReqDesc) * n);
  std::memcpy(img.data() + tab_bytes, p.first.data(), sizeof(uint32_t) * p.first.size());
  if (img != bs->staged) {
    e = batch_wait(bs);
    if (e != hipSuccess) {
      msg = std::string("batch: ") + hipGetErrorString(e);
      return e;
    }
    std::memcpy(bs->stage, img.data(), meta);
    bs->staged.swap(img);
    bs->dirty = true;
  }
  // buffer addresses are part of what a captured graph depends on
  p.sig.push_back((uint64_t)(uintptr_t)bs->fixed);
  p.sig.push_back((uint64_t)(uintptr_t)bs->var);
  p.sig.push_back((uint64_t)(uintptr_t)bs->res);
  p.sig.push_back((uint64_t)(uintptr_t)bs->meta);
  p.sig.push_back((uint64_t)(uintptr_t)bs->stage);
  return hipSuccess;
}

// Upload of the staged table and prefix counts when they changed, on
// stream s (ahead of the launches that read them; not part of a graph).
hipError_t upload_meta(BatchState *bs, hipStream_t s) {
  if (!bs->dirty) return hipSuccess;
  const hipError_t e = hipMemcpyAsync(bs->meta, bs->stage, bs->staged.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) bs->dirty = false;
  return e;
}

// One launch, with the timer's event pair around it when profiling.
hipError_t timed_launch(const BatchLaunch &L, hipStream_t s, LaunchTimer *lt) {
  if (!lt) return launch_batch_pass(L, s);
  const size_t k = lt->used;
  hipError_t e = hipSuccess;
  while (e == hipSuccess && lt->ev.size() < 2 * (k + 1)) {
    hipEvent_t ev = nullptr;
    e = hipEventCreate(&ev);
    if (e == hipSuccess) lt->ev.push_back(ev);
  }
  if (e != hipSuccess) return e;
  if (lt->tag.size() < k + 1) lt->tag.resize(k + 1);
  lt->tag[k] = 2 * L.pass + L.dtype;
  e = hipEventRecord(lt->ev[2 * k], s);
  if (e == hipSuccess) e = launch_batch_pass(L, s);
  if (e == hipSuccess) e = hipEventRecord(lt->ev[2 * k + 1], s);
  if (e == hipSuccess) lt->used = k + 1;
  return e;
}

// Every launch of plan p, on stream s.  With one request group and launches
// on lane 1, the side stream forks from s after the range scans, takes the
// lane-1 launches while s takes the others, and s waits for it at the
// end.  With G > 1 request groups the range scans of
// all groups run back to back on the side stream, each group's followed
// by an event, and the sampled passes of group g run on s once group g's
// scans are done: the scans of later groups overlap the sampled passes of
// earlier ones.  Either way a graph captured from this forks into two
// streams, and s waits for the side stream (its own waits already do)
// before the results are read.  Timed launches (the profile) all run on s,
// one after another, so that their event pairs time one launch each.
hipError_t enqueue_plan(BatchState *bs, const Plan &p, hipStream_t s, LaunchTimer *lt = nullptr) {
  hipError_t e = hipSuccess;
  const int G = p.groups;
  if (G == 1) {
    bool lanes = false;
    for (const BatchLaunch &L : p.launches) lanes = lanes || L.lane != 0;
    if (!lanes || lt) {
      for (size_t k = 0; k < p.launches.size() && e == hipSuccess; k++) e = timed_launch(p.launches[k], s, lt);
      return e;
    }
    // the range launches, then the other passes on two lanes (the side
    // stream forked after the scans and joined at the end)
    const size_t n = p.launches.size();
    size_t k = 0;
    for (; k < n && p.launches[k].pass == kBatchRange && e == hipSuccess; k++) e = timed_launch(p.launches[k], s, lt);
    if (e == hipSuccess) e = hipEventRecord(bs->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(bs->scan, bs->fork, 0);
    const bool forked = e == hipSuccess;
    for (; k < n && e == hipSuccess; k++) e = timed_launch(p.launches[k], p.launches[k].lane ? bs->scan : s, lt);
    if (forked) {  // joined even after a failed launch: s must not run ahead of the side stream
      hipError_t j = hipEventRecord(bs->scanned[0], bs->scan);
      if (j == hipSuccess) j = hipStreamWaitEvent(s, bs->scanned[0], 0);
      if (e == hipSuccess) e = j;
    }
    return e;
  }
  hipStream_t scan = bs->scan;
  e = hipEventRecord(bs->fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(scan, bs->fork, 0);
  const bool forked = e == hipSuccess;
  for (int g = 0; g < G && e == hipSuccess; g++) {
    for (size_t k = 0; k < p.launches.size() && e == hipSuccess; k++)
      if (p.launches[k].group == g && p.launches[k].pass == kBatchRange) e = timed_launch(p.launches[k], scan, lt);
    if (e == hipSuccess) e = hipEventRecord(bs->scanned[g], scan);
  }
  for (int g = 0; g < G && e == hipSuccess; g++) {
    e = hipStreamWaitEvent(s, bs->scanned[g], 0);
    for (size_t k = 0; k < p.launches.size() && e == hipSuccess; k++)
      if (p.launches[k].group == g && p.launches[k].pass != kBatchRange) e = timed_launch(p.launches[k], s, lt);
  }
  if (forked && e != hipSuccess) {  // after a failure s still waits for all of the side stream
    if (hipEventRecord(bs->scanned[0], scan) == hipSuccess) (void)hipStreamWaitEvent(s, bs->scanned[0], 0);
  }
  return e;
}

}  // namespace

// A batch state with its events and streams (no buffers yet).
static bool batch_state_create(BatchState *&bs, std::string &msg) {
  bs = new BatchState();
  bool ok = hipEventCreateWithFlags(&bs->done, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&bs->fork, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&bs->cap, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&bs->scan, hipStreamNonBlocking) == hipSuccess;
  for (int g = 0; g < kMaxGroupsPerBatch && ok; g++)
    ok = hipEventCreateWithFlags(&bs->scanned[g], hipEventDisableTiming) == hipSuccess;
  if (!ok) msg = "batch state: event or stream creation failed";
  return ok;
}

__global__ void k_stream_warm() {}

int batch_reserve(BatchState *&bs, int nreq, size_t var_bytes, hipStream_t s, std::string &msg) {
  if (nreq < 1 || nreq > kMaxBatch) {
    msg = "batch reserve: 1 to " + std::to_string(kMaxBatch) + " requests";
    return SZSEL_EINVAL;
  }
  if (!bs && !batch_state_create(bs, msg)) return SZSEL_EHIP;
  const size_t n = (size_t)nreq;
  const size_t meta = align_up(sizeof(ReqDesc) * n, 256) + sizeof(uint32_t) * (size_t)kBatchPasses * (n + 1);
  hipError_t e = batch_wait(bs);
  if (e == hipSuccess && request_fixed_bytes() * n > bs->fixed_cap)
    e = dev_grow(bs->fixed, bs->fixed_cap, request_fixed_bytes() * n, true);
  if (e == hipSuccess) e = dev_grow(bs->var, bs->var_cap, var_bytes, false);
  if (e == hipSuccess) e = dev_grow(bs->res, bs->res_cap, sizeof(szsel_result) * n, false);
  if (e == hipSuccess && meta > bs->meta_cap) {
    bs->staged.clear();
    e = dev_grow(bs->meta, bs->meta_cap, meta, false);
  }
  if (e == hipSuccess && meta > bs->stage_cap) {
    bs->staged.clear();
    if (bs->stage) (void)hipHostFree(bs->stage);
    bs->stage = nullptr;
    bs->stage_cap = 0;
    void *h = nullptr;
    e = hipHostMalloc(&h, meta, hipHostMallocDefault);
    if (e == hipSuccess) {
      bs->stage = (char *)h;
      bs->stage_cap = meta;
    }
  }
  if (e != hipSuccess) {
    msg = std::string("batch reserve: ") + hipGetErrorString(e);
    return SZSEL_ENOMEM;
  }
  // first launch and transfers of the stream (the staged table is marked
  // empty, so the next batch uploads its own)
  bs->staged.clear();
  hipLaunchKernelGGL(k_stream_warm, dim3(1), dim3(kWave), 0, s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(bs->meta, bs->stage, meta, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(bs->stage, bs->res, std::min(meta, sizeof(szsel_result) * n), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) {
    msg = std::string("batch reserve: ") + hipGetErrorString(e);
    return SZSEL_EHIP;
  }
  return SZSEL_OK;
}

int batch_run(szsel_ctx *ctx, int ncu, BatchState *&bs, size_t budget, const szsel_request *reqs, int n,
              szsel_result *out, hipStream_t s, const BatchOptions &opt, std::string &msg) {
  if (n > kMaxBatch) {
    msg = "batch of " + std::to_string(n) + " requests; at most " + std::to_string(kMaxBatch);
    return SZSEL_EBUSY;
  }
  if (!bs && !batch_state_create(bs, msg)) return SZSEL_EHIP;
  hipError_t e = hipSuccess;
  // the host waits for the state's previous batch only where it rewrites
  // what that batch may still read (bind_plan, graph re-capture); on the
  // device, this batch follows the previous one also across streams
  if (bs->used && (e = hipStreamWaitEvent(s, bs->done, 0)) != hipSuccess) {
    msg = std::string("batch: ") + hipGetErrorString(e);
    return SZSEL_EHIP;
  }
  // knobs: the tuned ones for this batch shape (and launch mode: the
  // autotuner times a graph replay or the launches, as the batch will run),
  // else the defaults
  std::vector<uint64_t> key = shape_key(reqs, n);
  key.push_back(opt.graph ? 1u : 0u);
  Tune tu = opt.fixed;
  bool tuned = false;
  if (bs->have_last && bs->last_key == key && bs->last_auto == opt.autotune &&
      (opt.autotune || std::memcmp(&bs->last_tune, &opt.fixed, sizeof(Tune)) == 0)) {
    tu = bs->last_tune;
    tuned = true;
  } else if (opt.autotune) {
    Tuner &T = tuner();
    std::lock_guard<std::mutex> lock(T.mu);
    tune_cache_load(T);
    auto it = T.best.find(std::make_pair(std::string(ctx_arch(ctx)), key));
    if (it != T.best.end()) {
      tu = it->second;
      tuned = true;
    }
  }
  if (opt.autotune && !tuned) {
    // coordinate search over the knobs, each candidate timed once after
    // its plan is bound (results are identical for every candidate)
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
      msg = "autotune: event creation failed";
      return SZSEL_EHIP;
    }
    // a candidate the planner rejects (more work items than a pass holds,
    // more workspace than the budget) times as never faster; only a HIP
    // error ends the search
    // every candidate timed, for the final check of the closest ones
    std::vector<std::pair<float, Tune>> seen;
    // reps > 0: the best of reps runs; reps < 0: the median of -reps runs
    auto time_of = [&](const Tune &c, float &ms, int reps = 5) -> int {
      Plan p;
      ms = 1e30f;
      std::string why;
      if (make_plan(ctx, ncu, reqs, n, c, p, why) != SZSEL_OK) return SZSEL_OK;
      if (bind_plan(bs, p, budget, why) != hipSuccess) return SZSEL_OK;
      hipError_t q = upload_meta(bs, s);
      // timed the way the batch will run: a captured graph replayed when
      // graphs are on (launches on two streams overlap differently there
      // than when enqueued one by one), else the launches themselves
      hipGraph_t gr = nullptr;
      hipGraphExec_t ge = nullptr;
      if (q == hipSuccess && opt.graph) {
        q = hipStreamBeginCapture(bs->cap, hipStreamCaptureModeThreadLocal);
        if (q == hipSuccess) {
          const hipError_t q2 = enqueue_plan(bs, p, bs->cap);
          q = hipStreamEndCapture(bs->cap, &gr);
          if (q == hipSuccess) q = q2;
        }
        if (q == hipSuccess) q = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
      }
      auto once = [&]() { return ge ? hipGraphLaunch(ge, s) : enqueue_plan(bs, p, s); };
      if (q == hipSuccess) q = once();  // warm-up (first touch, code load)
      std::vector<float> runs;
      for (int rep = 0; rep < (reps > 0 ? reps : -reps) && q == hipSuccess; rep++) {
        float one = 0.f;
        q = hipEventRecord(t0, s);
        if (q == hipSuccess) q = once();
        if (q == hipSuccess) q = hipEventRecord(t1, s);
        if (q == hipSuccess) q = hipEventSynchronize(t1);
        if (q == hipSuccess) q = hipEventElapsedTime(&one, t0, t1);
        if (q == hipSuccess) runs.push_back(one);
      }
      if (!runs.empty()) {
        std::sort(runs.begin(), runs.end());
        ms = reps > 0 ? runs.front() : runs[runs.size() / 2];
        if (reps > 0) seen.emplace_back(ms, c);
      }
      if (ge || gr) {
        const hipError_t qs = hipStreamSynchronize(s);  // (the last replay is done unless a step failed)
        if (q == hipSuccess) q = qs;
        if (ge) (void)hipGraphExecDestroy(ge);
        if (gr) (void)hipGraphDestroy(gr);
      }
      if (q != hipSuccess) {
        msg = std::string("autotune: ") + hipGetErrorString(q);
        return SZSEL_EHIP;
      }
      return SZSEL_OK;
    };
    Tune cur = opt.fixed;
    float best_ms = 0.f;
    int rc = time_of(cur, best_ms);
    const int share_opts[] = {0, 1, 2, 3};
    const int group_opts[] = {1, 2, 4, 8};
    const int lane_opts[] = {1, 2, 3};
    const int sz_opts[] = {2, 4, 8, 16, 32, 64, 128};
    const int zfp_opts[] = {16, 32, 64, 128};  // ZFP waves per CU of a launch class
    const int range_opts[] = {1, 2, 4, 8, 16, 32, 64};  // quarters of the CU count
    const int grid_opts[] = {0, 1, 2, 4};
    const int ovf_opts[] = {kOvfPerSlice, 2 * kOvfPerSlice, 4 * kOvfPerSlice};
    // two sweeps of the coordinates: the best group count depends on how
    // fast the sampled passes became with the other knobs
    for (int sweep = 0; sweep < 2; sweep++) {
    const Tune before = cur;
    for (int v : share_opts) {
      if (rc != SZSEL_OK || v == cur.share) continue;
      Tune c = cur;
      c.share = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    for (int v : group_opts) {
      if (rc != SZSEL_OK || v == cur.groups || v > n) continue;
      Tune c = cur;
      c.groups = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    for (int v : lane_opts) {
      if (rc != SZSEL_OK || v == cur.lanes || cur.groups > 1) continue;
      Tune c = cur;
      c.lanes = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    for (int v : sz_opts) {
      if (rc != SZSEL_OK || v == cur.sz_wgs_q) continue;
      Tune c = cur;
      c.sz_wgs_q = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    for (int v : zfp_opts) {
      if (rc != SZSEL_OK || v == cur.zfp_waves) continue;
      Tune c = cur;
      c.zfp_waves = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    for (int v : range_opts) {
      if (rc != SZSEL_OK || v == cur.range_wgs_q) continue;
      Tune c = cur;
      c.range_wgs_q = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    for (int v : grid_opts) {
      if (rc != SZSEL_OK || v == cur.range_grid) continue;
      Tune c = cur;
      c.range_grid = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    for (int v : ovf_opts) {
      if (rc != SZSEL_OK || v == cur.ovf_slice) continue;
      Tune c = cur;
      c.ovf_slice = v;
      float ms = 0.f;
      rc = time_of(c, ms);
      if (rc == SZSEL_OK && ms < best_ms) {
        best_ms = ms;
        cur = c;
      }
    }
    if (std::memcmp(&before, &cur, sizeof(Tune)) == 0) break;  // nothing moved
    }
    // the closest candidates differ by little more than the noise of a
    // best of 5: the three fastest distinct ones are timed again, 15 runs
    // each, and the lowest median wins
    if (rc == SZSEL_OK && seen.size() > 1) {
      std::stable_sort(seen.begin(), seen.end(),
                       [](const std::pair<float, Tune> &a, const std::pair<float, Tune> &b) { return a.first < b.first; });
      std::vector<Tune> top;
      for (const auto &c : seen) {
        bool dup = false;
        for (const Tune &t : top) dup = dup || std::memcmp(&t, &c.second, sizeof(Tune)) == 0;
        if (!dup) top.push_back(c.second);
        if (top.size() == 3) break;
      }
      float best_med = 1e30f;
      for (const Tune &c : top) {
        float ms = 0.f;
        rc = time_of(c, ms, -15);
        if (rc != SZSEL_OK) break;
        if (ms < best_med) {
          best_med = ms;
          cur = c;
        }
      }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc != SZSEL_OK) return rc;
    if (best_ms < 1e30f) {  // (no schedule planned: the plan below reports why)
      Tuner &T = tuner();
      std::lock_guard<std::mutex> lock(T.mu);
      T.best[std::make_pair(std::string(ctx_arch(ctx)), key)] = cur;
      tune_cache_append(T, ctx_arch(ctx), key, cur);
    }
    tu = cur;
  }
  bs->last_key = key;
  bs->last_tune = tu;
  bs->last_auto = opt.autotune;
  bs->have_last = true;

  Plan p;
  int rc = make_plan(ctx, ncu, reqs, n, tu, p, msg);
  if (rc != SZSEL_OK) return rc;
  if (bind_plan(bs, p, budget, msg) != hipSuccess) return SZSEL_ENOMEM;
  if ((e = upload_meta(bs, s)) != hipSuccess) {
    msg = std::string("batch upload: ") + hipGetErrorString(e);
    return SZSEL_EHIP;
  }
  const size_t res_bytes = sizeof(szsel_result) * (size_t)n;
  bool copied = false;
  if (opt.graph && !opt.timer) {
    // the results' copy is part of the graph when `out` came back from one
    // of the last calls (a caller rotating a few result buffers) and the
    // device can reach it (pinned host or device memory): a copy queued
    // after a graph starts several microseconds after it ends, one inside it
    // right away.  Such graphs are kept per destination; a destination seen
    // once gets the graph without the copy, so fresh buffers every call do
    // not capture every call.
    const bool again = std::find(bs->outs.begin(), bs->outs.end(), (const void *)out) != bs->outs.end();
    if (!again) {
      if (bs->outs.size() >= (size_t)kGraphCache - 1) bs->outs.erase(bs->outs.begin());
      bs->outs.push_back(out);
    }
    hipPointerAttribute_t at;
    const bool reach = again && hipPointerGetAttributes(&at, out) == hipSuccess &&
                       (at.type == hipMemoryTypeHost || at.type == hipMemoryTypeDevice);
    if (again && !reach) (void)hipGetLastError();  // unregistered host memory: not an error here
    std::vector<uint64_t> key = p.sig;
    key.push_back(reach ? (uint64_t)(uintptr_t)out : 0u);
    key.push_back((uint64_t)n);
    BatchState::Graph *g = nullptr;
    for (BatchState::Graph &c : bs->graphs)
      if (c.key == key) g = &c;
    if (!g) {
      if (bs->graphs.size() >= (size_t)kGraphCache) {
        if ((e = batch_wait(bs)) != hipSuccess) {  // the graph replaced may still run
          msg = std::string("batch: ") + hipGetErrorString(e);
          return SZSEL_EHIP;
        }
        auto lru = std::min_element(bs->graphs.begin(), bs->graphs.end(),
                                    [](const BatchState::Graph &a, const BatchState::Graph &b) { return a.used < b.used; });
        if (lru->exec) (void)hipGraphExecDestroy(lru->exec);
        if (lru->graph) (void)hipGraphDestroy(lru->graph);
        bs->graphs.erase(lru);
      }
      BatchState::Graph c;
      e = hipStreamBeginCapture(bs->cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e2 = enqueue_plan(bs, p, bs->cap);
        if (e2 == hipSuccess && reach) e2 = hipMemcpyAsync(out, bs->res, res_bytes, hipMemcpyDefault, bs->cap);
        e = hipStreamEndCapture(bs->cap, &c.graph);
        if (e == hipSuccess) e = e2;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
        if (c.graph) (void)hipGraphDestroy(c.graph);
        msg = std::string("batch graph capture: ") + hipGetErrorString(e);
        return SZSEL_EHIP;
      }
      c.key = std::move(key);
      bs->graphs.push_back(std::move(c));
      g = &bs->graphs.back();
    }
    g->used = ++bs->clock;
    e = hipGraphLaunch(g->exec, s);
    copied = reach;
  } else {
    e = enqueue_plan(bs, p, s, opt.timer);
  }
  if (e == hipSuccess && !copied) e = hipMemcpyAsync(out, bs->res, res_bytes, hipMemcpyDefault, s);
  if (e == hipSuccess) e = hipEventRecord(bs->done, s);
  if (e != hipSuccess) {
    msg = std::string("batch launch: ") + hipGetErrorString(e);
    return SZSEL_EHIP;
  }
  bs->used = true;
  return SZSEL_OK;
}

}  // namespace szsel
