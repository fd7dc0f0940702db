#!/usr/bin/env python
"""Throughput of the SZ-vs-ZFP rate-distortion estimator and selector on one GPU.

Default run (the headline): the uneven 3-D mix -- 13 FP32 fields of
100x500x500, 6 FP64 fields of 256x384x384, 4 FP32 fields of 512^3 and 20 FP32
fields of 64^3 (5,280,394,496 bytes), spectral slopes U[-5, -2], relative
error bounds drawn from {1e-2 ... 1e-6}, block stride (5, 4, 1) -- estimated
with Algorithm 1 for every field:

* batched, autotuned: one szsel_select_batch per step (one launch per pass
  and request class, HIP graph replay, the launch shape and stream lanes
  chosen by the library's autotuner) -- this is `value`;
* batched with the fixed schedule, and plain (one szsel_select per field),
  with the speedups.

Metric: input GB/s = bytes of all fields / GPU time of one step (HIP events
on the stream the work runs on; inputs resident in HBM; the results' copy
to pinned host memory included).  `roofline`: the kernel with the largest
GPU time per step, timed by the library's per-launch HIP events over a
profiled run of the same steps, its algorithmic bytes against the 8 TB/s
HBM peak.  `passes`: every class of launch timed that way; the profiled
run issues the launches one at a time on one stream, so where the batch
runs them on two stream lanes their sum exceeds the batch's time.  `cpu_baseline`: the C oracle on the same fields, one host core
and a thread pool.  Extra keys: the 79-field 2-D batch, the 512^3 field's
five-bound sweep (plain and batched), and a shortened Poisson serving run
with p50/p99 latency.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --workload atm79 | mix3d | turb512 | serve | accuracy
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input GB/s through SZ+ZFP RD estimation+selection (batched vs plain); p99 latency"
HBM_PEAK_GBS = 8000.0
PHASES = ("range", "zfp", "sz", "ovf", "ent")
KERNELS = {"range": "kb_range (value range over all N values)",
           "zfp": "kb_zfp (ZFP transform, coder count and decode of the sampled blocks)",
           "sz": "kb_sz (Lorenzo prediction, quantization codes, LDS histogram)",
           "ovf": "kb_ovf (counts of codes outside the LDS window)",
           "ent": "kb_ent (entropy, bit-rates, selection)"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--latency-calls", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only (no 2-D batch, 512^3 sweep or serving run)")
    ap.add_argument("--n", type=int, default=512, help="edge of the cubic field of the turb512 sweep")
    ap.add_argument("--workload", default="mix3d",
                    choices=["mix3d", "atm79", "turb512", "serve", "accuracy"],
                    help="mix3d: 43 uneven 3-D fields, FP32 and FP64 (default, the headline); "
                         "atm79: 79 fields of 1800x3600; turb512: one 512^3 field, 5 bounds; "
                         "serve: a Poisson stream of snapshots through the serving engine; "
                         "accuracy: the selection against whole-field compression (Step 4)")
    ap.add_argument("--serve-rate", type=float, default=20.0,
                    help="snapshots per second (0: all at once, the engine's capacity)")
    ap.add_argument("--serve-snapshots", type=int, default=1000)
    ap.add_argument("--serve-oracle-snapshots", type=int, default=200,
                    help="snapshots whose served results are replayed through the oracle")
    ap.add_argument("--serve-pool-gib", type=float, default=64.0)
    ap.add_argument("--serve-lanes", type=int, default=4)
    ap.add_argument("--autotune", type=int, default=1, help="autotune the batched launch shape")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="bound on each CPU-baseline leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device 5 times (scales the HBM byte counters)")
    return ap.parse_args()


def pct(sorted_vals, q):
    return sorted_vals[min(len(sorted_vals) - 1, int(q * len(sorted_vals)))]


def covered(n, nb_stride):
    """Coordinates along one axis that the SZ pass reads: every sampled
    block's 4 points plus the Lorenzo predecessor at -1, inside [0, n)."""
    nb = n // 4
    cells = set()
    for j in range(0, nb, nb_stride):
        for c in range(4 * j - 1, 4 * j + 4):
            if 0 <= c < n:
                cells.add(c)
    return len(cells)


def request_bytes(shape, stride, itemsize):
    """Algorithmic bytes each pass must move for one request: the range pass
    reads every value once; the ZFP pass the sampled blocks' values; the SZ
    pass the sampled values and their Lorenzo predecessors (unique values of
    the sampled boxes extended by one cell toward the origin); the entropy
    pass the 65536-bin histogram."""
    n, nblk, halo = 1, 1, 1
    for d, s in zip(shape, stride):
        n *= d
        nblk *= (d // 4 + s - 1) // s
        halo *= covered(d, s)
    return {"range": n * itemsize, "zfp": nblk * 4 ** len(shape) * itemsize,
            "sz": halo * itemsize, "ent": 65536 * 4}


COPY_BYTES = 256 << 20


def copy_calibration(torch):
    """A plain copy of known size: each launch reads and writes COPY_BYTES."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "launches": 5}))


def source_digest(root=None):
    """Digest of the kernel sources and of the planning that sets their
    launch shapes, to tell whether recorded counters still describe the
    current kernels: their code with comments and whitespace removed, so
    that an edited comment keeps the counters."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in ("device.hpp", "estimator.hpp", "kernels.hip", "launch.hpp", "runtime.hip",
                 "batch.hip", "batch_kernels.hip"):
        with open(os.path.join(root or ROOT, "paper_1806_08901_amd", "csrc", name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def recorded_traffic(profile, kernel):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (profiles/<profile>), or None when it is missing or was taken from
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    digest, val = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("sources:"):
                digest = line.split()[1]
            if line.startswith("traffic:") and line.split()[1] == kernel:
                val = int(line.split()[2])
    return val if digest == source_digest() else None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pool_threads():
    """Threads of the CPU pool: the cores this process may use, at most 16
    (a one-GPU machine's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class StepTimer:
    """HIP events around each of K steps on one stream: the mean over the
    bracketed region (the contract's ms_per_step) and the median step."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def run(self, step, warmup, steps):
        torch = self.torch
        for k in range(warmup):
            step(k)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(self.stream)
        for k in range(steps):
            step(k)
            ev[k + 1].record(self.stream)
        torch.cuda.synchronize()
        per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
        return ev[0].elapsed_time(ev[steps]) / steps, statistics.median(per)


def pass_profile(ctx, szsel, run_steps, steps, byte_table):
    """Per (pass, dtype) GPU time per step from the library's launch events
    over `steps` profiled steps (each launch alone on one stream: the
    profile does not overlap them), with the algorithmic bytes of that class
    of launches per step (byte_table[(pass, dtype)]) and their rate."""
    ctx.profile_read_split()  # clear
    ctx.set_option(szsel.OPT_PROFILE, 1)
    run_steps(steps)
    prof = ctx.profile_read_split()
    ctx.set_option(szsel.OPT_PROFILE, 0)
    out = {}
    for (ph, dt), (ms, calls) in prof.items():
        if calls == 0:
            continue
        e = {"ms_per_step": round(ms / steps, 5), "launches_per_step": round(calls / steps, 3),
             "avg_launch_ms": round(ms / calls, 5)}
        b = byte_table.get((ph, dt))
        other = "f64" if dt == "f32" else "f32"
        if ph in ("range", "ovf", "ent") and prof.get((ph, other), (0.0, 0))[1] == 0 \
                and byte_table.get((ph, other)):
            # one launch per request group serves both dtypes; it is
            # recorded under its first request's
            b = (b or 0) + byte_table.get((ph, other), 0)
            e["dtypes"] = "binary32 and binary64"
        if b:
            gbs = b / (ms / steps * 1e-3) / 1e9
            e.update({"bytes_per_step": b, "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
        out["%s_%s" % (ph, dt)] = e
    return out


def roofline_of(passes, traffic_profile=None, kernel_names=None):
    """The class of launches with the most GPU time per step."""
    k = max((k for k in passes if "GB/s" in passes[k]), key=lambda q: passes[q]["ms_per_step"])
    e = passes[k]
    ph, dt = k.split("_")
    traffic = None
    if traffic_profile and kernel_names:
        traffic = recorded_traffic(traffic_profile, kernel_names.get(k, ""))
    per_launch = e["bytes_per_step"] / e["launches_per_step"]
    fields = e.get("dtypes", "binary32" if dt == "f32" else "binary64")
    return {"bound": "hbm", "kernel": "%s, %s fields" % (KERNELS[ph], fields),
            "achieved": e["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": e["frac"],
            "traffic": traffic, "bytes_per_launch": int(per_launch), "avg_launch_ms": e["avg_launch_ms"],
            "launches_per_step": e["launches_per_step"]}


def kernel_name(cls, nd=3, vec=True, ec=False):
    """Template name of a batched kernel as rocprofv3 prints it (spaces
    removed), for the launch class `cls` = "<pass>_<f32|f64>"."""
    ph, dt = cls.split("_")
    t = "float" if dt == "f32" else "double"
    v = "true" if vec else "false"
    if ph == "range":
        return "szsel::kb_range"
    if ph == "zfp":
        return "szsel::kb_zfp<%s,%d,%s,%s>" % (t, nd, v, "true" if ec else "false")
    if ph == "sz":
        return "szsel::kb_sz<%s,%d,%s>" % (t, nd, v)
    if ph == "ovf":
        return "szsel::kb_ovf"
    return "szsel::kb_ent"


def cpu_baseline(fields, items, gpu_results, seconds, label):
    """The C oracle on the same requests (szsel_select semantics): one host
    core over the fields in order until `seconds` have passed, then a
    thread pool over every field; both checked against the GPU results."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    from tests.gpu_common import assert_matches_oracle

    def one(i):
        f, eb, m, st, op = items[i]
        o, _ = oracle.run(op, hosts[i], eb, m, st)
        return o

    hosts = {}
    mism = 0
    s1 = 0.0  # oracle time of the single-core leg (host copies excluded)
    done = nb1 = 0
    for i in range(len(items)):
        hosts[i] = np.ascontiguousarray(fields[i].cpu().numpy())
        t0 = time.perf_counter()
        o = one(i)
        s1 += time.perf_counter() - t0
        done += 1
        nb1 += hosts[i].nbytes
        try:
            assert_matches_oracle(gpu_results[i], o)
        except AssertionError:
            mism += 1
        if s1 > seconds:
            break
    for i in range(len(items)):
        if i not in hosts:
            hosts[i] = np.ascontiguousarray(fields[i].cpu().numpy())
    T = pool_threads()
    t = time.perf_counter()
    with cf.ThreadPoolExecutor(T) as ex:
        outs = list(ex.map(one, range(len(items))))
    sT = time.perf_counter() - t
    nbT = sum(h.nbytes for h in hosts.values())
    for i, o in enumerate(outs):
        if i < done:
            continue
        try:
            assert_matches_oracle(gpu_results[i], o)
        except AssertionError:
            mism += 1
    return {
        "value": round(nbT / sT / 1e9, 4), "unit": "GB/s", "cores": T, "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": "%s: szsel_select semantics on all %d fields (%.2f GB), C oracle in a pool of %d "
                  "threads (one field per task), %.1f s" % (label, len(items), nbT / 1e9, T, sT),
        "single_core": {"value": round(nb1 / s1 / 1e9, 4), "unit": "GB/s", "cores": 1,
                        "sample": "the first %d fields in order (%.2f GB), %.1f s" % (done, nb1 / 1e9, s1)},
        "parity_with_oracle": mism == 0, "oracle_mismatches": mism, "requests_checked": len(items),
    }


def batch_workload(args, torch, synth, szsel, name, cpu=False, profile_file=None):
    """Many fields, one request each: plain per-field launches, one batch
    with the fixed schedule and one with the autotuned schedule."""
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    specs = synth.workload_atm_specs() if name == "atm79" else synth.workload_mix3d_specs()
    fields = [synth.make_field(sp, device=dev) for sp in specs]
    torch.cuda.synchronize()
    strides = [(20, 1) if f.dim() == 2 else (5, 4, 1) for f in fields]
    items = [(f, sp["eb"], szsel.EB_REL, st, szsel.OP_SELECT) for f, sp, st in zip(fields, specs, strides)]
    nbytes = sum(f.numel() * f.element_size() for f in fields)
    table = {}
    for f, st in zip(fields, strides):
        dt = "f32" if f.dtype == torch.float32 else "f64"
        for ph, b in request_bytes(tuple(f.shape), st, f.element_size()).items():
            table[(ph, dt)] = table.get((ph, dt), 0) + b
    ctx = szsel.Context(0)
    stream = torch.cuda.current_stream()
    timer = StepTimer(torch, stream)
    warm = max(args.warmup, 8)  # every workspace of the rotation captured once

    plain = [ctx.run(szsel.OP_SELECT, f, eb, m, st) for (f, eb, m, st, op) in items]
    ms_plain, med_plain = timer.run(
        lambda k: [ctx.run(szsel.OP_SELECT, f, eb, m, st, sync=False) for (f, eb, m, st, op) in items],
        args.warmup, args.steps)
    reqs = ctx.make_requests(items)
    outs = [ctx.result_buffer(len(items)) for _ in range(4)]
    res = {}
    for mode in ("fixed", "autotuned"):
        ctx.set_option(szsel.OPT_AUTOTUNE, 1 if mode == "autotuned" else 0)
        first = ctx.select_batch(None, reqs=reqs)
        mean, med = timer.run(lambda k: ctx.select_batch(None, reqs=reqs, sync=False, out=outs[k % 4]),
                              warm, args.steps)
        res[mode] = (mean, med, first == plain)

    def run_steps(n):
        for k in range(n):
            ctx.select_batch(None, reqs=reqs, sync=False, out=outs[k % 4])
        torch.cuda.synchronize()

    passes = pass_profile(ctx, szsel, run_steps, args.steps, table)
    names = {cls: kernel_name(cls, nd=fields[0].dim()) for cls in passes}
    roof = roofline_of(passes, profile_file, names)
    lat = []
    for _ in range(max(1, args.latency_calls)):
        t = time.perf_counter()
        ctx.select_batch(None, reqs=reqs)
        lat.append((time.perf_counter() - t) * 1e3)
    lat.sort()
    gbs = lambda ms: nbytes / (ms * 1e-3) / 1e9
    ms_auto = res["autotuned"][0]
    value = gbs(ms_auto)
    shapes = sorted({(tuple(f.shape), str(f.dtype).replace("torch.", "")) for f in fields})
    hbm = None
    if profile_file:
        tot = 0
        for cls, e in passes.items():
            b = recorded_traffic(profile_file, names[cls])
            if b is None:
                tot = None
                break
            tot += b * e["launches_per_step"]
        if tot:
            hbm = {"bytes_per_step": int(tot), "GB/s": round(tot / (ms_auto * 1e-3) / 1e9, 1),
                   "frac": round(tot / (ms_auto * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "what": "rocprofv3 FETCH_SIZE + WRITE_SIZE of every kernel of one step (scaled by a "
                           "copy of known size) / the step's GPU time"}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_auto, 4),
        "ms_per_step_median": round(res["autotuned"][1], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s_batched_autotuned" % name, "fields": len(fields), "input_bytes": nbytes,
                   "shapes": [[list(sh), dt] for sh, dt in shapes],
                   "stride": {"2d": [20, 1], "3d": [5, 4, 1]},
                   "mode": "one szsel_select_batch per step (Algorithm 1 for every field; one launch "
                           "per pass and request class, HIP graph replay, autotuned launch shape and "
                           "stream lanes)",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "passes": passes,
        "plain": {"value": round(gbs(ms_plain), 2), "ms_per_step": round(ms_plain, 4),
                  "ms_per_step_median": round(med_plain, 4), "mode": "one szsel_select per field"},
        "batched_fixed": {"value": round(gbs(res["fixed"][0]), 2), "ms_per_step": round(res["fixed"][0], 4),
                          "ms_per_step_median": round(res["fixed"][1], 4),
                          "results_equal_plain": bool(res["fixed"][2])},
        "batched_autotuned": {"value": round(value, 2), "frac_of_hbm_peak": round(value / HBM_PEAK_GBS, 4),
                              "results_equal_plain": bool(res["autotuned"][2])},
        "speedup_batched_vs_plain": round(ms_plain / ms_auto, 3),
        "speedup_autotuned_vs_fixed": round(res["fixed"][0] / ms_auto, 3),
        "latency_ms": {"p50": round(pct(lat, 0.5), 4), "p99": round(pct(lat, 0.99), 4),
                       "calls": len(lat), "what": "one synchronous batch (host wall clock)"},
        "hbm_traffic": hbm,
    }
    if cpu and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(fields, items, plain, args.cpu_seconds, name)
    ctx.close()
    del fields
    torch.cuda.empty_cache()
    return out


def turb512_workload(args, torch, synth, szsel):
    """The 512^3 field's five-bound sweep: plain szsel_select calls and the
    same five requests as one batch (which scans the field once)."""
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    field = synth.workload_turb512(device=dev, n=n)
    torch.cuda.synchronize()
    ebs = list(synth.EB_SWEEP)
    stride = (5, 4, 1)
    nbytes = field.numel() * field.element_size()
    ctx = szsel.Context(0)
    stream = torch.cuda.current_stream()
    timer = StepTimer(torch, stream)
    gpu_results = [ctx.select(field, eb, stride=stride) for eb in ebs]

    def step(k):
        for eb in ebs:
            ctx.run(szsel.OP_SELECT, field, eb, szsel.EB_REL, stride, sync=False)

    ms_step, med_step = timer.run(step, args.warmup, args.steps)
    value = len(ebs) * nbytes / (ms_step * 1e-3) / 1e9
    # per-pass GPU time of plain steps (events recorded by the library)
    ctx.set_option(szsel.OPT_PROFILE, 1)
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.set_option(szsel.OPT_PROFILE, 0)
    one = request_bytes((n, n, n), stride, field.element_size())
    passes = {}
    for k, (ms, calls) in prof.items():
        e = {"avg_launch_ms": round(ms / max(1, calls), 5)}
        if k in one:
            gbs = one[k] / (ms / max(1, calls) * 1e-3) / 1e9
            e.update({"bytes_per_launch": one[k], "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
        passes[k] = e
    dom = max((k for k in passes if "GB/s" in passes[k]), key=lambda q: passes[q]["avg_launch_ms"])
    items = [(field, eb, szsel.EB_REL, stride, szsel.OP_SELECT) for eb in ebs]
    reqs = ctx.make_requests(items)
    if args.autotune:
        ctx.set_option(szsel.OPT_AUTOTUNE, 1)
    batch_results = ctx.select_batch(items, reqs=reqs)
    bouts = [ctx.result_buffer(len(items)) for _ in range(4)]
    ms_batch, med_batch = timer.run(lambda k: ctx.select_batch(None, reqs=reqs, sync=False, out=bouts[k % 4]),
                                    max(args.warmup, 8), args.steps)
    value_batch = len(ebs) * nbytes / (ms_batch * 1e-3) / 1e9
    # HBM bytes one batch moves: the counters of its launches (one of each
    # pass) from the committed summary, while it matches the sources
    hbm_batch = None
    per = [recorded_traffic("hbm_traffic_turb512.md", kernel_name(c)) for c in
           ("range_f32", "zfp_f32", "sz_f32", "ovf_f32", "ent_f32")]
    if all(b is not None for b in per):
        gbs = sum(per) / (ms_batch * 1e-3) / 1e9
        hbm_batch = {"bytes_per_step": int(sum(per)), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "what": "rocprofv3 FETCH_SIZE + WRITE_SIZE of the batch's five launches (the field is read "
                             "once) / the batch's GPU time"}
    lat = []
    for k in range(args.latency_calls):
        t = time.perf_counter()
        ctx.select(field, ebs[k % len(ebs)], stride=stride)
        lat.append((time.perf_counter() - t) * 1e3)
    lat.sort()
    out = {
        "value": round(value, 2), "unit": "GB/s", "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(med_step, 4),
        "config": {"workload": "turb%d_sweep5_plain" % n, "shape": [n, n, n], "field_dtype": "f32",
                   "eb_rel": ebs, "stride": list(stride), "sampled_blocks": int(gpu_results[0]["zfp_blocks"]),
                   "requests_per_step": len(ebs), "mode": "plain per-field launches (szsel_select)"},
        "roofline_plain": {"bound": "hbm", "kernel": "k_" + dom, "achieved": passes[dom]["GB/s"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": passes[dom]["frac"],
                           "traffic": recorded_traffic("hbm_traffic_turb512.md", "k_" + dom),
                           "bytes_per_launch": passes[dom]["bytes_per_launch"],
                           "avg_launch_ms": passes[dom]["avg_launch_ms"]},
        "passes_plain": passes,
        "latency_ms": {"p50": round(pct(lat, 0.5), 4), "p99": round(pct(lat, 0.99), 4), "calls": len(lat),
                       "what": "one synchronous szsel_select on the field"},
        "batched": {
            "input_GBps": round(value_batch, 2), "ms_per_step": round(ms_batch, 4),
            "ms_per_step_median": round(med_batch, 4), "speedup_vs_plain": round(value_batch / value, 3),
            "results_equal_plain": batch_results == gpu_results,
            "hbm_traffic": hbm_batch,
            "what": "the 5 requests as one szsel_select_batch: the field is scanned once for all five, "
                    "so input GB/s (5 x 512 MiB per step) counts that scan's bytes five times; it is "
                    "not a fraction of the HBM peak"},
        "choices": [r["choice"] for r in gpu_results],
    }
    ctx.close()
    del field
    torch.cuda.empty_cache()
    return out


def accuracy(args, torch, synth, szsel):
    """Algorithm 1 against Step 4: for every field and bound, the estimator's
    choice against the compressor that really needs fewer bits (SZ at the
    bound the selection hands it, ZFP at eb_abs, both over the whole field),
    and the estimates' errors; also the compressors' throughput."""
    dev = torch.device("cuda:0")
    cases = [("turb512", synth.workload_turb512(device=dev), (5, 4, 1))]
    for k, sp in enumerate(synth.workload_atm_specs()[:10]):
        cases.append(("atm%d" % k, synth.make_field(sp, device=dev), (20, 1)))
    for k, sp in enumerate(synth.workload_mix3d_specs()[::7]):
        cases.append(("mix%d" % k, synth.make_field(sp, device=dev), (5, 4, 1)))
    torch.cuda.synchronize()
    ctx = szsel.Context(0)
    rows = []
    t_sz = t_zfp = 0.0
    nbytes_c = 0
    huff_ok = 0
    for name, f, st in cases:
        for eb in synth.EB_SWEEP:
            ctx.set_option(szsel.OPT_HUFFMAN, 2)
            est_h = ctx.select(f, eb, stride=st)
            ctx.set_option(szsel.OPT_HUFFMAN, 0)
            est = ctx.select(f, eb, stride=st)
            if est["flags"] & 0x13:  # constant / non-finite / no blocks: nothing to compare
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sz, _, _ = ctx.sz_compress(f, est["sz_eb"], decoded=False)
            t1 = time.perf_counter()
            zf, _, _ = ctx.zfp_compress(f, est["eb_abs"], decoded=False)
            t2 = time.perf_counter()
            t_sz += t1 - t0
            t_zfp += t2 - t1
            nbytes_c += f.numel() * f.element_size()
            truth = 0 if sz["bitrate"] < zf["bitrate"] else 1
            huff_ok += 1 if est_h["choice"] == truth else 0
            chosen = sz["bitrate"] if est["choice"] == 0 else zf["bitrate"]
            best = min(sz["bitrate"], zf["bitrate"])
            rows.append({
                "field": name, "eb_rel": eb, "choice": est["choice"], "best": truth,
                "br_sz": [round(est["sz_bitrate"], 4), round(sz["bitrate"], 4)],
                "br_zfp": [round(est["zfp_bitrate"], 4), round(zf["bitrate"], 4)],
                "psnr_sz": [round(est["sz_psnr_model"], 3), round(sz["psnr"], 3)],
                "psnr_zfp": [round(est["zfp_psnr"], 3), round(zf["psnr"], 3)],
                "loss_pct": round(100.0 * (chosen / best - 1.0), 3) if best > 0 else 0.0,
            })
    ok = sum(1 for r in rows if r["choice"] == r["best"])

    def rel(a):
        return abs(a[0] - a[1]) / a[1] if a[1] else 0.0

    out = {
        "metric": "selection accuracy of Algorithm 1 against Step 4 (whole-field compression)",
        "value": round(ok / max(1, len(rows)), 4), "unit": "fraction", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic", "dtype": "f64",
        "config": {"workload": "accuracy: turb512, 10 atm fields, 7 mix3d fields x 5 bounds",
                   "cases": len(rows)},
        "mean_bitrate_loss_pct": round(sum(r["loss_pct"] for r in rows) / max(1, len(rows)), 4),
        "accuracy_selecting_with_huffman_cost": round(huff_ok / max(1, len(rows)), 4),
        "estimate_error": {
            "br_sz_mean_rel": round(sum(rel(r["br_sz"]) for r in rows) / max(1, len(rows)), 4),
            "br_zfp_mean_rel": round(sum(rel(r["br_zfp"]) for r in rows) / max(1, len(rows)), 4),
            "psnr_sz_mean_abs_db": round(sum(abs(r["psnr_sz"][0] - r["psnr_sz"][1]) for r in rows) / max(1, len(rows)), 4),
            "psnr_zfp_mean_abs_db": round(sum(abs(r["psnr_zfp"][0] - r["psnr_zfp"][1]) for r in rows) / max(1, len(rows)), 4),
        },
        "compress_GBps": {"sz": round(nbytes_c / t_sz / 1e9, 2), "zfp": round(nbytes_c / t_zfp / 1e9, 2),
                          "what": "host wall clock around each synchronous call, whole fields"},
        "rows": rows,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def serve_workload(args, torch, synth, szsel, snapshots, rate, oracle_snapshots, oracle_seconds=None):
    """Poisson arrivals of snapshots (5-40 fields each, shapes 64^3, 512^3
    and 1800x3600 FP32, eb_rel uniform in [1e-6, 1e-2]) through the serving
    engine.  At its arrival time a snapshot asks for pool room (admission by
    HBM footprint; it waits in arrival order while the pool is full), the
    producer copies its fields into the reservation on its own stream, and
    the snapshot is submitted.  Latency: arrival to results on the host.
    The first `oracle_snapshots` snapshots' served results are then replayed
    through the C oracle (a thread pool; bounded by `oracle_seconds` when
    given) and compared field by field."""
    import random
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shapes = [(64, 64, 64), (512, 512, 512), (1800, 3600)]
    strides = {3: (5, 4, 1), 2: (20, 1)}
    src = {sh: [synth.spectral(sh, slope=-5.0 / 3.0 if len(sh) == 3 else -2.5, kmax=min(64.0, min(sh) / 2.0),
                               seed=5000 + 10 * i + k, device=dev) for k in range(3)]
           for i, sh in enumerate(shapes)}
    torch.cuda.synchronize()
    rng = random.Random(5000)
    snaps, t = [], 0.0
    for i in range(snapshots):
        t += rng.expovariate(rate) if rate > 0 else 0.0
        fl = []
        for _ in range(rng.randint(5, 40)):
            sh = shapes[rng.randrange(3)]
            fl.append((sh, rng.randrange(3), rng.uniform(1e-6, 1e-2)))
        snaps.append((t, fl))
    ctx = szsel.Context(0)
    pool = torch.empty(int(args.serve_pool_gib * (1 << 30)), dtype=torch.uint8, device=dev)
    srv = szsel.Server(ctx, pool, lanes=args.serve_lanes)
    prod = torch.cuda.Stream()
    rnd = lambda nb: (nb + 255) // 256 * 256

    def put(fl, got):
        """Copies the snapshot's fields into its reservation (producer
        stream) and submits it."""
        off, tk = got
        items = []
        with torch.cuda.stream(prod):
            for sh, k, eb in fl:
                f = src[sh][k]
                nb = f.numel() * 4
                v = pool[off:off + nb].view(torch.float32).view(sh)
                v.copy_(f)
                off += rnd(nb)
                items.append((v, eb, szsel.EB_REL, strides[len(sh)], szsel.OP_SELECT))
        srv.submit(tk, items, stream=prod)
        return tk

    # warm-up, untimed like the other workloads' warm-up steps: a burst of
    # two snapshots per lane submitted at once, so that the producer and
    # every lane have run, also concurrently, before the measured stream
    # (the runtime sets up queues at their first use: milliseconds)
    warm = []
    for _, fl in snaps[:2 * args.serve_lanes]:
        got = srv.reserve(sum(rnd(src[sh][k].numel() * 4) for sh, k, _ in fl))
        if got is None:
            break
        warm.append(put(fl, got))
    n_warm = len(warm)
    while warm:
        srv.progress(wait=True)
        warm = [tk for tk in warm if srv.status(tk) is None]
    torch.cuda.synchronize()
    st0 = srv.stats()
    waiting, inflight, lat, done_bytes = [], {}, [], 0
    waits, wait_ms, nxt, sample, reported = 0, 0.0, 0, [], 0
    served = {}
    t0 = time.perf_counter()
    t_first, t_last = None, None
    while len(lat) < len(snaps):
        now = time.perf_counter() - t0
        while nxt < len(snaps) and snaps[nxt][0] <= now:
            waiting.append(nxt)
            nxt += 1
        while waiting:  # admission in arrival order
            i = waiting[0]
            fl = snaps[i][1]
            need = sum(rnd(src[sh][k].numel() * 4) for sh, k, _ in fl)
            got = srv.reserve(need)
            if got is None:
                break
            waiting.pop(0)
            tw = time.perf_counter() - t0 - snaps[i][0]
            if tw > 1e-3:
                waits += 1
                wait_ms += tw * 1e3
            tk = put(fl, got)
            inflight[tk] = (i, need, [(src[sh][k], eb, szsel.EB_REL, strides[len(sh)], szsel.OP_SELECT)
                                      for sh, k, eb in fl])
            if t_first is None:
                t_first = snaps[i][0]
        srv.progress(wait=False)
        for tk in list(inflight):
            r = srv.status(tk)
            if r is None:
                continue
            i, need, orig = inflight.pop(tk)
            tdone = time.perf_counter() - t0
            lat.append((tdone - snaps[i][0]) * 1e3)
            done_bytes += sum(f.numel() * 4 for f, *_ in orig)
            t_last = tdone
            if i < oracle_snapshots:
                served[i] = r[0]
            if len(sample) < 3 and len(orig) <= 12:
                sample.append((orig, r[0]))
        if not inflight and not waiting and nxt < len(snaps):
            time.sleep(max(0.0, min(0.002, snaps[nxt][0] - (time.perf_counter() - t0))))
        if len(lat) // 200 > reported:
            reported = len(lat) // 200
            print("served %d of %d snapshots, %.1f s" % (len(lat), len(snaps), time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    st = srv.stats()
    same = all([ctx.run(op, f, eb, m, stv) for (f, eb, m, stv, op) in orig] == res for orig, res in sample)
    srv.close()
    del pool
    lat.sort()
    span = t_last - t_first
    value = done_bytes / span / 1e9
    out = {
        "value": round(value, 2), "unit": "GB/s",
        "config": {"workload": "serve_poisson%g" % rate if rate > 0 else "serve_saturated",
                   "snapshots": len(snaps), "fields_per_snapshot": [5, 40],
                   "shapes": [list(sh) for sh in shapes], "eb_rel": [1e-6, 1e-2],
                   "pool_gib": args.serve_pool_gib, "lanes": args.serve_lanes,
                   "mode": "szsel_server: HBM-pool admission, continuous batching over lanes"},
        "latency_ms": {"p50": round(pct(lat, 0.5), 3), "p99": round(pct(lat, 0.99), 3),
                       "max": round(lat[-1], 3), "what": "snapshot arrival to its results on the host, "
                                                          "including admission wait and the producer's copy-in"},
        "sustained": {"input_bytes": done_bytes, "seconds": round(span, 3),
                      "what": "input bytes of completed snapshots / time from first arrival to last completion"},
        "engine": {"batches": st["batches"] - st0["batches"],
                   "requests": st["batched_requests"] - st0["batched_requests"],
                   "requests_per_batch": round((st["batched_requests"] - st0["batched_requests"]) /
                                               max(1, st["batches"] - st0["batches"]), 2),
                   "warmup_snapshots": n_warm,
                   "admission_waits": waits, "admission_wait_ms_total": round(wait_ms, 2)},
        "results_equal_alone": bool(same),
    }
    if oracle_snapshots > 0 and not args.no_cpu_baseline:
        out["oracle_replay"] = serve_oracle_replay(snaps, served, src, strides, oracle_seconds)
    ctx.close()
    del src
    torch.cuda.empty_cache()
    return out


def serve_oracle_replay(snaps, served, src, strides, seconds):
    """Every request of the replayed snapshots through the C oracle (thread
    pool, one request per task), compared with what the server returned."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    from tests.gpu_common import assert_matches_oracle

    hosts = {key: [np.ascontiguousarray(f.cpu().numpy()) for f in fl] for key, fl in src.items()}
    todo = []
    for i in sorted(served):
        for j, (sh, k, eb) in enumerate(snaps[i][1]):
            todo.append((i, j, sh, k, eb))
    T = pool_threads()
    t = time.perf_counter()
    deadline = None if seconds is None else t + seconds

    def one(q):
        i, j, sh, k, eb = q
        if deadline is not None and time.perf_counter() > deadline:
            return None
        o, _ = oracle.run(oracle.OP_SELECT, hosts[sh][k], eb, oracle.EB_REL, strides[len(sh)])
        return o

    with cf.ThreadPoolExecutor(T) as ex:
        outs = list(ex.map(one, todo))
    secs = time.perf_counter() - t
    checked, mism, snaps_full = 0, 0, set()
    complete = {}
    for (i, j, sh, k, eb), o in zip(todo, outs):
        complete.setdefault(i, True)
        if o is None:
            complete[i] = False
            continue
        checked += 1
        try:
            assert_matches_oracle(served[i][j], o)
        except AssertionError:
            mism += 1
    snaps_full = sum(1 for v in complete.values() if v)
    return {"parity_with_oracle": mism == 0 and checked > 0, "requests_checked": checked,
            "oracle_mismatches": mism, "snapshots_replayed_whole": snaps_full,
            "seconds": round(secs, 1), "threads": T,
            "what": "served results of the first snapshots against the C oracle on the same fields and "
                    "bounds, bit-exact keys exact, log-derived keys to 1e-9 relative"}


def contract_line(args, part, workload_dtype="f64"):
    """The one JSON line's fixed keys around a workload's figures."""
    out = {"metric": METRIC, "value": part["value"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": part.get("ms_per_step"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": workload_dtype, "data": "synthetic"}
    for k, v in part.items():
        if k not in out:
            out[k] = v
    return out


def brief(part):
    """The figures of an extra workload kept in the headline line."""
    keep = ("value", "ms_per_step", "ms_per_step_median", "config", "roofline", "plain", "batched_fixed",
            "batched_autotuned", "speedup_batched_vs_plain", "speedup_autotuned_vs_fixed", "latency_ms",
            "hbm_traffic")
    return {k: part[k] for k in keep if k in part}


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(fields would shard across GPUs by whole fields, with no exchange)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return

    from paper_1806_08901_amd import synth, szsel

    if args.workload == "accuracy":
        accuracy(args, torch, synth, szsel)
        return
    if args.workload == "serve":
        part = serve_workload(args, torch, synth, szsel, args.serve_snapshots, args.serve_rate,
                              args.serve_oracle_snapshots)
        part["ms_per_step"] = round(part["sustained"]["seconds"] * 1e3 / args.serve_snapshots, 4)
        out = contract_line(args, part)
        out["steps"], out["warmup"] = args.serve_snapshots, 0
        print(json.dumps(out), flush=True)
        return
    if args.workload == "turb512":
        part = turb512_workload(args, torch, synth, szsel)
        print(json.dumps(contract_line(args, part)), flush=True)
        return
    if args.workload == "atm79":
        part = batch_workload(args, torch, synth, szsel, "atm79", cpu=True, profile_file="hbm_traffic_atm79.md")
        print(json.dumps(contract_line(args, part)), flush=True)
        return
    progress("mix3d: 43 fields, plain / fixed / autotuned batches")
    head = batch_workload(args, torch, synth, szsel, "mix3d", cpu=True, profile_file="hbm_traffic_mix3d.md")
    out = contract_line(args, head)
    if not args.no_extras:
        progress("atm79: 79 fields of 1800x3600")
        out["atm79"] = brief(batch_workload(args, torch, synth, szsel, "atm79"))
        progress("turb512: five-bound sweep")
        out["turb512"] = turb512_workload(args, torch, synth, szsel)
        progress("serve: 200 snapshots, Poisson 20/s")
        out["serve"] = serve_workload(args, torch, synth, szsel, 200, 20.0, 200,
                                      oracle_seconds=args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
