"""Batched execution (szsel_select_batch) against single requests and the oracle (needs a GPU).

A batch runs one launch per pass over all of its requests, shares the
value-range scan of requests on the same field, replays a captured HIP graph
while the batch shape repeats and may autotune its launch shape; none of this
may change a single bit of any result.
"""
import sys

import pytest
import torch

import oracle
from paper_1806_08901_amd import synth
from tests.gpu_common import assert_matches_oracle

pytestmark = pytest.mark.gpu

OPS = [oracle.OP_SZ, oracle.OP_ZFP, oracle.OP_SELECT, oracle.OP_FIXED_EB]


def _note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1806_08901_amd import szsel
    c = szsel.Context(0)
    yield c
    c.close()


def _fields():
    base = synth.spectral((70, 90), slope=-2.0, seed=61).cuda()
    return [
        synth.spectral((40, 36, 44), seed=62).cuda(),
        synth.spectral((33, 50, 47), slope=-3.0, seed=63, dtype=torch.float64).cuda(),
        synth.spectral((60, 90), slope=-1.5, seed=64, dtype=torch.float64).cuda(),
        base,
        base.view(-1)[1:1 + 69 * 90].view(69, 90),  # 4-byte offset: rows not 16-byte aligned
        synth.gaussian_bumps((1030,), sigma_range=(3.0, 30.0), seed=65).cuda(),
        synth.spiky_constant((48, 64), frac=0.01, seed=66).cuda(),
        torch.full((16, 20), 3.0, device="cuda"),  # constant field
        synth.gaussian_bumps((24, 24, 24), seed=67).cuda(),
    ]


def _items(fields, ebs=(1e-2, 1e-4, 1e-6)):
    items = []
    for i, f in enumerate(fields):
        for j, eb in enumerate(ebs):
            st = (2,) + (1,) * (f.dim() - 1) if (i + j) % 3 == 0 else (1,) * f.dim()
            items.append((f, eb, oracle.EB_REL, st, OPS[(i + j) % 4]))
    return items


def _singles(ctx, items):
    return [ctx.run(op, f, eb, mode, st) for (f, eb, mode, st, op) in items]


def test_mixed_batch_equals_single_calls(ctx):
    items = _items(_fields())
    _note("mixed batch of", len(items))
    batch = ctx.select_batch(items)
    for k, (b, s) in enumerate(zip(batch, _singles(ctx, items))):
        assert b == s, "request %d" % k


def test_batch_matches_oracle(ctx):
    f3 = synth.spectral((28, 24, 36), slope=-2.0, seed=68)
    f2 = synth.spectral((50, 66), slope=-2.5, seed=69, dtype=torch.float64)
    items = [(f3.cuda(), 1e-3, oracle.EB_REL, (1, 1, 1), oracle.OP_SELECT),
             (f2.cuda(), 1e-5, oracle.EB_REL, (2, 1), oracle.OP_SELECT),
             (f3.cuda(), 2e-3, oracle.EB_ABS, (1, 2, 1), oracle.OP_FIXED_EB)]
    batch = ctx.select_batch(items)
    for (f, eb, mode, st, op), g, host in zip(items, batch, [f3, f2, f3]):
        orc, _ = oracle.run(op, host.numpy(), eb, mode, st)
        assert_matches_oracle(g, orc, "batch op %d eb %g" % (op, eb))


def test_shared_range_scan_sweep(ctx):
    """Five bounds on one field: one range scan serves all five."""
    f = synth.spectral((64, 64, 64), slope=-5.0 / 3.0, seed=70).cuda()
    items = [(f, eb, oracle.EB_REL, (2, 2, 1), oracle.OP_SELECT) for eb in synth.EB_SWEEP]
    batch = ctx.select_batch(items)
    assert batch == _singles(ctx, items)


def test_graph_replays_follow_new_inputs(ctx):
    """Same batch shape three times: the captured graph is replayed with new
    bounds, new field contents and new field pointers, with eager work and
    synchronisations in between; every replay must equal the single calls."""
    fields = [synth.spectral((40, 36, 44), seed=71).cuda(), synth.spectral((60, 90), seed=72).cuda()]
    for rep in range(3):
        if rep == 1:
            fields[0].mul_(1.5).add_(0.25)  # same pointer, new contents
        if rep == 2:
            fields = [f.clone() for f in fields]  # new pointers, same shapes
        ebs = [(1e-2, 1e-4), (1e-3, 1e-5), (1e-4, 1e-6)][rep]
        items = [(f, eb, oracle.EB_REL, (1,) * f.dim(), oracle.OP_SELECT) for f in fields for eb in ebs]
        batch = ctx.select_batch(items)
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work
        assert batch == _singles(ctx, items), "replay %d" % rep


def test_autotune_and_no_graph_give_the_same_results(ctx):
    from paper_1806_08901_amd import szsel
    items = _items(_fields()[:4], ebs=(1e-3, 1e-5))
    ref = ctx.select_batch(items)
    try:
        ctx.set_option(szsel.OPT_AUTOTUNE, 1)
        tuned = ctx.select_batch(items)
        again = ctx.select_batch(items)
        ctx.set_option(szsel.OPT_BATCH_GRAPH, 0)
        eager = ctx.select_batch(items)
    finally:
        ctx.set_option(szsel.OPT_AUTOTUNE, 0)
        ctx.set_option(szsel.OPT_BATCH_GRAPH, 1)
    assert tuned == ref
    assert again == ref
    assert eager == ref


def test_request_group_schedules_equal_single_calls(ctx):
    """Fixed schedules with 2, 4 and 8 request groups (scans on a side
    stream, captured graphs replayed, and uncaptured), with the default
    range grid and with resident range workgroups (1 and 2 per CU), give
    the single calls' results."""
    from paper_1806_08901_amd import szsel
    items = _items(_fields(), ebs=(1e-3, 1e-5))
    singles = _singles(ctx, items)
    try:
        for grid in (0, 1, 2):
            ctx.set_option(szsel.OPT_RANGE_GRID, grid)
            for g in (1, 2, 4, 8):
                ctx.set_option(szsel.OPT_BATCH_GROUPS, g)
                for graph in (1, 0):
                    ctx.set_option(szsel.OPT_BATCH_GRAPH, graph)
                    for rep in range(2):
                        assert ctx.select_batch(items) == singles, "grid %d groups %d graph %d rep %d" % (
                            grid, g, graph, rep)
        with pytest.raises(szsel.SzselError):
            ctx.set_option(szsel.OPT_RANGE_GRID, 65)
    finally:
        ctx.set_option(szsel.OPT_BATCH_GROUPS, 0)
        ctx.set_option(szsel.OPT_RANGE_GRID, 0)
        ctx.set_option(szsel.OPT_BATCH_GRAPH, 1)


def test_stream_lanes_equal_single_calls(ctx):
    """One stream and two lanes (the passes after the scans of alternate
    launch classes, or of the two halves of the sampled work, on a side
    stream), with each share mode's launch shapes, captured graphs replayed
    three times with a single call between replays, and uncaptured: the
    single calls' results every time; a lane setting outside 0..3 is
    rejected."""
    from paper_1806_08901_amd import szsel
    items = _items(_fields(), ebs=(1e-3, 1e-5))
    singles = _singles(ctx, items)
    f, eb, mode, st, op = items[0]
    try:
        for share in (0, 3):
            ctx.set_option(szsel.OPT_BATCH_SHARE, share)
            for lanes in (2, 3, 1):
                ctx.set_option(szsel.OPT_BATCH_LANES, lanes)
                for graph in (1, 0):
                    ctx.set_option(szsel.OPT_BATCH_GRAPH, graph)
                    for rep in range(3):
                        _note("lanes", lanes, "share", share, "graph", graph, "rep", rep)
                        assert ctx.select_batch(items) == singles, "lanes %d share %d graph %d rep %d" % (
                            lanes, share, graph, rep)
                        assert ctx.run(op, f, eb, mode, st) == singles[0]
        with pytest.raises(szsel.SzselError):
            ctx.set_option(szsel.OPT_BATCH_LANES, 4)
    finally:
        ctx.set_option(szsel.OPT_BATCH_LANES, 0)
        ctx.set_option(szsel.OPT_BATCH_SHARE, 0)
        ctx.set_option(szsel.OPT_BATCH_GRAPH, 1)


@pytest.mark.parametrize("option,value", [("OPT_HUFFMAN", 1), ("OPT_EC_SAMPLING", 1)])
def test_stream_lanes_with_huffman_and_point_sampling(ctx, option, value):
    """Two lanes with the exact Huffman pass (one launch per class and lane
    after the entropy pass) and with point sub-sampling (the sub-sampling
    ZFP kernels): the single calls' results under the same option, for both
    lane settings, replayed twice."""
    from paper_1806_08901_amd import szsel
    opt = getattr(szsel, option)
    items = _items(_fields(), ebs=(1e-3, 1e-5))
    try:
        ctx.set_option(opt, value)
        singles = _singles(ctx, items)
        for lanes in (2, 3):
            ctx.set_option(szsel.OPT_BATCH_LANES, lanes)
            for rep in range(2):
                _note(option, "lanes", lanes, "rep", rep)
                assert ctx.select_batch(items) == singles, "%s lanes %d rep %d" % (option, lanes, rep)
    finally:
        ctx.set_option(opt, 0)
        ctx.set_option(szsel.OPT_BATCH_LANES, 0)


def test_rotating_result_buffers(ctx):
    """Three result buffers used in turn over seven calls with no host
    synchronisation (from the second round on, each destination's graph
    holds the results' copy), the field changed on the stream before every
    call: each call's buffer holds that call's results."""
    from paper_1806_08901_amd.szsel import _as_dict
    f = synth.spectral((48, 40, 36), seed=76).cuda()
    items_of = lambda a: [(a, eb, oracle.EB_REL, (1, 2, 1), oracle.OP_SELECT) for eb in (1e-2, 1e-4, 1e-6)]
    items = items_of(f)
    reqs = ctx.make_requests(items)
    bufs = [ctx.result_buffer(len(items)) for _ in range(3)]
    snaps, got = [], []
    for k in range(7):
        f.mul_(0.75).add_(0.05 * k)
        snaps.append(f.clone())
        ctx.select_batch(None, reqs=reqs, sync=False, out=bufs[k % 3])
        if k % 3 == 2 or k == 6:  # read the round's buffers once the stream is there
            torch.cuda.synchronize()
            for j in range(k - k % 3, k + 1):
                got.append([_as_dict(bufs[j % 3][i]) for i in range(len(items))])
    for k in range(7):
        assert got[k] == _singles(ctx, items_of(snaps[k])), "call %d" % k


def test_workgroup_share_modes_equal_single_calls(ctx):
    """Fixed schedules that deal the SZ count, or the SZ and range counts,
    over the batch or within each launch class give the single calls'
    results; a mode outside 0..3 is rejected."""
    from paper_1806_08901_amd import szsel
    items = _items(_fields(), ebs=(1e-3, 1e-5))
    singles = _singles(ctx, items)
    try:
        for mode in (1, 2, 3, 0):
            ctx.set_option(szsel.OPT_BATCH_SHARE, mode)
            for groups in (1, 2):
                ctx.set_option(szsel.OPT_BATCH_GROUPS, groups)
                assert ctx.select_batch(items) == singles, "share %d groups %d" % (mode, groups)
        with pytest.raises(szsel.SzselError):
            ctx.set_option(szsel.OPT_BATCH_SHARE, 4)
    finally:
        ctx.set_option(szsel.OPT_BATCH_SHARE, 0)
        ctx.set_option(szsel.OPT_BATCH_GROUPS, 0)


def test_launch_shapes_equal_default(ctx):
    """Single calls and batches under other launch shapes (ZFP chunks from
    one 16-block round per wave to 1,024 blocks, SZ workgroups from a
    quarter of the CU count to 64 per CU, range chunks from a quarter to 8
    per CU) give the default schedule's results, 3-D fields large enough
    for several levels of completion counters included; ZFP chunks that are
    not a power of two from 16 to 65536 are rejected."""
    from paper_1806_08901_amd import szsel
    big = [synth.spectral((96, 96, 100), slope=-3.0, seed=161).cuda(),
           synth.spectral((64, 72, 64), slope=-2.0, seed=162, dtype=torch.float64).cuda()]
    items = _items(_fields() + big, ebs=(1e-3, 1e-6))
    singles = _singles(ctx, items)
    try:
        for zc, sw, rw in ((16, 1, 0.25), (32, 256, 8), (1024, 3, 2)):
            _note("launch shape zfp_chunk", zc, "sz_wgs_q", sw, "range_wgs", rw)
            ctx.set_option(szsel.OPT_ZFP_CHUNK, zc)
            ctx.set_option(szsel.OPT_SZ_WGS, sw)
            ctx.set_option(szsel.OPT_RANGE_WGS, rw)
            assert _singles(ctx, items) == singles, "single calls, zfp chunk %d" % zc
            assert ctx.select_batch(items) == singles, "batch, zfp chunk %d" % zc
        for bad in (8, 48, 131072):
            with pytest.raises(szsel.SzselError):
                ctx.set_option(szsel.OPT_ZFP_CHUNK, bad)
    finally:
        for opt in (szsel.OPT_ZFP_CHUNK, szsel.OPT_SZ_WGS, szsel.OPT_RANGE_WGS):
            ctx.set_option(opt, 0)


def test_batches_in_flight_on_two_streams(ctx):
    a_items = _items(_fields()[:3], ebs=(1e-3,))
    b_items = _items(_fields()[3:6], ebs=(1e-4,))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    oa = ctx.select_batch(a_items, stream=s1, sync=False)
    ob = ctx.select_batch(b_items, stream=s2, sync=False)
    s1.synchronize()
    s2.synchronize()
    from paper_1806_08901_amd.szsel import _as_dict
    ra = [_as_dict(oa[i]) for i in range(len(a_items))]
    rb = [_as_dict(ob[i]) for i in range(len(b_items))]
    assert ra == _singles(ctx, a_items)
    assert rb == _singles(ctx, b_items)


def test_unchanged_batches_queue_without_waiting(ctx):
    """The same batch queued four times with no host synchronisation (an
    unchanged plan makes the host wait for nothing), with stream-ordered
    changes of a field in between: every call sees the field as the stream
    leaves it and fills its own result buffer."""
    from paper_1806_08901_amd.szsel import _as_dict
    f = synth.spectral((64, 80), seed=74).cuda()
    g = synth.spectral((24, 28, 32), slope=-3.0, seed=75).cuda()
    def items_of(a, b):
        return [(a, 1e-3, oracle.EB_REL, (1, 1), oracle.OP_SELECT),
                (b, 1e-4, oracle.EB_REL, (2, 1, 1), oracle.OP_SELECT),
                (a, 1e-5, oracle.EB_REL, (1, 1), oracle.OP_FIXED_EB)]
    items = items_of(f, g)
    ctx.select_batch(items)  # plan and capture
    outs, snaps = [], []
    for k in range(4):
        f.mul_(1.25).add_(0.1 * k)
        snaps.append((f.clone(), g.clone()))
        outs.append(ctx.select_batch(items, sync=False))
    torch.cuda.synchronize()
    for k in range(4):
        got = [_as_dict(outs[k][i]) for i in range(len(items))]
        assert got == _singles(ctx, items_of(*snaps[k])), "call %d" % k


def test_batch_argument_errors(ctx):
    from paper_1806_08901_amd import szsel
    f = synth.spectral((20, 20), seed=73).cuda()
    bad = [(f, 1e-3, oracle.EB_REL, (1, 1), oracle.OP_SELECT), (f, -1.0, oracle.EB_REL, (1, 1), oracle.OP_SELECT)]
    with pytest.raises(szsel.SzselError, match="request 1"):
        ctx.select_batch(bad)
    too_many = [(f, 1e-3, oracle.EB_REL, (1, 1), oracle.OP_SELECT)] * 1025
    with pytest.raises(szsel.SzselError, match="1024"):
        ctx.select_batch(too_many)
    # the context still works afterwards
    good = [(f, 1e-3, oracle.EB_REL, (1, 1), oracle.OP_SELECT)]
    assert ctx.select_batch(good) == _singles(ctx, good)
