"""Serving engine on the GPU: snapshots in flight together give the same
results, bit for bit, as each request alone and as the CPU oracle; admission
waits for pool room; the estimation waits for the producer's writes;
invalid snapshots are refused at submission without disturbing the others;
lane batches respect the lane budget; failed batches are retried in halves
and a request that cannot run completes flagged."""
import os
import sys

import pytest
import torch

import oracle
from paper_1806_08901_amd import synth
from tests.gpu_common import assert_matches_oracle

pytestmark = pytest.mark.gpu


def _note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1806_08901_amd import szsel
    c = szsel.Context(0)
    yield c
    c.close()


def _place(pool, off, src):
    """Copies src into the pool at byte offset off; returns the view."""
    nb = src.numel() * src.element_size()
    view = pool[off:off + nb].view(src.dtype).view(src.shape)
    view.copy_(src)
    return view


def _snapshot(seed):
    g = torch.Generator().manual_seed(seed)
    fields = []
    for k in range(int(torch.randint(3, 7, (), generator=g))):
        kind = int(torch.randint(0, 3, (), generator=g))
        if kind == 0:
            f = synth.spectral((32, 40, 36), slope=-2.0, seed=seed * 10 + k)
        elif kind == 1:
            f = synth.spectral((90, 120), slope=-3.0, seed=seed * 10 + k, dtype=torch.float64)
        else:
            f = synth.gaussian_bumps((20, 20, 20), seed=seed * 10 + k)
        eb = float(10 ** (-2 - 4 * torch.rand((), generator=g)))
        fields.append((f.cuda(), eb))
    return fields


def _items(views):
    return [(v, eb, oracle.EB_REL, (1,) * v.dim(), oracle.OP_SELECT) for v, eb in views]


def _alone(ctx, items):
    return [ctx.run(op, f, eb, mode, st) for (f, eb, mode, st, op) in items]


def test_snapshots_in_the_mix_equal_alone(ctx):
    from paper_1806_08901_amd import szsel
    pool = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    srv = szsel.Server(ctx, pool, lanes=3)
    prod = torch.cuda.Stream()
    tickets, expect = [], {}
    for seed in range(6):
        snap = _snapshot(100 + seed)
        need = sum((f.numel() * f.element_size() + 255) // 256 * 256 for f, _ in snap)
        got = srv.reserve(need)
        while got is None:
            srv.progress(wait=True)
            got = srv.reserve(need)
        off, t = got
        views = []
        with torch.cuda.stream(prod):
            for f, eb in snap:
                views.append((_place(pool, off, f), eb))
                off += (f.numel() * f.element_size() + 255) // 256 * 256
        items = _items(views)
        srv.submit(t, items, stream=prod)
        tickets.append(t)
        expect[t] = (items, [(f, eb) for f, eb in snap])
    st = srv.stats()
    _note("in flight after submits:", st)
    results = {}
    while len(results) < len(tickets):
        srv.progress(wait=True)
        for t in tickets:
            if t not in results:
                r = srv.status(t)
                if r is not None:
                    results[t] = r[0]
    for t in tickets:
        items, orig = expect[t]
        alone = _alone(ctx, [(f, eb, m, st, op) for (f, eb), (_, _, m, st, op) in zip(orig, items)])
        assert results[t] == alone, "snapshot %d" % t
        # and against the oracle on the same values
        for (f, eb), (_, _, m, st, op), got in zip(orig, items, results[t]):
            want, _ = oracle.run(op, f.cpu().numpy(), eb, m, st)
            assert_matches_oracle(got, want, "snapshot %d eb %g" % (t, eb))
    assert srv.stats()["pool_reserved"] == 0
    srv.close()


def _serve(ctx, srv, pool, snaps, prod=None):
    """Reserves, fills and submits each snapshot (waiting for room), then
    drives the server until all complete.  snaps: list of [(field, eb)].
    Returns {index: results}."""
    tickets = {}
    for i, snap in enumerate(snaps):
        need = sum((f.numel() * f.element_size() + 255) // 256 * 256 for f, _ in snap)
        got = srv.reserve(need)
        while got is None:
            srv.progress(wait=True)
            got = srv.reserve(need)
        off, t = got
        views = []
        for f, eb in snap:
            views.append((_place(pool, off, f), eb))
            off += (f.numel() * f.element_size() + 255) // 256 * 256
        torch.cuda.synchronize()
        srv.submit(t, _items(views))
        tickets[t] = i
    out = {}
    while len(out) < len(tickets):
        srv.progress(wait=True)
        for t, i in tickets.items():
            if i not in out:
                r = srv.status(t)
                if r is not None:
                    out[i] = r[0]
    return out


def test_invalid_snapshot_refused_others_complete(ctx):
    from paper_1806_08901_amd import szsel
    pool = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    srv = szsel.Server(ctx, pool, lanes=2)
    good = [_snapshot(300), _snapshot(301)]
    f = synth.spectral((16, 16, 16), seed=302).cuda()
    nb = f.numel() * 4
    for bad_eb, bad_stride, what in ((0.0, 1, "eb"), (1e-3, -1, "stride")):
        off, t = srv.reserve(nb)
        v = _place(pool, off, f)
        with pytest.raises(szsel.SzselError, match=what):
            srv.submit(t, [(v, bad_eb, oracle.EB_REL, (bad_stride,) * 3, oracle.OP_SELECT)])
        srv.cancel(t)  # refused snapshots keep their reservation until cancelled
    res = _serve(ctx, srv, pool, good)
    for i, snap in enumerate(good):
        alone = [ctx.run(oracle.OP_SELECT, g, eb, oracle.EB_REL, (1,) * g.dim()) for g, eb in snap]
        assert res[i] == alone
        assert not any(r["flags"] & szsel.FLAG_FAILED for r in res[i])
    assert srv.stats()["pool_reserved"] == 0
    srv.close()


def test_lane_budget_limits_batches(ctx):
    from paper_1806_08901_amd import szsel
    pool = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    # about two requests' worth of workspace per lane (a request of these
    # sizes needs about 4.8 MB: mostly its 16 histogram copies)
    srv = szsel.Server(ctx, pool, lanes=1, lane_workspace_bytes=10 << 20)
    snaps = [_snapshot(310), _snapshot(311)]
    res = _serve(ctx, srv, pool, snaps)
    st = srv.stats()
    nreq = sum(len(s) for s in snaps)
    assert st["batches"] >= nreq // 2, st  # the budget split them into small batches
    for i, snap in enumerate(snaps):
        assert res[i] == [ctx.run(oracle.OP_SELECT, g, eb, oracle.EB_REL, (1,) * g.dim()) for g, eb in snap]
    # one request larger than a lane is refused at submission
    tiny = szsel.Server(ctx, pool, lanes=1, lane_workspace_bytes=1 << 20)
    f = synth.spectral((16, 16, 16), seed=312).cuda()
    off, t = tiny.reserve(f.numel() * 4)
    v = _place(pool, off, f)
    with pytest.raises(szsel.SzselError, match="lane"):
        tiny.submit(t, [(v, 1e-3, oracle.EB_REL, (1, 1, 1), oracle.OP_SELECT)])
    tiny.cancel(t)
    tiny.close()
    srv.close()


@pytest.mark.parametrize("failures", [1, 1000])
def test_failed_batches_retry_in_halves(ctx, failures):
    from paper_1806_08901_amd import szsel
    pool = torch.empty(32 << 20, dtype=torch.uint8, device="cuda")
    os.environ["SZSEL_SERVER_FAIL_BATCHES"] = str(failures)
    try:
        srv = szsel.Server(ctx, pool, lanes=1)
    finally:
        del os.environ["SZSEL_SERVER_FAIL_BATCHES"]
    snap = _snapshot(320)
    res = _serve(ctx, srv, pool, [snap])[0]
    alone = [ctx.run(oracle.OP_SELECT, g, eb, oracle.EB_REL, (1,) * g.dim()) for g, eb in snap]
    if failures == 1:  # the first batch failed; its halves ran
        assert res == alone
    else:  # nothing could run: every request completes flagged, the pool is free again
        assert all(r["flags"] == szsel.FLAG_FAILED and r["choice"] == -1 for r in res)
    assert srv.stats()["pool_reserved"] == 0
    srv.close()


def test_admission_waits_for_room(ctx):
    from paper_1806_08901_amd import szsel
    f = synth.spectral((64, 64, 64), seed=120).cuda()
    nb = f.numel() * 4
    pool = torch.empty(nb + 4096, dtype=torch.uint8, device="cuda")  # one snapshot at a time
    srv = szsel.Server(ctx, pool, lanes=2)
    off, t1 = srv.reserve(nb)
    v = _place(pool, off, f)
    items = [(v, 1e-4, oracle.EB_REL, (2, 2, 1), oracle.OP_SELECT)]
    srv.submit(t1, items)
    assert srv.reserve(nb) is None                # busy until the first completes
    while srv.status(t1) is None:
        srv.progress(wait=True)
    got = srv.reserve(nb)
    assert got is not None
    srv.cancel(got[1])
    srv.close()


def test_submit_rejects_fields_outside_the_reservation(ctx):
    from paper_1806_08901_amd import szsel
    pool = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    srv = szsel.Server(ctx, pool, lanes=1)
    off, t = srv.reserve(4096)
    outside = torch.zeros(64, 64, device="cuda")
    with pytest.raises(szsel.SzselError, match="outside"):
        srv.submit(t, [(outside, 1e-3, oracle.EB_REL, (1, 1), oracle.OP_SELECT)])
    srv.cancel(t)
    srv.close()
