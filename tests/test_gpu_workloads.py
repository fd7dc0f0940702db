"""The batched workloads at full size, in the launch configuration the
benchmark times (one batch, autotuned schedule), against single calls (every
request, bit for bit) and the CPU oracle (a sample of requests)."""
import sys

import pytest
import torch

import oracle
from paper_1806_08901_amd import synth
from tests.gpu_common import assert_matches_oracle, is_tie

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


def _run_workload(ctx, specs, sample):
    from paper_1806_08901_amd import szsel
    fields = [synth.make_field(sp, device="cuda") for sp in specs]
    torch.cuda.synchronize()
    items = [(f, sp["eb"], szsel.EB_REL, (20, 1) if f.dim() == 2 else (5, 4, 1), szsel.OP_SELECT)
             for f, sp in zip(fields, specs)]
    try:
        ctx.set_option(szsel.OPT_AUTOTUNE, 1)
        batch = ctx.select_batch(items)
        again = ctx.select_batch(items)  # graph replay
    finally:
        ctx.set_option(szsel.OPT_AUTOTUNE, 0)
    assert again == batch
    for k, ((f, eb, m, st, op), b) in enumerate(zip(items, batch)):
        assert b == ctx.run(op, f, eb, m, st), "request %d vs its single call" % k
    for k in sample:
        f, eb, m, st, op = items[k]
        _note("oracle on request", k, tuple(f.shape), f.dtype)
        orc, _ = oracle.run(oracle.OP_SELECT, f.cpu().numpy(), eb, m, st)
        assert_matches_oracle(batch[k], orc, "request %d" % k)
        assert not is_tie(orc)


def test_atm79_full_size(ctx):
    """79 FP32 fields of 1800x3600 (every tenth mostly constant with spikes),
    eb_rel from {1e-2, 1e-4, 1e-6}, stride (20, 1)."""
    specs = synth.workload_atm_specs()
    _run_workload(ctx, specs, sample=[0, 9, 19, 33, 47, 58, 69, 78])


def test_mix3d_full_size(ctx):
    """13 x 100x500x500 FP32, 6 x 256x384x384 FP64, 4 x 512^3 FP32 and
    20 x 64^3 FP32, stride (5, 4, 1): 5.28 GB in one batch."""
    specs = synth.workload_mix3d_specs()
    kinds = {}
    for k, sp in enumerate(specs):
        kinds.setdefault((sp["shape"], str(sp["dtype"])), k)
    _run_workload(ctx, specs, sample=sorted(kinds.values()) + [len(specs) - 1])
