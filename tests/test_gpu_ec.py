"""The paper's point sub-sampling of the ZFP side on the GPU against the
oracle (needs a GPU): 3/9/16 sampled coefficients per block, interpolated
significant-bit rate, transform-domain MSE of the sampled points (plain, or
weighted by the inverse transform's column norms), and the selection made
with them; bit-exact like the exact path."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1806_08901_amd import synth
from tests.gpu_common import assert_matches_oracle, debug_buffers, debug_to_numpy

pytestmark = pytest.mark.gpu

OPS = [oracle.OP_ZFP, oracle.OP_SELECT, oracle.OP_FIXED_EB]


def _note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1806_08901_amd import szsel
    c = szsel.Context(0)
    yield c
    c.set_option(szsel.OPT_EC_SAMPLING, 0)
    c.close()


def _with_ec(ctx, mode, fn):
    from paper_1806_08901_amd import szsel
    ctx.set_option(szsel.OPT_EC_SAMPLING, mode)
    try:
        return fn()
    finally:
        ctx.set_option(szsel.OPT_EC_SAMPLING, 0)


CASES = [
    ("bumps 3d f32", lambda: synth.gaussian_bumps((24, 20, 28), seed=51), (1, 1, 1)),
    ("ragged 3d f32", lambda: synth.spectral((37, 29, 43), slope=-2.0, seed=52), (2, 1, 1)),
    ("3d f64", lambda: synth.spectral((21, 34, 27), slope=-3.0, seed=53, dtype=torch.float64), (1, 2, 1)),
    ("2d f32", lambda: synth.spectral((45, 70), slope=-2.5, seed=54), (1, 1)),
    ("2d f64 stride", lambda: synth.spectral((66, 131), slope=-1.5, seed=55, dtype=torch.float64), (3, 1)),
    ("1d f32", lambda: synth.gaussian_bumps((1003,), sigma_range=(3.0, 40.0), seed=56), (1,)),
    ("1d f64", lambda: synth.spectral((777,), slope=-1.0, seed=57, dtype=torch.float64), (2,)),
    ("spiky 2d", lambda: synth.spiky_constant((52, 64), frac=0.02, seed=58), (1, 1)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", [1, 2])
def test_sub_sampled_estimate_matches_oracle(ctx, case, mode):
    label, make, stride = case
    x = make()
    xd = x.cuda()
    for op in OPS:
        for eb in (1e-2, 1e-4, 1e-6):
            _note("ec", mode, label, "op", op, "eb", eb)
            gpu = _with_ec(ctx, mode, lambda: ctx.run(op, xd, eb, oracle.EB_REL, stride))
            orc, _ = oracle.run(op, x.numpy(), eb, oracle.EB_REL, stride, ec_points=1, ec_weight=mode - 1)
            assert_matches_oracle(gpu, orc, "%s mode %d op %d eb %g" % (label, mode, op, eb))
            assert gpu["flags"] & oracle.FLAG_EC_SAMPLED


def test_per_block_counts_and_errors(ctx):
    """Per sampled block: twice the interpolated significant bits, and the
    pair-tree sum of the sampled points' squared errors."""
    x = synth.spectral((40, 36, 44), slope=-2.0, seed=59)
    st = (1, 1, 1)
    nblk = oracle.num_sampled_blocks(tuple(x.shape), st)
    bufs = debug_buffers(torch, nblk, 3)
    ctx.set_debug(bufs)
    gpu = _with_ec(ctx, 1, lambda: ctx.run(oracle.OP_ZFP, x.cuda(), 1e-4, oracle.EB_REL, st))
    gd = debug_to_numpy(bufs, nblk, 3)
    orc, od = oracle.run(oracle.OP_ZFP, x.numpy(), 1e-4, oracle.EB_REL, st, dump=True, ec_points=1)
    assert_matches_oracle(gpu, orc, "per-block")
    assert np.array_equal(gd["zfp_bits"], od["ec_nsb2"])
    assert np.array_equal(gd["zfp_emax"], od["zfp_emax"])
    e2 = od["ec_err"].reshape(nblk, 16) ** 2
    while e2.shape[1] > 1:
        e2 = e2[:, 0::2] + e2[:, 1::2]
    assert np.array_equal(gd["zfp_sse"], e2[:, 0])


def test_batch_with_sub_sampling_equals_single_calls(ctx):
    fields = [synth.spectral((40, 36, 44), seed=60).cuda(),
              synth.spectral((60, 90), slope=-1.5, seed=61, dtype=torch.float64).cuda(),
              synth.gaussian_bumps((1030,), sigma_range=(3.0, 30.0), seed=62).cuda()]
    ops = [oracle.OP_SELECT, oracle.OP_ZFP, oracle.OP_FIXED_EB, oracle.OP_SZ]
    items = [(f, eb, oracle.EB_REL, (1,) * f.dim(), ops[(i + j) % 4])
             for i, f in enumerate(fields) for j, eb in enumerate((1e-2, 1e-4, 1e-6))]
    for mode in (1, 2):
        batch = _with_ec(ctx, mode, lambda: ctx.select_batch(items))
        singles = _with_ec(ctx, mode, lambda: [ctx.run(op, f, eb, m, st) for (f, eb, m, st, op) in items])
        assert batch == singles, "mode %d" % mode
    exact = ctx.select_batch(items)
    assert all(not (r["flags"] & oracle.FLAG_EC_SAMPLED) for r in exact)


def test_full_size_sweep_matches_oracle(ctx):
    """The 512^3 benchmark field, stride (5, 4, 1), the five bounds, both
    weightings: one batch against the oracle."""
    field = synth.workload_turb512(device="cuda")
    host = field.cpu().numpy()
    items = [(field, eb, oracle.EB_REL, (5, 4, 1), oracle.OP_SELECT) for eb in synth.EB_SWEEP]
    for mode in (1, 2):
        batch = _with_ec(ctx, mode, lambda: ctx.select_batch(items))
        for eb, g in zip(synth.EB_SWEEP, batch):
            _note("turb512 ec", mode, "eb", eb)
            orc, _ = oracle.run(oracle.OP_SELECT, host, eb, oracle.EB_REL, (5, 4, 1), ec_points=1,
                                ec_weight=mode - 1)
            assert_matches_oracle(g, orc, "turb512 mode %d eb %g" % (mode, eb))


def test_option_values(ctx):
    from paper_1806_08901_amd import szsel
    for bad in (-1, 3, 1.5):
        with pytest.raises(szsel.SzselError, match="EC sampling"):
            ctx.set_option(szsel.OPT_EC_SAMPLING, bad)
