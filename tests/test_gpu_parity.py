"""HIP path vs CPU oracle, element by element, through the C ABI (needs a GPU)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1806_08901_amd import synth
from tests.gpu_common import (assert_matches_oracle, debug_buffers, debug_to_numpy, is_tie)

pytestmark = pytest.mark.gpu

OPS = [oracle.OP_SZ, oracle.OP_ZFP, oracle.OP_SELECT, oracle.OP_FIXED_EB]


@pytest.fixture(scope="module")
def ctx():
    from paper_1806_08901_amd import szsel
    c = szsel.Context(0)
    yield c
    c.close()


def _note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run_both(ctx, x_cpu: torch.Tensor, op, eb, mode=oracle.EB_REL, stride=None, dump=False):
    xd = x_cpu.cuda()
    nd = x_cpu.dim()
    st = tuple(stride) if stride is not None else (1,) * nd
    orc, odump = oracle.run(op, x_cpu.numpy(), eb, mode, st, dump=dump)
    gdump = None
    if dump:
        nblk = oracle.num_sampled_blocks(tuple(x_cpu.shape), st)
        bufs = debug_buffers(torch, nblk, nd)
        ctx.set_debug(bufs)
        gpu = ctx.run(op, xd, eb, mode, st)
        gdump = debug_to_numpy(bufs, nblk, nd)
    else:
        gpu = ctx.run(op, xd, eb, mode, st)
    return gpu, orc, gdump, odump


def _compare_dumps(gd, od, op, orc):
    if op != oracle.OP_SZ and not (orc["flags"] & 0x3B):
        assert np.array_equal(gd["zfp_bits"], od["zfp_bits"])
        assert np.array_equal(gd["zfp_emax"], od["zfp_emax"])
        assert np.array_equal(gd["zfp_sse"], od["zfp_sse"])
    if op != oracle.OP_ZFP and not (orc["flags"] & 0x3B):
        assert np.array_equal(gd["codes"], od["codes"])
        assert np.array_equal(gd["hist"], od["hist"])
        assert np.array_equal(gd["sz_sse"], od["sz_sse"])


SMALL_CASES = [
    # (label, maker, eb, stride)
    ("bumps 24x20x28 f32", lambda: synth.gaussian_bumps((24, 20, 28), seed=31), 1e-4, (1, 1, 1)),
    ("ragged 3d 37x29x43 f32", lambda: synth.spectral((37, 29, 43), slope=-2.0, seed=32), 1e-3, (2, 1, 1)),
    ("ragged 3d f64", lambda: synth.spectral((21, 34, 27), slope=-3.0, seed=33, dtype=torch.float64),
     1e-6, (1, 2, 1)),
    ("2d 45x70 f32", lambda: synth.spectral((45, 70), slope=-2.5, seed=34), 1e-4, (1, 1)),
    ("2d 66x131 f64 stride", lambda: synth.spectral((66, 131), slope=-1.5, seed=35, dtype=torch.float64),
     1e-2, (3, 1)),
    ("1d 1003 f32", lambda: synth.gaussian_bumps((1003,), sigma_range=(3.0, 40.0), seed=36), 1e-5, (1,)),
    ("1d 777 f64 stride", lambda: synth.spectral((777,), slope=-1.0, seed=37, dtype=torch.float64), 1e-3, (2,)),
    ("spiky 2d", lambda: synth.spiky_constant((52, 64), frac=0.02, seed=38), 1e-2, (1, 1)),
    ("noise 3d eb 1e-6", lambda: torch.randn(16, 24, 20, generator=torch.Generator().manual_seed(39)),
     1e-6, (1, 1, 1)),
]


@pytest.mark.parametrize("case", SMALL_CASES, ids=[c[0] for c in SMALL_CASES])
@pytest.mark.parametrize("op", OPS)
def test_small_fields_bit_exact(ctx, case, op):
    label, make, eb, stride = case
    _note("case", label, "op", op)
    x = make()
    gpu, orc, gd, od = _run_both(ctx, x, op, eb, oracle.EB_REL, stride, dump=True)
    assert_matches_oracle(gpu, orc, label)
    _compare_dumps(gd, od, op, orc)


def test_bumps64_every_block(ctx):
    """64^3 FP32 Gaussian bumps, eb_rel 1e-4, every block and point sampled."""
    x = synth.workload_bumps64()
    for op in OPS:
        gpu, orc, gd, od = _run_both(ctx, x, op, 1e-4, oracle.EB_REL, (1, 1, 1), dump=True)
        assert_matches_oracle(gpu, orc, "bumps64 op %d" % op)
        _compare_dumps(gd, od, op, orc)


def test_absolute_error_bounds(ctx):
    x = synth.spectral((40, 40, 40), seed=41)
    for eb in (1e-1, 1e-3, 3.7e-5):
        gpu, orc, _, _ = _run_both(ctx, x, oracle.OP_SELECT, eb, oracle.EB_ABS, (2, 2, 1))
        assert_matches_oracle(gpu, orc, "abs eb %g" % eb)


def test_extreme_magnitudes(ctx):
    g = torch.Generator().manual_seed(42)
    cases = {
        "tiny f32 (subnormals)": (torch.randn(16, 16, 16, generator=g) * 1e-40).float(),
        "huge f32": (torch.randn(16, 16, 16, generator=g) * 1e37).float(),
        "tiny f64": torch.randn(12, 16, 20, generator=g, dtype=torch.float64) * 1e-310,
        "huge f64": torch.randn(12, 16, 20, generator=g, dtype=torch.float64) * 1e300,
        "mixed scales f32": (torch.randn(32, 32, generator=g) * torch.logspace(-20, 20, 32)).float(),
        "signed zeros": torch.tensor([0.0, -0.0] * 128, dtype=torch.float32).view(16, 16)
        + torch.eye(16) * 1e-3,
    }
    for label, x in cases.items():
        for eb in (1e-2, 1e-5):
            gpu, orc, gd, od = _run_both(ctx, x.contiguous(), oracle.OP_SELECT, eb, oracle.EB_REL,
                                         None, dump=True)
            assert_matches_oracle(gpu, orc, label)
            _compare_dumps(gd, od, oracle.OP_SELECT, orc)


def test_degenerate_fields(ctx):
    c = torch.full((8, 8, 8), 3.25)
    for op in OPS:
        gpu, orc, _, _ = _run_both(ctx, c, op, 1e-3)
        assert_matches_oracle(gpu, orc, "constant")
    nanf = torch.ones(8, 12)
    nanf[3, 5] = float("nan")
    inff = torch.ones(8, 12, dtype=torch.float64)
    inff[7, 11] = -float("inf")
    for x in (nanf, inff):
        gpu, orc, _, _ = _run_both(ctx, x, oracle.OP_SELECT, 1e-3)
        assert_matches_oracle(gpu, orc, "nonfinite")
        assert gpu["flags"] & oracle.FLAG_NONFINITE
    small = torch.arange(27, dtype=torch.float32).view(3, 3, 3)
    gpu, orc, _, _ = _run_both(ctx, small, oracle.OP_SELECT, 1e-3)
    assert_matches_oracle(gpu, orc, "no blocks")
    blocks = torch.arange(8, dtype=torch.float32).view(2, 2, 2)
    pc = torch.kron(blocks, torch.ones(4, 4, 4)).contiguous()
    gpu, orc, _, _ = _run_both(ctx, pc, oracle.OP_SELECT, 1e-3)
    assert_matches_oracle(gpu, orc, "zero mse")
    assert gpu["flags"] & oracle.FLAG_ZERO_MSE
    lin = torch.linspace(0, 1e-10, 512, dtype=torch.float64).view(8, 8, 8)
    gpu, orc, _, _ = _run_both(ctx, lin, oracle.OP_SELECT, 1e-320)
    assert_matches_oracle(gpu, orc, "bad eb")


def test_unaligned_field_pointer(ctx):
    base = synth.spectral((4 * 33 * 40 + 3,), seed=43)
    for off in (1, 2, 3):
        x = base[off:off + 33 * 40 * 4].view(33, 160)
        xd = base.cuda()[off:off + 33 * 40 * 4].view(33, 160)
        assert xd.data_ptr() % 16 != 0
        orc, _ = oracle.run(oracle.OP_SELECT, x.contiguous().numpy(), 1e-4, oracle.EB_REL, (1, 1))
        gpu = ctx.run(oracle.OP_SELECT, xd, 1e-4, oracle.EB_REL, (1, 1))
        assert_matches_oracle(gpu, orc, "offset %d" % off)


def test_repeatable(ctx):
    x = synth.spectral((64, 64, 64), seed=44).cuda()
    a = ctx.select(x, 1e-4, stride=(2, 2, 1))
    b = ctx.select(x, 1e-4, stride=(2, 2, 1))
    assert a == b


def test_batch_equals_single(ctx):
    items = []
    fields = [synth.spectral((40, 36, 44), seed=45).cuda(),
              synth.spectral((60, 90), seed=46, dtype=torch.float64).cuda(),
              synth.gaussian_bumps((24, 24, 24), seed=47).cuda(),
              torch.full((16, 16), 2.0, device="cuda")]
    for i, f in enumerate(fields):
        for eb in (1e-2, 1e-4, 1e-6):
            st = (1,) * f.dim()
            items.append((f, eb, oracle.EB_REL, st, OPS[(i + int(-math.log10(eb))) % 4]))
    batch = ctx.select_batch(items)
    for (f, eb, mode, st, op), b in zip(items, batch):
        single = ctx.run(op, f, eb, mode, st)
        assert b == single


@pytest.fixture(scope="module")
def turb512():
    _note("generating 512^3 turbulent field")
    return synth.workload_turb512(device="cuda")


@pytest.mark.parametrize("eb", synth.EB_SWEEP)
def test_turb512_full_size(ctx, turb512, eb):
    """512^3 FP32, default ~5% stride, the launch configuration the benchmark times."""
    _note("turb512 eb", eb)
    stride = (5, 4, 1)
    gpu = ctx.select(turb512, eb, stride=stride)
    orc, _ = oracle.select(turb512.cpu().numpy(), eb, stride=stride)
    assert_matches_oracle(gpu, orc, "turb512 eb %g" % eb)
    assert not is_tie(orc)


def test_turb512_most_range_chunks(ctx, turb512):
    """The largest range-chunk setting (64 per CU: more chunks than a pass
    holds on this field) is capped at the pass's limit instead of failing,
    and gives the default schedule's results."""
    from paper_1806_08901_amd import szsel
    stride = (5, 4, 1)
    ref = ctx.select(turb512, 1e-3, stride=stride)
    try:
        ctx.set_option(szsel.OPT_RANGE_WGS, 64)
        assert ctx.select(turb512, 1e-3, stride=stride) == ref
    finally:
        ctx.set_option(szsel.OPT_RANGE_WGS, 0)


@pytest.mark.parametrize("eb", [1e-5, 1e-6])
def test_turb512_full_dump_tight_bounds(ctx, turb512, eb):
    """512^3 at the tight bounds, where the histogram is widest and the
    overflow pass counts most codes: every code, the 65,536-bin histogram
    and every per-block ZFP and SZ value against the oracle."""
    _note("turb512 dump eb", eb)
    stride = (5, 4, 1)
    nblk = oracle.num_sampled_blocks((512, 512, 512), stride)
    bufs = debug_buffers(torch, nblk, 3)
    ctx.set_debug(bufs)
    gpu = ctx.select(turb512, eb, stride=stride)
    gd = debug_to_numpy(bufs, nblk, 3)
    orc, od = oracle.select(turb512.cpu().numpy(), eb, stride=stride, dump=True)
    assert_matches_oracle(gpu, orc, "turb512 dump eb %g" % eb)
    _compare_dumps(gd, od, oracle.OP_SELECT, orc)
    assert int((od["hist"] > 0).sum()) > 4096  # wider than the SZ pass's LDS window


@pytest.mark.parametrize("eb", [1e-2, 1e-6])
def test_turb512_long_sz_workgroups(ctx, turb512, eb):
    """512^3 with SZ workgroups of 2,048 sampled blocks (8 tiles, 131,072
    points per workgroup, 52 workgroups): at 1e-2 most points share a few
    bins of the LDS window, at 1e-6 most codes go through the overflow
    regions.  Codes and the histogram equal the oracle's bin for bin, and
    the results equal the default schedule's."""
    from paper_1806_08901_amd import szsel
    _note("turb512 long SZ workgroups eb", eb)
    stride = (5, 4, 1)
    ref = ctx.select(turb512, eb, stride=stride)
    nblk = oracle.num_sampled_blocks((512, 512, 512), stride)
    bufs = debug_buffers(torch, nblk, 3)
    try:
        ctx.set_option(szsel.OPT_SZ_WGS, 1)  # 64 SZ workgroups for 106,496 blocks
        ctx.set_debug(bufs)
        gpu = ctx.select(turb512, eb, stride=stride)
    finally:
        ctx.set_option(szsel.OPT_SZ_WGS, 0)
    gd = debug_to_numpy(bufs, nblk, 3)
    assert gpu == ref
    orc, od = oracle.select(turb512.cpu().numpy(), eb, stride=stride, dump=True)
    assert_matches_oracle(gpu, orc, "turb512 long SZ workgroups eb %g" % eb)
    assert np.array_equal(gd["hist"], od["hist"])
    assert np.array_equal(gd["codes"], od["codes"])


@pytest.mark.parametrize("dtype,offset,want", [(torch.float32, 0.5, 6.25), (torch.float64, 0.25, 10.0)])
def test_sz_bitrate_hand_fixture(ctx, dtype, offset, want):
    """The 16-value field whose codes are known by construction (8 x 0, 4 x 1,
    2 x 2 and 2 escapes at delta = 1): entropy 1.75 bits, bit-rate by hand."""
    from paper_1806_08901_amd import szsel
    steps = [0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 40000, 40000, 0, 0, 0, 0]
    x = torch.tensor(steps, dtype=torch.float64).cumsum(0).to(dtype).cuda()
    ctx.set_option(szsel.OPT_SZ_OFFSET, offset)
    ctx.set_option(szsel.OPT_HUFFMAN, 1)
    try:
        r = ctx.estimate_sz(x, 0.5, oracle.EB_ABS, (1,))
    finally:
        ctx.set_option(szsel.OPT_SZ_OFFSET, 0.5)
        ctx.set_option(szsel.OPT_HUFFMAN, 0)
    W = 32 if dtype == torch.float32 else 64
    assert r["sz_unpredictable"] == 2 and r["sz_entropy"] == 1.75
    assert r["sz_bitrate"] == want
    assert r["sz_huffman_bits"] == 28 and r["sz_huffman_bitrate"] == 1.75 + 2 * W / 16
