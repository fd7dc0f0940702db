"""Exact Huffman cost of the SZ code histogram on the GPU against the oracle
(needs a GPU).

The optimal prefix code's total length is unique, so the device's run-length
merge must give the oracle's heap-built cost bit for bit, and so must the
bit-rate derived from it and, with option value 2, the selection made with
it.  Asking for the cost changes no other output.
"""
import sys

import pytest
import torch

import oracle
from paper_1806_08901_amd import synth
from tests.gpu_common import assert_matches_oracle

pytestmark = pytest.mark.gpu

HUFF_KEYS = ("sz_huffman_bits", "sz_huffman_bitrate")


def _note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1806_08901_amd import szsel
    c = szsel.Context(0)
    yield c
    c.set_option(szsel.OPT_HUFFMAN, 0)
    c.close()


def _with_huffman(ctx, mode, fn):
    from paper_1806_08901_amd import szsel
    ctx.set_option(szsel.OPT_HUFFMAN, mode)
    try:
        return fn()
    finally:
        ctx.set_option(szsel.OPT_HUFFMAN, 0)


CASES = [
    ("bumps3d", lambda: synth.gaussian_bumps((40, 44, 36), seed=81), (1, 1, 1)),
    ("spectral3d_f64", lambda: synth.spectral((36, 40, 33), slope=-3.0, seed=82, dtype=torch.float64), (2, 1, 1)),
    ("spectral2d", lambda: synth.spectral((130, 170), slope=-2.0, seed=83), (1, 1)),
    ("spectral2d_f64", lambda: synth.spectral((90, 75), seed=84, dtype=torch.float64), (1, 2)),
    ("bumps1d", lambda: synth.gaussian_bumps((4099,), sigma_range=(3.0, 40.0), seed=85), (1,)),
    ("spiky2d", lambda: synth.spiky_constant((64, 80), frac=0.01, seed=86), (1, 1)),
]


@pytest.mark.parametrize("name,make,stride", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("eb", [1e-2, 1e-4, 1e-6])
def test_huffman_cost_matches_oracle(ctx, name, make, stride, eb):
    x = make()
    _note("huffman", name, tuple(x.shape), x.dtype, eb, stride)
    xd = x.cuda()
    for op in (oracle.OP_SZ, oracle.OP_SELECT):
        gpu = _with_huffman(ctx, 1, lambda: ctx.run(op, xd, eb, oracle.EB_REL, stride))
        orc, _ = oracle.run(op, x.numpy(), eb, oracle.EB_REL, stride, huffman=1)
        assert_matches_oracle(gpu, orc, "%s eb %g op %d" % (name, eb, op))
        assert gpu["sz_huffman_bits"] > 0
        plain = ctx.run(op, xd, eb, oracle.EB_REL, stride)
        assert all(plain[k] == 0 for k in HUFF_KEYS)
        assert {k: v for k, v in gpu.items() if k not in HUFF_KEYS} == \
            {k: v for k, v in plain.items() if k not in HUFF_KEYS}


@pytest.mark.parametrize("eb", [1e-3, 1e-5])
def test_selection_with_huffman_bitrate(ctx, eb):
    x = synth.spectral((48, 40, 44), slope=-2.5, seed=87)
    xd = x.cuda()
    for op, mode in ((oracle.OP_SELECT, oracle.EB_REL), (oracle.OP_FIXED_EB, oracle.EB_REL)):
        gpu = _with_huffman(ctx, 2, lambda: ctx.run(op, xd, eb, mode, (1, 1, 1)))
        orc, _ = oracle.run(op, x.numpy(), eb, mode, (1, 1, 1), huffman=2)
        assert_matches_oracle(gpu, orc, "select-with-huffman eb %g op %d" % (eb, op))


def test_single_symbol_costs_one_bit_per_value(ctx):
    """Zero on every sampled block, the only nonzero value in the ragged
    tail: every code is the centre code."""
    x = torch.zeros(66, 66)
    x[65, 65] = 1.0
    gpu = _with_huffman(ctx, 1, lambda: ctx.run(oracle.OP_SZ, x.cuda(), 1e-3, oracle.EB_REL, (1, 1)))
    orc, _ = oracle.run(oracle.OP_SZ, x.numpy(), 1e-3, oracle.EB_REL, (1, 1), huffman=1)
    assert_matches_oracle(gpu, orc, "one symbol")
    assert gpu["sz_huffman_bits"] == gpu["sz_values"] == 4096


def test_constant_field_reports_no_cost(ctx):
    x = torch.full((32, 32), 2.5, device="cuda")
    gpu = _with_huffman(ctx, 2, lambda: ctx.select(x, 1e-3))
    assert gpu["sz_huffman_bits"] == 0 and gpu["choice"] == 0


def test_many_large_counts_are_sorted(ctx):
    """16.7 M sampled values of noise: about 1000 codes occur 8192 times or
    more, so the sorted list of large counts is exercised."""
    g = torch.Generator().manual_seed(88)
    x = torch.rand(4096, 4096, generator=g)
    gpu = _with_huffman(ctx, 1, lambda: ctx.run(oracle.OP_SZ, x.cuda(), 5e-4, oracle.EB_ABS, (1, 1)))
    orc, dump = oracle.run(oracle.OP_SZ, x.numpy(), 5e-4, oracle.EB_ABS, (1, 1), huffman=1, dump=True)
    assert (dump["hist"] >= 8192).sum() > 500
    assert_matches_oracle(gpu, orc, "noise 4096^2")


def test_too_many_distinct_counts_fall_back(ctx):
    """105 M sampled values of noise with bins of 2 eb: the counts take some
    9000 distinct values, more than the pass holds, so the cost is not
    computed, the flag says so, and the selection falls back to entropy +
    offset."""
    from paper_1806_08901_amd import szsel
    g = torch.Generator(device="cuda").manual_seed(89)
    x = torch.rand(10240, 10240, generator=g, device="cuda")
    plain = ctx.run(oracle.OP_FIXED_EB, x, 1e-4, oracle.EB_ABS, (1, 1))
    for mode in (1, 2):
        got = _with_huffman(ctx, mode, lambda: ctx.run(oracle.OP_FIXED_EB, x, 1e-4, oracle.EB_ABS, (1, 1)))
        assert got["flags"] == plain["flags"] | szsel.FLAG_NO_HUFFMAN
        assert got["sz_huffman_bits"] == 0
        assert {k: v for k, v in got.items() if k != "flags"} == {k: v for k, v in plain.items() if k != "flags"}


def test_batch_with_huffman_equals_single_calls(ctx):
    fields = [synth.spectral((40, 36, 44), seed=90).cuda(),
              synth.spectral((60, 90), slope=-1.5, seed=91, dtype=torch.float64).cuda(),
              synth.gaussian_bumps((1030,), sigma_range=(3.0, 30.0), seed=92).cuda()]
    ops = [oracle.OP_SELECT, oracle.OP_SZ, oracle.OP_ZFP, oracle.OP_FIXED_EB]
    items = [(f, eb, oracle.EB_REL, (1,) * f.dim(), ops[(i + j) % 4])
             for i, f in enumerate(fields) for j, eb in enumerate((1e-2, 1e-4, 1e-6))]
    for mode in (1, 2):
        batch = _with_huffman(ctx, mode, lambda: ctx.select_batch(items))
        singles = _with_huffman(ctx, mode, lambda: [ctx.run(op, f, eb, m, st) for (f, eb, m, st, op) in items])
        assert batch == singles, "huffman %d" % mode
        for (f, eb, m, st, op), b in zip(items, batch):
            if op != oracle.OP_ZFP:
                assert b["sz_huffman_bits"] > 0
    host = fields[1].cpu().numpy()
    orc, _ = oracle.run(oracle.OP_SELECT, host, 1e-6, oracle.EB_REL, (1, 1), huffman=2)
    got = _with_huffman(ctx, 2, lambda: ctx.select_batch([(fields[1], 1e-6, oracle.EB_REL, (1, 1), oracle.OP_SELECT)]))
    assert_matches_oracle(got[0], orc, "batch huffman=2")


def test_option_values(ctx):
    from paper_1806_08901_amd import szsel
    for bad in (-1, 3, 0.5):
        with pytest.raises(szsel.SzselError, match="Huffman"):
            ctx.set_option(szsel.OPT_HUFFMAN, bad)
