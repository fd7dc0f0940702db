"""Step 4 ZFP compression of the whole field on the GPU against the oracle
(needs a GPU): the stream word for word, the decompressed field value for
value, the totals bit for bit, and the round trip within the bound."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1806_08901_amd import synth

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


CASES = [
    ("1d ragged f32", lambda: synth.gaussian_bumps((1030,), sigma_range=(3.0, 30.0), seed=81)),
    ("1d f64", lambda: synth.spectral((777,), slope=-1.0, seed=82, dtype=torch.float64)),
    ("2d f32", lambda: synth.spectral((70, 90), slope=-2.0, seed=83)),
    ("2d ragged f64", lambda: synth.spectral((66, 131), slope=-1.5, seed=84, dtype=torch.float64)),
    ("3d ragged f32", lambda: synth.spectral((37, 29, 43), slope=-2.0, seed=85)),
    ("3d f64", lambda: synth.spectral((21, 34, 28), slope=-3.0, seed=86, dtype=torch.float64)),
    ("spiky 2d", lambda: synth.spiky_constant((52, 64), frac=0.02, seed=87)),
    ("tiny 3d", lambda: synth.spectral((3, 2, 5), seed=88)),
]

KEYS = ("bits", "values", "blocks", "bitrate", "sse", "mse", "psnr", "maxerr", "vr", "eb_abs")


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("eb", [1e-2, 1e-4, 1e-6])
def test_compression_matches_oracle(ctx, case, eb):
    label, make = case
    x = make()
    host = x.numpy()
    eb_abs = eb * float(host.max() - host.min())
    _note("step4 zfp", label, eb)
    gpu, words, dec = ctx.zfp_compress(x.cuda(), eb_abs)
    orc, owords, odec = oracle.zfp_compress(host, eb_abs)
    for k in KEYS:
        assert gpu[k] == orc[k], "%s: gpu %r oracle %r" % (k, gpu[k], orc[k])
    assert np.array_equal(words.cpu().numpy().view(np.uint64), owords)
    assert np.array_equal(dec.cpu().numpy().astype(np.float64), odec)
    assert gpu["maxerr"] <= eb_abs


def test_whole_blocks_match_the_estimator(ctx):
    """On a field of whole blocks the stream holds the bits the estimator
    counts at stride 1."""
    from paper_1806_08901_amd import szsel
    x = synth.spectral((64, 48, 32), slope=-2.0, seed=89).cuda()
    for eb in (1e-2, 1e-5):
        est = ctx.run(szsel.OP_ZFP, x, eb, szsel.EB_REL, (1, 1, 1))
        gpu, _, _ = ctx.zfp_compress(x, est["eb_abs"], decoded=False)
        assert gpu["bits"] == est["zfp_bits"]
        assert gpu["sse"] == est["zfp_sse"]


def test_full_size_field(ctx):
    """The 512^3 benchmark field at three bounds: totals against the
    estimator at stride 1 (whole blocks), the round trip, and the stream
    and decompressed values of sampled blocks against the oracle."""
    from paper_1806_08901_amd import szsel
    field = synth.workload_turb512(device="cuda")
    for eb in (1e-2, 1e-4, 1e-6):
        est = ctx.run(szsel.OP_ZFP, field, eb, szsel.EB_REL, (1, 1, 1))
        gpu, words, dec = ctx.zfp_compress(field, est["eb_abs"])
        _note("turb512 step4 eb", eb, gpu["bitrate"], gpu["psnr"])
        assert gpu["bits"] == est["zfp_bits"]
        assert gpu["sse"] == est["zfp_sse"]
        assert gpu["maxerr"] == est["zfp_maxerr"] <= est["eb_abs"]
        err = (dec.double() - field.double()).abs().max().item()
        assert err == gpu["maxerr"]
        # one 16^3 corner against the oracle's decompression of that corner
        # (whole blocks, so the blocks and their bits are the same)
        sub = field[:16, :16, :16].contiguous()
        _, _, odec = oracle.zfp_compress(sub.cpu().numpy(), est["eb_abs"])
        assert np.array_equal(dec[:16, :16, :16].cpu().numpy().astype(np.float64), odec)


def test_argument_errors(ctx):
    from paper_1806_08901_amd import szsel
    x = synth.spectral((20, 20), seed=90).cuda()
    with pytest.raises(szsel.SzselError, match="eb_abs"):
        ctx.zfp_compress(x, 0.0)
    with pytest.raises(szsel.SzselError, match="eb_abs"):
        ctx.zfp_compress(x, float("inf"))


# ---------------------------------------------------------------- SZ side

SZ_EXACT = ("bits", "values", "sse", "mse", "maxerr", "vr", "eb_abs", "unpredictable", "symbols",
            "code_bits", "bitrate", "psnr")


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("eb", [1e-2, 1e-4, 1e-6])
def test_sz_compression_matches_oracle(ctx, case, eb):
    label, make = case
    x = make()
    host = x.numpy()
    eb_abs = eb * float(host.max() - host.min())
    _note("step4 sz", label, eb)
    gpu, syms, dec = ctx.sz_compress(x.cuda(), eb_abs, symbols=True)
    orc, hist, osyms, odec = oracle.sz_compress(host, eb_abs)
    assert gpu["flags"] == 0
    for k in SZ_EXACT:
        assert gpu[k] == orc[k], "%s: gpu %r oracle %r" % (k, gpu[k], orc[k])
    assert abs(gpu["code_entropy"] - orc["code_entropy"]) <= 1e-9 * max(1.0, orc["code_entropy"])
    assert np.array_equal(syms.cpu().numpy().view(np.uint16), osyms)
    assert np.array_equal(dec.cpu().numpy().astype(np.float64), odec)
    assert gpu["maxerr"] <= eb_abs


def test_sz_full_size_field(ctx):
    """The 512^3 benchmark field (2^27 values): the round trip within the
    bound; the exact size always computed (no NO_HUFFMAN flag) and made of
    its parts, its code bits equal to the oracle's heap-built optimal code
    cost of the symbols' counts; and a 16^3 corner's symbols and values
    against the oracle on that corner (the corner's predictions only look
    backwards)."""
    field = synth.workload_turb512(device="cuda")
    vr = float(field.max() - field.min())
    for eb in (1e-2, 1e-4, 1e-6):
        gpu, syms, dec = ctx.sz_compress(field, eb * vr, symbols=True)
        _note("turb512 sz step4 eb", eb, gpu["bitrate"], gpu["psnr"], gpu["flags"], gpu["symbols"])
        assert gpu["maxerr"] <= eb * vr
        assert (dec.double() - field.double()).abs().max().item() == gpu["maxerr"]
        assert gpu["flags"] == 0
        assert gpu["bits"] == gpu["code_bits"] + 32 * gpu["unpredictable"] + 32 * gpu["symbols"]
        counts = torch.bincount(syms.reshape(-1).view(torch.int16).to(torch.int32) & 0xFFFF,
                                minlength=65536).cpu().numpy()
        assert int(counts.sum()) == field.numel() and int((counts > 0).sum()) == gpu["symbols"]
        assert gpu["code_bits"] == oracle.huffman_bits(counts)
        # whole-field SSE: the adjacent-pair tree of the squared errors in
        # field order (2^27 values, no padding), on the host
        v = (dec.double() - field.double()).cpu().numpy().reshape(-1)
        v = v * v
        while v.size > 1:
            v = v[0::2] + v[1::2]
        assert float(v[0]) == gpu["sse"]
        del v
        sub = field[:16, :16, :16].contiguous().cpu().numpy()
        _, _, osyms, odec = oracle.sz_compress(sub, eb * vr)
        assert np.array_equal(syms[:16, :16, :16].cpu().numpy().view(np.uint16), osyms)
        assert np.array_equal(dec[:16, :16, :16].cpu().numpy().astype(np.float64), odec)


def test_non_finite_fields_are_flagged(ctx):
    from paper_1806_08901_amd import szsel
    x = synth.spectral((24, 20), seed=91)
    x[3, 7] = float("nan")
    x[10, 2] = float("inf")
    for fn in (ctx.zfp_compress, ctx.sz_compress):
        res, _, _ = fn(x.cuda(), 1e-3, decoded=False)
        assert res["flags"] & szsel.FLAG_NONFINITE
