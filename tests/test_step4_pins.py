"""Pins of the oracle's Step 4 ZFP compressor (Section 3; Algorithm 1's ZFP branch):
the stream round trip, agreement with the estimator's exact bit count, the
edge padding of partial blocks, and an independent decoder of the stream
format.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1806_08901_amd import synth


def _fields():
    return [
        synth.gaussian_bumps((1030,), sigma_range=(3.0, 30.0), seed=71).numpy(),
        synth.spectral((70, 90), slope=-2.0, seed=72).numpy(),
        synth.spectral((37, 29, 43), slope=-2.0, seed=73).numpy(),
        synth.spectral((21, 34, 27), slope=-3.0, seed=74).numpy().astype(np.float64),
        synth.spiky_constant((52, 64), frac=0.02, seed=75).numpy(),
    ]


@pytest.mark.parametrize("case", range(5))
@pytest.mark.parametrize("eb", [1e-2, 1e-4, 1e-6])
def test_round_trip_within_the_bound(case, eb):
    x = _fields()[case]
    eb_abs = eb * float(x.max() - x.min())
    r, words, dec = oracle.zfp_compress(x, eb_abs)
    assert r["maxerr"] <= eb_abs
    assert np.max(np.abs(dec - x.astype(np.float64))) == r["maxerr"]
    assert r["bits"] <= 64 * words.size < r["bits"] + 64
    assert r["bitrate"] == r["bits"] / x.size


@pytest.mark.parametrize("shape,dtype", [((64,), np.float32), ((32, 48), np.float32),
                                         ((16, 20, 24), np.float64)])
def test_whole_blocks_match_the_estimator(shape, dtype):
    """Without partial blocks, the stream holds exactly the bits the
    estimator counts at stride 1, and decoding the stream gives the
    estimator's decoded error."""
    x = synth.spectral(shape, slope=-2.0, seed=76).numpy().astype(dtype)
    for eb in (1e-2, 1e-5):
        est, _ = oracle.run(oracle.OP_ZFP, x, eb, oracle.EB_REL, (1,) * len(shape))
        r, _, _ = oracle.zfp_compress(x, est["eb_abs"])
        assert r["bits"] == est["zfp_bits"]
        assert r["sse"] == est["zfp_sse"]
        assert r["maxerr"] == est["zfp_maxerr"]


@pytest.mark.parametrize("shape", [(5,), (6, 7), (5, 9, 6)])
def test_partial_blocks_repeat_the_edge(shape):
    """A ragged field codes like the field padded by edge repetition to whole
    blocks: same stream, same decoded values where the field is."""
    x = synth.spectral(shape, slope=-1.5, seed=77).numpy()
    padded = np.pad(x, [(0, (-n) % 4) for n in shape], mode="edge")
    eb_abs = 1e-4
    r1, w1, d1 = oracle.zfp_compress(x, eb_abs)
    r2, w2, d2 = oracle.zfp_compress(padded, eb_abs)
    assert r1["bits"] == r2["bits"] and np.array_equal(w1, w2)
    assert np.array_equal(d1, d2[tuple(slice(0, n) for n in shape)])


def test_zero_field_costs_one_bit_per_block():
    x = np.zeros((9, 10), np.float32)
    x[0, 0] = 1e-3  # a nonzero range; every other block is all zero
    r, words, dec = oracle.zfp_compress(x, 1.0)  # 2^-10 <= 1e-3 < 2^-9: no plane above 2^0 - 2(d+1)
    assert r["bits"] == oracle.zfp_num_blocks(x.shape)
    assert not dec.any() and r["maxerr"] == np.float64(np.float32(1e-3))


def _decode_stream(words, shape, dtype, eb_abs):
    """Decoder written from the stream format alone (not the oracle's)."""
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")
    nd = len(shape)
    W = 32 if dtype == np.float32 else 64
    E = 8 if W == 32 else 11
    P = W - 2
    bias = (1 << (E - 1)) - 1
    size = 4 ** nd
    minexp = math.frexp(eb_abs)[1] - 1
    perm = oracle.reorder_table(nd)
    nb = [(n + 3) // 4 for n in shape]
    out = np.zeros([4 * b for b in nb], np.float64)
    pos = 0

    def rd():
        nonlocal pos
        b = int(bits[pos])
        pos += 1
        return b

    for jb in range(int(np.prod(nb))):
        bo = np.unravel_index(jb, nb)
        xh = np.zeros(size)
        if rd():
            e = sum(rd() << b for b in range(E))
            emax = e - bias
            prec = max(0, min(W, emax - minexp + 2 * (nd + 1)))
            u = [0] * size
            n = 0
            for k in range(W - 1, W - prec - 1, -1):
                for i in range(n):
                    u[i] |= rd() << k
                p = n
                while p < size and rd():
                    while p < size - 1 and not rd():
                        p += 1
                    u[p] |= 1 << k
                    p += 1
                    n = p
            mask = int("AA" * (W // 8), 16)
            c = np.zeros(size, np.int64)
            for r_ in range(size):
                v = ((u[r_] ^ mask) - mask) & ((1 << W) - 1)
                c[perm[r_]] = v - (1 << W) if v >> (W - 1) else v
            d = oracle.inv_xform(c, nd, W)
            xh = np.array([math.ldexp(float(v), emax - P) for v in d])
            if W == 32:
                xh = xh.astype(np.float32).astype(np.float64)
        sl = tuple(slice(4 * b, 4 * b + 4) for b in bo)
        out[sl] = xh.reshape([4] * nd)
    return out[tuple(slice(0, n) for n in shape)]


@pytest.mark.parametrize("shape,dtype", [((13, 10), np.float32), ((6, 5, 7), np.float64), ((23,), np.float32)])
def test_independent_decoder_reads_the_stream(shape, dtype):
    x = synth.spectral(shape, slope=-2.0, seed=78).numpy().astype(dtype)
    eb_abs = 3e-4
    r, words, dec = oracle.zfp_compress(x, eb_abs)
    assert np.array_equal(_decode_stream(words, shape, dtype, eb_abs), dec)


# ---------------------------------------------------------------- SZ side


def _sz_decode(symbols, raw, shape, eb_abs, dtype):
    """Sequential decoder written from the format: each value's q is its
    symbol - 32768 plus the integer Lorenzo sum of the decoded neighbours'
    q (0 outside); an escape's value is stored raw and its q recomputed."""
    nd = len(shape)
    delta = 2.0 * eb_abs
    inv = 1.0 / delta
    q = np.zeros(shape, np.int64)
    out = np.zeros(shape, np.float64)
    for idx in np.ndindex(*shape):
        pred = 0
        for S in range(1, 1 << nd):
            nb = tuple(i - ((S >> k) & 1) for k, i in enumerate(idx))
            if min(nb) < 0:
                continue
            pred += int(q[nb]) if bin(S).count("1") % 2 else -int(q[nb])
        s = int(symbols[idx])
        if s == 0:
            x = float(raw[idx])
            t = abs(x) * inv + 0.5
            qq = int(math.floor(t)) if t < 2.0 ** 50 else 0
            q[idx] = -qq if x < 0 else qq
            out[idx] = x
        else:
            q[idx] = s - 32768 + pred
            out[idx] = float(dtype(float(q[idx]) * delta))
    return out


@pytest.mark.parametrize("case", range(5))
@pytest.mark.parametrize("eb", [1e-2, 1e-4, 1e-6])
def test_sz_round_trip_and_size(case, eb):
    x = _fields()[case]
    eb_abs = eb * float(x.max() - x.min())
    r, hist, syms, dec = oracle.sz_compress(x, eb_abs)
    assert r["maxerr"] <= eb_abs
    assert int(hist.sum()) == x.size and int(hist[0]) == r["unpredictable"]
    assert r["symbols"] == int((hist > 0).sum())
    assert r["code_bits"] == oracle.huffman_bits(hist)
    W = 32 if x.dtype == np.float32 else 64
    assert r["bits"] == r["code_bits"] + W * r["unpredictable"] + 32 * r["symbols"]
    assert abs(r["code_entropy"] - oracle.entropy(hist, x.size)) <= 1e-12 * max(1.0, r["code_entropy"])
    esc = syms == 0
    assert np.array_equal(dec[esc], x[esc].astype(np.float64))


@pytest.mark.parametrize("shape,dtype", [((37,), np.float32), ((9, 11), np.float64), ((5, 6, 7), np.float32)])
def test_sz_independent_decoder(shape, dtype):
    x = synth.spectral(shape, slope=-2.0, seed=79).numpy().astype(dtype)
    for eb in (1e-2, 1e-5):
        eb_abs = eb * float(x.max() - x.min())
        r, hist, syms, dec = oracle.sz_compress(x, eb_abs)
        assert np.array_equal(_sz_decode(syms, x, shape, eb_abs, dtype), dec)


def test_sz_bilinear_field_predicts_exactly():
    """Values on the quantization grid that are bilinear in the indices:
    the 2-D Lorenzo predictor is exact away from the first row and column."""
    eb = 0.5
    i, j = np.meshgrid(np.arange(30), np.arange(40), indexing="ij")
    x = (2 * eb * (3 * i + 5 * j + 7)).astype(np.float64)
    r, hist, syms, dec = oracle.sz_compress(x, eb)
    assert np.all(syms[1:, 1:] == 32768)
    assert r["sse"] == 0.0 and r["unpredictable"] == 0
