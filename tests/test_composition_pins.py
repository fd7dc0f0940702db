"""Hand-computed pins of two compositions the paper leaves to a reading.

* BR_sz (Section 5.1 Eq. 5 with the +0.5 offset of Section 6.2 and W raw
  bits per unpredictable point): a field whose quantization codes are known
  by construction, with the bit-rate written out by hand.
* The ZFP fixed-accuracy precision (external to the paper: emax - minexp +
  2(d + 1) coded planes, clamped to [0, W]): hand values on both clamps, and
  a two-sided check of the tolerance it buys -- every block within tau with
  the rule's planes, some block past tau with two planes fewer (three in
  3-D, where the guard of 2(d + 1) planes leaves the most slack).
"""
import math

import numpy as np
import pytest

import oracle

# 1-D field of 16 values (four 4-point blocks, all sampled).  The Lorenzo
# predictor in 1-D is the previous value (0 before the first), so with
# delta = 1 (eb_abs = 0.5, the SZ side's delta = 2 eb_abs) the code of each
# value is its difference from the previous one plus 32768:
#   8 differences of 0, 4 of 1, 2 of 2, and 2 jumps of 40000 >= 32768 that
#   cannot be quantized (code 0, the escape).
STEPS = [0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 40000, 40000, 0, 0, 0, 0]
FIELD = np.cumsum(STEPS).astype(np.float64)


@pytest.mark.parametrize("dtype,W,offset,want_br", [
    # H = 1/2 + 2/4 + 3/8 + 3/8 = 1.75 bits; escapes 2 x W bits over 16 values
    (np.float32, 32, 0.5, 1.75 + 0.5 + 4.0),    # 6.25
    (np.float64, 64, 0.25, 1.75 + 0.25 + 8.0),  # 10.0
    (np.float32, 32, 0.0, 5.75),
])
def test_sz_bitrate_composition_by_hand(dtype, W, offset, want_br):
    f = FIELD.astype(dtype)
    r, dump = oracle.run(oracle.OP_SZ, f, 0.5, oracle.EB_ABS, (1,), sz_offset=offset, dump=True, huffman=1)
    codes = list(dump["codes"])
    want_codes = [0 if s >= 32768 else 32768 + s for s in STEPS]
    assert codes == want_codes
    hist = dump["hist"]
    assert hist[32768] == 8 and hist[32769] == 4 and hist[32770] == 2 and hist[0] == 2
    assert hist.sum() == 16
    assert r["sz_delta"] == 1.0 and r["sz_unpredictable"] == 2
    assert r["sz_entropy"] == 1.75
    assert r["sz_bitrate"] == want_br
    # the optimal prefix code of counts {8, 4, 2, 2}: lengths 1, 2, 3, 3 = 28 bits
    assert r["sz_huffman_bits"] == 28
    assert r["sz_huffman_bitrate"] == 28 / 16 + 2 * W / 16
    assert r["sz_sse"] == 0.0 and r["sz_maxerr"] == 0.0


@pytest.mark.parametrize("emax,minexp,nd,W,want", [
    (0, -10, 1, 32, 14), (0, -10, 2, 32, 16), (0, -10, 3, 32, 18),
    (5, 5, 3, 32, 8), (5, 12, 3, 32, 1), (5, 13, 3, 32, 0), (5, 20, 1, 64, 0),
    (40, 0, 3, 32, 32), (40, 0, 3, 64, 48), (60, 0, 3, 64, 64), (-126, -149, 2, 32, 29),
    (1024, -1074, 1, 64, 64), (-1022, -1074, 3, 64, 60),
])
def test_precision_hand_values(emax, minexp, nd, W, want):
    assert oracle.precision(emax, minexp, nd, W) == want


def _blocks(nd, rng):
    size = 4 ** nd
    for trial in range(300):
        kind = trial % 3
        if kind == 0:
            x = rng.standard_normal(size)
        elif kind == 1:
            x = np.cumsum(rng.standard_normal(size))
        else:
            x = rng.standard_normal(size) * 10.0 ** rng.uniform(-3, 3)
        yield x


@pytest.mark.parametrize("nd", [1, 2, 3])
@pytest.mark.parametrize("dt", [oracle.F32, oracle.F64])
def test_precision_rule_is_tight_from_both_sides(nd, dt):
    rng = np.random.default_rng(40 + nd)
    W = 32 if dt == oracle.F32 else 64
    worst_rule, worst_fewer = 0.0, 0.0
    for x in _blocks(nd, rng):
        xv = x.astype(np.float32).astype(np.float64) if dt == oracle.F32 else x
        tau = 10.0 ** rng.uniform(-6, -1) * float(np.abs(xv).max())
        me = oracle.floor_log2(tau)
        _, xh, _, _, emax = oracle.zfp_block(xv, nd, dt, me)
        if oracle.precision(emax, me, nd, W) >= W:
            continue
        worst_rule = max(worst_rule, float(np.abs(xv - xh).max()) / tau)
        # fewer planes: the same block with the lowest coded plane raised
        _, xh2, _, _, _ = oracle.zfp_block(xv, nd, dt, me + (3 if nd == 3 else 2))
        worst_fewer = max(worst_fewer, float(np.abs(xv - xh2).max()) / tau)
    assert worst_rule <= 1.0
    assert worst_fewer > 1.0
