"""The C oracle against an independent pure-Python brute force of the whole
estimator (tests/brute), on tiny fields: 1-3 D, binary32 and binary64, every
op, strides up to 3, ragged extents, relative and absolute bounds, and the
exact Huffman cost.  Every result must agree bit for bit, including the
values derived with log2/log10 (both sides call the same C library).
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1806_08901_amd import synth
from tests.brute import pipeline as brute

OPS = (oracle.OP_SZ, oracle.OP_ZFP, oracle.OP_SELECT, oracle.OP_FIXED_EB)


def field_of(kind, shape, seed, dtype):
    if kind == "bumps":
        f = synth.gaussian_bumps(shape, nbumps=4, sigma_range=(1.5, 4.0), noise=1e-3, seed=seed).numpy()
    elif kind == "spectral":
        f = synth.spectral(shape, slope=-2.0, kmax=min(shape) / 2.0, noise=0.05, seed=seed).numpy()
    else:  # integers with jumps: escapes and exact reconstructions
        rng = np.random.default_rng(seed)
        f = np.cumsum(rng.integers(-3, 4, size=shape), axis=-1).astype(np.float64)
        f.reshape(-1)[rng.integers(0, f.size, 3)] += 1e6
    return np.ascontiguousarray(f.astype(dtype))


CASES = [
    # (kind, shape, stride, dtype, eb, eb_mode)
    ("bumps", (16,), (1,), np.float32, 1e-3, oracle.EB_REL),
    ("jumps", (67,), (3,), np.float64, 0.5, oracle.EB_ABS),
    ("spectral", (16, 16), (1, 1), np.float32, 1e-4, oracle.EB_REL),
    ("bumps", (13, 18), (2, 1), np.float64, 1e-2, oracle.EB_REL),
    ("jumps", (12, 16), (1, 3), np.float32, 2.0, oracle.EB_ABS),
    ("bumps", (8, 8, 8), (1, 1, 1), np.float32, 1e-4, oracle.EB_REL),
    ("spectral", (9, 14, 17), (2, 3, 1), np.float64, 1e-3, oracle.EB_REL),
    ("bumps", (16, 16, 16), (3, 2, 1), np.float32, 1e-2, oracle.EB_REL),
    ("spectral", (12, 12, 16), (1, 2, 3), np.float32, 1e-6, oracle.EB_REL),
]


def compare(got, want, label):
    bad = [k for k in want if not (got[k] == want[k] or (got[k] != got[k] and want[k] != want[k]))]
    assert not bad, label + "\n" + "\n".join("%s: brute %r oracle %r" % (k, got[k], want[k]) for k in bad)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_oracle_equals_brute_force(case):
    kind, shape, stride, dtype, eb, mode = CASES[case]
    f = field_of(kind, shape, 100 + case, dtype)
    for op in OPS:
        want, _ = oracle.run(op, f, eb, mode, stride, huffman=1)
        got = brute.run(op, f, eb, mode, stride, huffman=1)
        compare(got, want, "%s %s %s op %d" % (kind, shape, stride, op))


def test_oracle_equals_brute_force_options_and_degenerate_fields():
    f = field_of("bumps", (8, 12), 7, np.float32)
    for off in (0.0, 0.25, 1.5):  # the Section 6.2 offset is an option
        want, _ = oracle.run(oracle.OP_SELECT, f, 1e-3, oracle.EB_REL, (1, 1), sz_offset=off, huffman=2)
        compare(brute.run(oracle.OP_SELECT, f, 1e-3, oracle.EB_REL, (1, 1), sz_offset=off, huffman=2), want,
                "offset %g" % off)
    degenerate = [np.full((8, 8), 3.0, np.float32),               # constant
                  np.ones((3, 9), np.float64),                     # no full block (and constant)
                  np.arange(27, dtype=np.float64).reshape(3, 9),   # no full block
                  np.zeros((8, 8, 8), np.float32),                 # all zero
                  np.where(np.arange(64) % 7 == 0, 1.0, 0.0).reshape(4, 16).astype(np.float32)]
    bad = np.ones((8, 8), np.float32)
    bad[2, 3] = np.nan
    degenerate.append(bad)
    for f, op in itertools.product(degenerate, OPS):
        want, _ = oracle.run(op, f, 1e-2, oracle.EB_REL, None)
        compare(brute.run(op, f, 1e-2, oracle.EB_REL, None), want, "degenerate %s op %d" % (f.shape, op))
    # an absolute bound at the binary32 subnormal range and one far above VR
    f = field_of("spectral", (8, 8, 8), 9, np.float32) * np.float32(1e-36)
    for eb in (1e-44, 1e-30):
        want, _ = oracle.run(oracle.OP_SELECT, f, eb, oracle.EB_ABS, None)
        compare(brute.run(oracle.OP_SELECT, f, eb, oracle.EB_ABS, None), want, "tiny eb %g" % eb)
