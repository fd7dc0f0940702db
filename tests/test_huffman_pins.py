"""Pins of the oracle's exact Huffman cost (the entropy-coding stage whose
cost the +0.5 bits/value offset stands in for).  The minimum of sum h_i L_i
over prefix codes is unique; it is checked against an exhaustive search over
every binary merge tree, closed forms, and the entropy bound."""
import itertools
import math
import random

import numpy as np
import pytest

import oracle


def brute_force(weights):
    """Minimum over all full binary trees: cost(S) = min over pairs of
    (a + b) + cost(S - {a, b} + {a + b})."""
    memo = {}

    def best(ws):
        if len(ws) <= 1:
            return 0
        key = tuple(sorted(ws))
        if key in memo:
            return memo[key]
        m = None
        for i, j in itertools.combinations(range(len(ws)), 2):
            rest = [w for k, w in enumerate(ws) if k not in (i, j)] + [ws[i] + ws[j]]
            c = ws[i] + ws[j] + best(rest)
            m = c if m is None else min(m, c)
        memo[key] = m
        return m

    return best(list(weights))


def test_exhaustive_small_alphabets():
    rng = random.Random(7)
    for _ in range(300):
        n = rng.randint(2, 6)
        w = [rng.randint(1, 40) for _ in range(n)]
        hist = np.zeros(65536, np.uint32)
        pos = rng.sample(range(65536), n)
        hist[pos] = w
        assert oracle.huffman_bits(hist) == brute_force(w), w


@pytest.mark.parametrize("k", [1, 2, 5, 10])
def test_equal_counts_cost_log2_of_the_alphabet(k):
    hist = np.zeros(65536, np.uint32)
    hist[100:100 + 2 ** k] = 7
    assert oracle.huffman_bits(hist) == 7 * 2 ** k * k


def test_one_two_and_no_symbols():
    hist = np.zeros(65536, np.uint32)
    assert oracle.huffman_bits(hist) == 0
    hist[5] = 9
    assert oracle.huffman_bits(hist) == 9          # one symbol: 1 bit each
    hist[70000 % 65536] = 4
    assert oracle.huffman_bits(hist) == 13         # two symbols: 1 bit each


def test_within_one_bit_of_the_entropy():
    rng = np.random.default_rng(11)
    for _ in range(20):
        hist = np.zeros(65536, np.uint32)
        m = int(rng.integers(3, 3000))
        hist[rng.choice(65536, m, replace=False)] = rng.geometric(0.01, m).astype(np.uint32)
        n = int(hist.sum())
        p = hist[hist > 0] / n
        H = float(-(p * np.log2(p)).sum())
        bits = oracle.huffman_bits(hist)
        assert n * H <= bits + 1e-6 * n
        assert bits < n * (H + 1)


def test_pipeline_reports_the_cost_of_its_histogram():
    from paper_1806_08901_amd import synth
    x = synth.spectral((24, 28, 32), slope=-2.0, seed=90).numpy()
    r, d = oracle.run(oracle.OP_SELECT, x, 1e-4, oracle.EB_REL, (1, 1, 1), dump=True, huffman=1)
    assert r["sz_huffman_bits"] == oracle.huffman_bits(d["hist"])
    n = r["sz_values"]
    assert r["sz_huffman_bitrate"] == r["sz_huffman_bits"] / n + r["sz_unpredictable"] * 32 / n
    # Huffman costs at least the entropy and less than entropy + 1 bit
    assert r["sz_entropy"] * n <= r["sz_huffman_bits"] * (1 + 1e-12)
    assert r["sz_huffman_bits"] < (r["sz_entropy"] + 1) * n
    # the estimate without Huffman leaves the fields at zero
    r0, _ = oracle.run(oracle.OP_SELECT, x, 1e-4, oracle.EB_REL, (1, 1, 1))
    assert r0["sz_huffman_bits"] == 0 and r0["choice"] == r["choice"]


def test_selection_with_the_huffman_bitrate():
    from paper_1806_08901_amd import synth
    x = synth.spectral((24, 28, 32), slope=-2.0, seed=91).numpy()
    for eb in (1e-2, 1e-4, 1e-6):
        r, _ = oracle.run(oracle.OP_SELECT, x, eb, oracle.EB_REL, (1, 1, 1), huffman=2)
        expect = 0 if r["sz_huffman_bitrate"] < r["zfp_bitrate"] else 1
        assert r["choice"] == expect
