"""The GPU's way of counting ZFP coder bits, checked on the CPU against the
oracle's literal bit emission.

The HIP kernels do not run the group-testing coder; they count its output
from per-coefficient quantities: with msb_j the highest set bit of the j-th
coefficient in coding order (-1 for zero), M_j the maximum of msb over
positions >= j, and kmin the lowest coded plane, the coder emits

    sum_j max(0, M_j - kmin + 1) + W - max(kmin, msb_last + 1)
    + #{j : u_j != 0 and msb_j == M_j >= kmin} - [msb_last >= kmin]

bits.  This test restates that count in Python and compares it with the
number of bits the oracle emits, over random and structured inputs.
"""
import random

import oracle


def closed_form(u, W, kmin):
    S = len(u)
    msb = [int(v).bit_length() - 1 for v in u]
    M = [max(msb[j:]) for j in range(S)]
    verbatim = sum(max(0, M[j] - kmin + 1) for j in range(S))
    empty_tests = W - max(kmin, msb[-1] + 1)
    found = sum(1 for j in range(S) if u[j] != 0 and msb[j] == M[j] and msb[j] >= kmin)
    implied = 1 if msb[-1] >= kmin else 0
    return verbatim + empty_tests + found - implied


def test_closed_form_count_equals_emitted_bits():
    rnd = random.Random(5)
    for S in (4, 16, 64):
        for W in (32, 64):
            for trial in range(600):
                kind = trial % 4
                if kind == 0:
                    u = [rnd.getrandbits(W) for _ in range(S)]
                elif kind == 1:
                    tops = sorted((rnd.randrange(W) for _ in range(S)), reverse=True)
                    u = [rnd.getrandbits(k + 1) for k in tops]
                elif kind == 2:
                    u = [0] * S
                    for _ in range(rnd.randrange(4)):
                        u[rnd.randrange(S)] = rnd.getrandbits(W)
                else:
                    u = [rnd.randrange(4) for _ in range(S)] if trial % 8 != 3 else [0] * S
                prec = rnd.randrange(1, W + 1)
                assert closed_form(u, W, W - prec) == oracle.encode_planes(u, W, prec)
