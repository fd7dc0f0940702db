"""The oracle against the stored fixtures under tests/golden/."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1806_08901_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_closed_form_eq11():
    x = synth.spectral((16, 16, 16), seed=21).numpy()
    for eb, psnr in _load("closed_forms.json")["eq11_psnr_sz"]["cases"]:
        r, _ = oracle.run(oracle.OP_SZ, x, eb, oracle.EB_REL, (1, 1, 1))
        assert math.isclose(r["sz_psnr_model"], psnr, rel_tol=1e-12)


def test_closed_form_equal_probability_bitrate():
    h = np.zeros(65536, np.uint32)
    for k, bits in _load("closed_forms.json")["equal_probability_bitrate"]["cases"]:
        h[:] = 0
        h[:k] = 5
        assert math.isclose(oracle.entropy(h), bits, rel_tol=1e-13)


def test_closed_form_uniform_mse():
    # A field whose Lorenzo residuals are spread uniformly over many bins:
    # the measured SZ MSE approaches delta^2 / 12 (Eq. 7 with equal bins).
    rng = np.random.default_rng(22)
    x = np.cumsum(rng.uniform(-1, 1, 4096 * 4)).astype(np.float64)
    for delta, mse in _load("closed_forms.json")["eq7_uniform_mse"]["cases"]:
        r, _ = oracle.run(oracle.OP_SZ, x, delta / 2, oracle.EB_ABS, (1,))
        assert r["sz_delta"] == delta
        assert abs(r["sz_mse"] / mse - 1.0) < 0.05


def test_oracle_regression_fixture():
    import importlib.util
    spec = importlib.util.spec_from_file_location("mog", os.path.join(GOLDEN, "make_oracle_golden.py"))
    mog = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mog)
    makers = {name: (make, eb, stride) for name, make, eb, stride in mog.CASES}
    fields = {}
    for rec in _load("oracle_small.json"):
        make, eb, stride = makers[rec["case"]]
        if rec["case"] not in fields:
            fields[rec["case"]] = make().numpy()
        r, _ = oracle.run(rec["op"], fields[rec["case"]], rec["eb_rel"], oracle.EB_REL, tuple(rec["stride"]))
        for k, v in rec["result"].items():
            got = repr(r[k]) if isinstance(r[k], float) else r[k]
            assert got == v, (rec["case"], rec["op"], k)
