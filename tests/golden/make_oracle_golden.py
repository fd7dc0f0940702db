"""Writes oracle_small.json: oracle results on small seeded fields.

Calls only the oracle (and the seeded generators).  The stored values guard
against unintended changes to the oracle's arithmetic; a deliberate change
regenerates this file and names, in its commit message, the passage of the
paper (or its reading) that justifies it.

    python tests/golden/make_oracle_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1806_08901_amd import synth  # noqa: E402

CASES = [
    ("bumps 24x20x28 f32", lambda: synth.gaussian_bumps((24, 20, 28), seed=11), 1e-4, (1, 1, 1)),
    ("spectral 32^3 f32", lambda: synth.spectral((32, 32, 32), seed=12), 1e-3, (2, 2, 1)),
    ("spectral 40x52 f64", lambda: synth.spectral((40, 52), slope=-2.5, seed=13,
                                                  dtype=synth.torch.float64), 1e-5, (3, 1)),
    ("spiky 36x44 f32", lambda: synth.spiky_constant((36, 44), frac=0.01, seed=14), 1e-2, (1, 1)),
    ("bumps 64 f32 1d", lambda: synth.gaussian_bumps((203,), sigma_range=(3.0, 20.0), seed=15), 1e-6, (1,)),
]


def main():
    out = []
    for name, make, eb, stride in CASES:
        x = make().numpy()
        for op in (oracle.OP_SZ, oracle.OP_ZFP, oracle.OP_SELECT, oracle.OP_FIXED_EB):
            r, _ = oracle.run(op, x, eb, oracle.EB_REL, stride)
            out.append({"case": name, "op": op, "eb_rel": eb, "stride": list(stride),
                        "result": {k: (repr(v) if isinstance(v, float) else v) for k, v in r.items()}})
    with open(os.path.join(HERE, "oracle_small.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
