"""The autotuner's schedules persist across processes through the file named
by SZSEL_TUNE_CACHE (needs a GPU).  Two fresh processes run the same
autotuned batch: the first tunes and appends one line, the second finds the
schedule in the file and appends nothing; malformed lines and lines of
another build are skipped.  Results are the same in both and equal the
fixed schedule's."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import json, sys
sys.path.insert(0, %r)
import torch
from paper_1806_08901_amd import synth, szsel
f3a = synth.spectral((40, 48, 52), slope=-3.0, kmax=12.0, seed=71).cuda()
f3b = synth.spectral((36, 44, 60), slope=-2.5, kmax=12.0, seed=72, dtype=torch.float64).cuda()
f2 = synth.spectral((64, 72), slope=-2.0, kmax=20.0, seed=73).cuda()
items = [(f3a, 1e-3, szsel.EB_REL, (1, 1, 1), szsel.OP_SELECT),
         (f3b, 1e-4, szsel.EB_REL, (2, 1, 1), szsel.OP_SELECT),
         (f2, 1e-2, szsel.EB_REL, (2, 1), szsel.OP_SELECT)]
ctx = szsel.Context(0)
fixed = ctx.select_batch(items)
ctx.set_option(szsel.OPT_AUTOTUNE, 1)
tuned = ctx.select_batch(items)
print(json.dumps({"same": tuned == fixed, "bits": [r["zfp_bits"] for r in tuned],
                  "choice": [r["choice"] for r in tuned]}))
""" % ROOT


def _run(cache):
    env = dict(os.environ)
    env["SZSEL_TUNE_CACHE"] = cache
    print("tune-cache subprocess, cache", cache, flush=True)
    out = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True,
                         timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_tuned_schedule_is_reused_by_a_new_process(tmp_path):
    cache = str(tmp_path / "tune.jsonl")
    junk = ['not json at all\n',
            '{"build":"another build","arch":"gfx950","key":[3],"tune":{"sz_wgs_q":8}}\n']
    with open(cache, "w") as f:
        f.writelines(junk)
    first = _run(cache)
    lines = open(cache).read().splitlines()
    assert lines[:2] == [j.rstrip("\n") for j in junk]
    assert len(lines) == 3, lines
    entry = json.loads(lines[2])
    assert entry["arch"].startswith("gfx") and len(entry["key"]) > 1
    assert set(entry["tune"]) == {"sz_wgs_q", "zfp_chunk", "zfp_waves", "range_wgs_q", "range_grid", "groups",
                                 "lanes", "ovf_slice", "share"}
    second = _run(cache)
    assert open(cache).read().splitlines() == lines  # found, not tuned again
    assert first["same"] and second["same"]
    assert first["bits"] == second["bits"] and first["choice"] == second["choice"]
