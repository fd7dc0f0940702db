"""Host-side helpers of bench.py (no GPU): the algorithmic bytes each pass
must move, which the roofline figures divide by, and the digest that tells
whether recorded counters still describe the kernels."""
import os
import shutil

import bench


def test_request_bytes_of_the_512_cube():
    """512^3 binary32, stride (5, 4, 1): the range pass reads every value,
    the ZFP pass the 106,496 sampled blocks of 64 values, the SZ pass the
    sampled values and their Lorenzo predecessors (each sampled block grown
    by one cell toward the origin, overlaps counted once), the entropy pass
    the 65,536 bins."""
    b = bench.request_bytes((512, 512, 512), (5, 4, 1), 4)
    assert b["range"] == 512 ** 3 * 4
    assert b["zfp"] == 26 * 32 * 128 * 64 * 4 == 27262976
    # along an axis with stride s, the blocks j = 0, s, 2s, ... cover
    # [4js - 1, 4js + 3]: 5 cells each (4 for the first), and unit stride
    # covers the whole axis
    z = 26 * 5 - 1
    y = 32 * 5 - 1
    x = 512
    assert b["sz"] == z * y * x * 4 == 42006528
    assert b["ent"] == 65536 * 4


def test_request_bytes_of_a_ragged_2d_field():
    """1800 x 3600 binary32 with stride (20, 1): 23 of 450 block rows."""
    b = bench.request_bytes((1800, 3600), (20, 1), 4)
    assert b["zfp"] == 23 * 900 * 16 * 4
    assert b["sz"] == (23 * 5 - 1) * 3600 * 4


def _copy_sources(tmp_path):
    src = os.path.join(bench.ROOT, "paper_1806_08901_amd", "csrc")
    dst = tmp_path / "paper_1806_08901_amd" / "csrc"
    shutil.copytree(src, dst)
    return str(tmp_path), dst


def test_source_digest_ignores_comments_but_not_code(tmp_path):
    root, dst = _copy_sources(tmp_path)
    base = bench.source_digest(root)
    assert base == bench.source_digest()
    p = dst / "estimator.hpp"
    text = p.read_text()
    p.write_text("// an added comment line\n" + text.replace("\n", "\n  ", 1) + "\n/* and a block comment */\n")
    assert bench.source_digest(root) == base
    p.write_text(text.replace("kHistWin = 4096", "kHistWin = 2048", 1))
    assert bench.source_digest(root) != base


def test_recorded_traffic_missing_profile():
    assert bench.recorded_traffic("no_such_profile.md", "szsel::kb_range") is None
