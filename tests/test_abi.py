"""The C-ABI library loads and exports every declared symbol (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1806_08901_amd import szsel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(szsel_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = szsel.load_library()
    declared = _declared()
    assert declared, "no declarations found"
    assert declared == set(szsel.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_result_layout_matches_header():
    # 2 x u32, 4 doubles, 2 x i32, 6 doubles, 4 u64, 10 doubles, 2 u64, 1 double
    assert ctypes.sizeof(szsel.Result) == 8 + 32 + 8 + 48 + 32 + 80 + 16 + 8 + 16 + 16
    assert ctypes.sizeof(szsel.Request) == 8 + 24 + 8 + 8 + 8 + 12 + 4


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every field offset of the binding's structures equals the one a C
    compiler gives for include/szsel.h."""
    import os
    import subprocess
    structs = {"szsel_result": szsel.Result, "szsel_request": szsel.Request,
               "szsel_compressed": szsel.Compressed, "szsel_debug": szsel.Debug}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "szsel.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("shape,rate,want", [
    ((512, 512, 512), 0.05, (5, 4, 1)),
    ((1800, 3600), 0.05, (20, 1)),
    ((100, 500, 500), 0.05, None),
    ((64, 64, 64), 1.0, (1, 1, 1)),
])
def test_stride_for_rate(shape, rate, want):
    st = szsel.stride_for_rate(rate, shape)
    assert st[-1] == 1
    if want is not None:
        assert st == want
    nb = [n // 4 for n in shape]
    frac = 1.0
    for b, s in zip(nb, st):
        frac *= -(-b // s) / b
    assert 0.5 * rate <= frac <= 2.0 * rate


def test_stride_for_rate_rejects_bad_input():
    with pytest.raises(szsel.SzselError):
        szsel.stride_for_rate(0.0, (64, 64))
    with pytest.raises(szsel.SzselError):
        szsel.stride_for_rate(0.05, (2, 64))


def test_no_gpu_means_loud_failure():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(szsel.SzselError):
        szsel.Context(0)


def test_oracle_struct_layouts_match_the_c_compiler(tmp_path):
    """The oracle's ctypes structures against its C header."""
    import os
    import subprocess
    import oracle
    structs = {"orc_result": oracle.Result, "orc_dump": oracle.Dump, "orc_step4": oracle.Step4}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "szsel_oracle.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "olayout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "olayout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
