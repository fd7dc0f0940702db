"""szsel_select_noalloc (the entry point that allocates nothing) against
szsel_select and the oracle, through the C ABI (needs a GPU)."""
import sys

import pytest
import torch

import oracle
from paper_1806_08901_amd import synth
from tests.gpu_common import assert_matches_oracle

pytestmark = pytest.mark.gpu


def _note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a: dict, b: dict, label):
    bad = [k for k in a if a[k] != b[k] and not (a[k] != a[k] and b[k] != b[k])]
    assert not bad, "%s: %s" % (label, ", ".join("%s %r vs %r" % (k, a[k], b[k]) for k in bad))


@pytest.fixture(scope="module")
def ctx():
    from paper_1806_08901_amd import szsel
    c = szsel.Context(0)
    yield c
    c.close()


# (label, field maker, eb_rel, stride): the first call is the larger one
CASES = [
    ("bumps64_f32_stride1", lambda: synth.gaussian_bumps((64, 64, 64), seed=11), 1e-4, (1, 1, 1)),
    ("bumps24x20x36_f32", lambda: synth.gaussian_bumps((24, 20, 36), seed=12), 1e-3, (2, 1, 1)),
    ("spectral_2d_f64", lambda: synth.spectral((96, 130), slope=-2.5, kmax=24.0, seed=13,
                                                dtype=torch.float64), 1e-5, (2, 1)),
    ("spectral_1d_f32", lambda: synth.spectral((1000,), slope=-2.0, kmax=40.0, seed=14), 1e-2, (1,)),
]


def test_noalloc_matches_select_and_oracle_twice_in_a_row(ctx):
    """Two calls in a row (the second on a smaller field, which leaves the
    first call's contents in the shared array), each equal to szsel_select
    bit for bit and to the oracle."""
    fields = [(lab, mk(), eb, st) for lab, mk, eb, st in CASES]
    for lab, x, eb, st in fields:
        _note("noalloc case", lab, tuple(x.shape), x.dtype, eb, st)
        xd = x.cuda()
        ref = ctx.select(xd, eb, stride=st)
        got = ctx.select_noalloc(xd, eb, stride=st)
        _same(got, ref, lab)
        orc, _ = oracle.select(x.numpy(), eb, stride=st)
        assert_matches_oracle(got, orc, lab)


def test_noalloc_queued_calls_on_one_stream(ctx):
    """Calls queued on one stream with no host synchronisation between them
    (the stream orders them on the shared array), the second smaller."""
    from paper_1806_08901_amd import szsel
    big = synth.gaussian_bumps((48, 64, 40), seed=21).cuda()
    small = synth.spectral((40, 36, 44), slope=-3.0, kmax=12.0, seed=22).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ref_big = ctx.select(big, 1e-4, stride=(1, 2, 1), stream=s)
        ref_small = ctx.select(small, 1e-3, stride=(1, 1, 1), stream=s)
    import ctypes as C
    size = C.sizeof(szsel.Result)
    pinned = torch.empty(2 * size, dtype=torch.uint8, pin_memory=True)
    res = (szsel.Result * 2).from_address(pinned.data_ptr())
    for k, (x, eb, st) in enumerate([(big, 1e-4, (1, 2, 1)), (small, 1e-3, (1, 1, 1))]):
        dims = (C.c_int64 * 3)(*x.shape)
        stv = (C.c_int32 * 3)(*st)
        out = C.cast(C.c_void_p(pinned.data_ptr() + k * size), C.POINTER(szsel.Result))
        rc = ctx.lib.szsel_select_noalloc(ctx.h, C.c_void_p(x.data_ptr()), dims, 3, szsel.F32, eb,
                                          szsel.EB_REL, stv, out, C.c_void_p(s.cuda_stream))
        assert rc == 0, ctx.lib.szsel_last_error(ctx.h).decode()
    s.synchronize()
    _same(szsel._as_dict(res[0]), ref_big, "queued big")
    _same(szsel._as_dict(res[1]), ref_small, "queued small")


def test_noalloc_rejects_a_request_beyond_the_array(ctx):
    """Every block of a 384^3 field: 2 bytes per sampled value exceed the
    64 MiB array, so the call returns SZSEL_ENOMEM and names the sizes; the
    next call still works."""
    from paper_1806_08901_amd import szsel
    x = torch.zeros((384, 384, 384), dtype=torch.float32, device="cuda")
    with pytest.raises(szsel.SzselError) as ei:
        ctx.select_noalloc(x, 1e-3, stride=(1, 1, 1))
    assert "(-3)" in str(ei.value) and "szsel_select_noalloc has 67108864" in str(ei.value)
    del x
    y = synth.gaussian_bumps((32, 32, 32), seed=31)
    got = ctx.select_noalloc(y.cuda(), 1e-4, stride=(1, 1, 1))
    orc, _ = oracle.select(y.numpy(), 1e-4, stride=(1, 1, 1))
    assert_matches_oracle(got, orc, "after ENOMEM")
