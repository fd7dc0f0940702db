"""Admission bookkeeping of the serving engine (szsel_server_*), without a
device: reservations are first fit over 256-byte granules, freed ranges
coalesce, a full pool answers "busy" and an oversized snapshot "no memory"."""
import pytest

from paper_1806_08901_amd import szsel


@pytest.fixture
def server():
    try:
        szsel.load_library()
    except szsel.SzselError as e:
        pytest.skip(str(e))
    s = szsel.Server(ctx=None, pool_bytes=1 << 20)
    yield s
    s.close()


def test_first_fit_granules_and_busy(server):
    a = server.reserve(1000)        # rounds up to 1024
    b = server.reserve(256)
    c = server.reserve(1)           # one granule
    assert a[0] == 0 and b[0] == 1024 and c[0] == 1280
    st = server.stats()
    assert st["pool_reserved"] == 1024 + 256 + 256 and st["pool_bytes"] == 1 << 20
    rest = server.reserve((1 << 20) - 1536)
    assert rest is not None and rest[0] == 1536
    assert server.reserve(256) is None          # full: busy, not an error
    server.cancel(b[1])
    assert server.reserve(512) is None          # only 256 bytes free
    d = server.reserve(200)
    assert d[0] == 1024                         # the freed granule is reused


def test_release_coalesces_neighbours(server):
    parts = [server.reserve(4096) for _ in range(8)]
    for k in (1, 3, 2):                         # free three adjacent ranges out of order
        server.cancel(parts[k][1])
    assert server.stats()["largest_free"] >= 3 * 4096
    big = server.reserve(3 * 4096)
    assert big[0] == 4096                       # one coalesced range at the first hole


def test_oversized_snapshot_and_bad_cancel(server):
    with pytest.raises(szsel.SzselError, match="larger than the pool"):
        server.reserve((1 << 20) + 1)
    with pytest.raises(szsel.SzselError):
        server.cancel(12345)
