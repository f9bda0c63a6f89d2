"""Device prefix scans (collected first: every compaction of the restructure
and the adjacency build relies on them) against host scans of the same
pseudo-random inputs, across tile boundaries (8192 elements per tile), ragged
tails, and look-back spans of more than one step (256 tiles per step)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1608_07411_amd import otf

    c = otf.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n", [0, 1, 31, 8191, 8192, 8193, 3 * 8192 + 77, (1 << 20) + 37, 256 * 8192 + 5,
                               5_000_003, 12_921_469])
def test_scans_match_host(ctx, n):
    print(f"selftest_scan n={n}", flush=True)
    assert ctx.selftest_scan(n, seed=n) == 0


def test_scans_repeat(ctx):
    """Many scans in a row reuse the epoch-tagged tile states."""
    for k in range(20):
        assert ctx.selftest_scan(300_000 + 8192 * k, seed=1000 + k) == 0
