"""wallace_fill_static (the fill whose per-call scratch is the library's
static device array) against wallace_fill on the same generators.

Two generators with the same seed and options: one is filled through
wallace_fill (scratch in its workspace), the other through
wallace_fill_static. Two calls in a row, the second smaller, must give the
same output bit for bit, and leave the same sum of squares, pass count and
pool. The cases use each kind of scratch: a streamed pool's partial sums
(fused n = 4 pass, two-launch n = 16 pass), the sum-of-squares tree of a
workspace check, and of restart refills on a pool-resident generator.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1004_3114_amd import wallace as W  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    # (n, N, options, first count, second count)
    (4, 1 << 15, {}, 3 * 4 * (1 << 15) + 1000, 4 * (1 << 15) + 17),
    (16, 1 << 13, {"check_workspace": 1}, 2 * 16 * (1 << 13) + 5, 16 * (1 << 13) - 3),
    (2, 1 << 16, {"restart_passes": 2}, 5 * 2 * (1 << 16), 2 * (1 << 16) + 9),
    (4, 1024, {"restart_passes": 4}, 9 * 4096 + 100, 3 * 4096),
    # the largest scratch of any supported shape: n = 16, N = 2^22 streamed
    # (4096 partial nodes per component) with the 2^26-value check tree
    (16, 1 << 22, {"check_workspace": 1}, 16 * (1 << 22) + 5, 16 * (1 << 22) - 2),
]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    W.lib()


def _bits(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n,N,opts,c1,c2", CASES, ids=lambda v: str(v))
def test_fill_static_matches_fill(n, N, opts, c1, c2):
    print(f"fill_static: n={n} N={N} opts={opts} counts=({c1}, {c2})", flush=True)
    ga = W.Generator(1234, n, N, **opts)
    gb = W.Generator(1234, n, N, **opts)
    for count in (c1, c2):
        oa = torch.full((count,), float("nan"), dtype=torch.float32, device="cuda")
        ob = torch.full((count,), float("nan"), dtype=torch.float32, device="cuda")
        ga.fill(oa)
        gb.fill_static(ob)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(oa), _bits(ob)), f"count {count}"
        assert np.isfinite(ob.cpu().numpy()).all()
        assert ga.sumsq() == gb.sumsq()
        assert np.array_equal(ga.pool().view(np.uint32), gb.pool().view(np.uint32))
    assert ga.status() == (0, 0) and gb.status() == (0, 0)


def test_fill_static_interleaved_generators_share_the_array():
    # calls ordered on one stream may share the array: two streamed
    # generators of different shapes alternate, each checked against its twin
    print("fill_static: interleaved generators", flush=True)
    shapes = [(4, 1 << 15), (16, 1 << 13)]
    twins = [(W.Generator(7 + i, n, N), W.Generator(7 + i, n, N)) for i, (n, N) in
             enumerate(shapes)]
    for rnd in range(3):
        for (n, N), (ga, gb) in zip(shapes, twins):
            count = (2 - rnd % 2) * n * N + 11 * rnd
            oa = torch.empty(count, dtype=torch.float32, device="cuda")
            ob = torch.empty(count, dtype=torch.float32, device="cuda")
            ga.fill(oa)
            gb.fill_static(ob)
            torch.cuda.synchronize()
            assert np.array_equal(_bits(oa), _bits(ob)), (n, N, rnd)
