"""GPU parity: the HIP path against the FP32 oracle, bit for bit.

Every case runs the library's kernels through the C ABI on the same seeded
inputs as the oracle (tests/ uses the oracle only as a reference) and
compares every output word, plus the generator state (sum of squares,
passes, current pool).
"""
import math

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
from paper_1004_3114_amd import wallace as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda")


def assert_bits_equal(got, ref, what=""):
    got = np.ascontiguousarray(got, dtype=np.float32)
    ref = np.ascontiguousarray(ref, dtype=np.float32)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    gb, rb = got.view(np.uint32), ref.view(np.uint32)
    bad = np.nonzero(gb != rb)[0]
    if bad.size:
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} of {got.size} words differ; first at {i}: "
                             f"gpu {got[i]!r} oracle {ref[i]!r}")


def gpu_stream(gen, counts):
    outs = []
    for c in counts:
        t = torch.empty(max(c, 1), dtype=torch.float32, device=_dev())
        gen.fill(t, c)
        outs.append(t[:c].cpu().numpy())
    return np.concatenate(outs) if outs else np.empty(0, np.float32)


# ---------------------------------------------------------------------------
# single generators, pool on chip
# ---------------------------------------------------------------------------

def test_single_small_full_run():
    # n = 4, N = 1024, seed 42, 1000 passes: every one of 4,096,000 values
    _dev()
    print("case single_small 4x1024 seed 42 x1000", flush=True)
    g = W.Generator(42, 4, 1024)
    out = torch.empty(4096 * 1000, dtype=torch.float32, device="cuda")
    g.fill(out)
    ref_gen = oracle.Gen(42, 4, 1024)
    ref = ref_gen.fill(4096 * 1000)
    assert_bits_equal(out.cpu().numpy(), ref, "single_small")
    sigma, passes = g.sumsq()
    assert passes == 1000 and sigma == ref_gen.sigma
    assert_bits_equal(g.pool(), ref_gen.pool, "final pool")


SHAPES = [(2, 4), (2, 64), (2, 256), (2, 1024), (2, 4096), (2, 16384),
          (4, 4), (4, 8), (4, 16), (4, 32), (4, 64), (4, 128), (4, 256), (4, 512),
          (4, 1024), (4, 2048), (4, 4096), (4, 8192), (4, 16384),
          (16, 16), (16, 32), (16, 64), (16, 128), (16, 256), (16, 512), (16, 1024),
          (16, 2048), (16, 4096)]


@pytest.mark.parametrize("n,N", SHAPES)
def test_pool_resident_shapes(n, N):
    _dev()
    passes = 12 if n * N <= 4096 else 5
    seed = 1000 + n * 7 + N
    print(f"case pool n={n} N={N} seed={seed} passes={passes}", flush=True)
    g = W.Generator(seed, n, N)
    got = gpu_stream(g, [n * N * passes])
    ref = oracle.Gen(seed, n, N).fill(n * N * passes)
    assert_bits_equal(got, ref, f"n={n} N={N}")


# (4, 8192) and (4, 16384) hold more than 4 tuples per lane: whole pools
# leave through LDS in chunk order, partial ones element by element
@pytest.mark.parametrize("n,N", [(4, 256), (16, 64), (4, 4096), (2, 512), (4, 8192),
                                 (4, 16384), (4, 1 << 15), (2, 1 << 15)])
def test_ragged_call_splits(n, N):
    # the last two pools stream through HBM (fused passes, partial pools
    # copied from the workspace)
    _dev()
    rng = np.random.default_rng(N)
    nu = n * N
    counts = [0, 1, 3, nu - 4, nu, 2 * nu + 5, 17, 0, nu * 3 + 1, 1000]
    counts += [int(x) for x in rng.integers(0, 2 * nu, size=6)]
    print(f"case ragged n={n} N={N}", flush=True)
    g = W.Generator(9, n, N)
    got = gpu_stream(g, counts)
    ref = oracle.Gen(9, n, N).fill(sum(counts))
    assert_bits_equal(got, ref, "ragged")


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("n,N", [(4, 1024), (16, 256), (4, 16384), (2, 2048)])
def test_reduce_modes(mode, n, N):
    _dev()
    print(f"case reduce_mode={mode} n={n} N={N}", flush=True)
    g = W.Generator(5, n, N, reduce_mode=mode)
    got = gpu_stream(g, [n * N * 20])
    ref_gen = oracle.Gen(5, n, N, sum_mode=mode)
    ref = ref_gen.fill(n * N * 20)
    assert_bits_equal(got, ref, f"reduce_mode {mode}")
    assert g.sumsq()[0] == ref_gen.sigma


def test_full_odd_strides():
    _dev()
    g = W.Generator(11, 4, 512, a_mode=1)
    got = gpu_stream(g, [2048 * 30])
    ref = oracle.Gen(11, 4, 512, a_mode=oracle.A_FULL_ODD).fill(2048 * 30)
    assert_bits_equal(got, ref, "a_mode 1")


@pytest.mark.parametrize("n,f,withhold", [(4, 2, 0), (4, 3, 1), (4, 1, 1), (2, 3, 0)])
def test_throwaway_and_withheld_driver(n, f, withhold):
    # RANN4 (n = 2) itself uses f = 3 (section 8)
    _dev()
    N = 256
    emit = n * N - withhold
    g = W.Generator(21, n, N, f=f, withhold_driver=withhold)
    counts = [emit * 3 + 7, emit - 7, 5]
    got = gpu_stream(g, counts)
    ref = oracle.Gen(21, n, N, f=f, withhold=withhold).fill(sum(counts))
    assert_bits_equal(got, ref, f"f={f} withhold={withhold}")


@pytest.mark.parametrize("N", [1024, 8192, 16384])
def test_normal_epilogue(N):
    _dev()
    print(f"case normal epilogue n=4 N={N}", flush=True)
    g = W.Generator(3, 4, N)
    out = torch.empty(4 * N * 5 + 3, dtype=torch.float32, device="cuda")
    g.fill_normal(out, 2.5, 0.75)
    x = oracle.Gen(3, 4, N).fill(out.numel())
    ref = np.float32(2.5) + np.float32(0.75) * x  # one FP32 multiply, one add
    assert_bits_equal(out.cpu().numpy(), ref.astype(np.float32), "mu + sigma x")


@pytest.mark.parametrize("n,N", [(4, 1 << 15), (2, 1 << 15)])
def test_normal_epilogue_streamed(n, N):
    # streamed pools write mu + sigma x to the output and keep the pool in the
    # workspace (a scaled output cannot be the next pass's old pool)
    _dev()
    g = W.Generator(5, n, N)
    total = n * N * 3 + 11
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    g.fill_normal(out, -1.25, 2.0)
    x = oracle.Gen(5, n, N).fill(total)
    ref = np.float32(-1.25) + np.float32(2.0) * x
    assert_bits_equal(out.cpu().numpy(), ref.astype(np.float32), "streamed mu + sigma x")
    # and the stream continues unscaled from the same state
    out2 = torch.empty(n * N, dtype=torch.float32, device="cuda")
    g.fill(out2)
    ref_gen = oracle.Gen(5, n, N)
    ref_gen.fill(total)
    assert_bits_equal(out2.cpu().numpy(), ref_gen.fill(n * N), "continued stream")


def test_corruption_is_detected():
    # Section 8 footnote: a large change in the sum of squares means the work
    # area was overwritten. Force it from the host: overwrite pool bytes.
    _dev()
    g = W.Generator(4, 4, 256, check_workspace=1)
    out = torch.empty(1024 * 4, dtype=torch.float32, device="cuda")
    g.fill(out)
    assert g.status() == (0, 0)
    ws = g.workspace
    base = g._ws_ptr - ws.data_ptr()
    pool_off = 512  # header (256) + state, aligned to 256
    ws[base + pool_off: base + pool_off + 64] = 0x3F
    g.fill(out)
    rc, flags = g.status()
    assert rc == W.WALLACE_ECORRUPT and flags & W.FLAG_CORRUPT


def test_corruption_is_detected_streamed():
    # a streamed pool is checked by the tree kernels at the start of a call
    _dev()
    n, N = 4, 1 << 15
    nu = n * N
    g = W.Generator(4, n, N, check_workspace=1)
    out = torch.empty(nu * 3, dtype=torch.float32, device="cuda")
    g.fill(out)
    assert g.status() == (0, 0)
    ws = g.workspace
    base = g._ws_ptr - ws.data_ptr()
    pool_off = 512  # header (256) + state, aligned to 256; both pool buffers follow
    ws[base + pool_off: base + pool_off + 2 * nu * 4] = 0x3F
    g.fill(out)
    rc, flags = g.status()
    assert rc == W.WALLACE_ECORRUPT and flags & W.FLAG_CORRUPT


# ---------------------------------------------------------------------------
# streaming (pool in HBM)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,N,passes", [(4, 1 << 15, 6), (16, 1 << 13, 6), (4, 1 << 17, 3),
                                        (2, 1 << 15, 6), (2, 1 << 18, 3)])
def test_streaming_small(n, N, passes):
    _dev()
    print(f"case stream n={n} N={N}", flush=True)
    g = W.Generator(77, n, N)
    got = gpu_stream(g, [n * N * passes - 5, 5, 100])
    ref_gen = oracle.Gen(77, n, N)
    ref = ref_gen.fill(n * N * passes + 100)
    assert_bits_equal(got, ref, f"stream n={n} N={N}")


@pytest.mark.parametrize("n,N,f,withhold,mode", [(4, 1 << 15, 2, 1, 0), (2, 1 << 15, 3, 0, 0),
                                                  (4, 1 << 15, 1, 0, 1), (4, 1 << 15, 1, 0, 2),
                                                  (2, 1 << 16, 1, 0, 2)])
def test_streaming_options(n, N, f, withhold, mode):
    # n = 2 and 4 stream with one fused launch per pass (combine, then the
    # next pass's permutation); throw-away passes, a withheld driver and the
    # FP32 sums change which buffers hold the permuted pool between launches
    _dev()
    print(f"case stream options n={n} N={N} f={f} withhold={withhold} mode={mode}", flush=True)
    emit = n * N - withhold
    g = W.Generator(31, n, N, f=f, withhold_driver=withhold, reduce_mode=mode)
    counts = [emit * 2 + 3, emit - 3, 1, emit * 2]
    got = gpu_stream(g, counts)
    ref_gen = oracle.Gen(31, n, N, f=f, withhold=withhold, sum_mode=mode)
    ref = ref_gen.fill(sum(counts))
    assert_bits_equal(got, ref, "stream options")
    assert g.sumsq()[0] == ref_gen.sigma


@pytest.mark.parametrize("n", [4, 2])
def test_streaming_largest_pool(n):
    # N = 2^24, the largest streamed pool (4096 blocks of partial sums per
    # component for n = 4, 2048 for n = 2): two passes word for word
    _dev()
    N = 1 << 24
    nu = n * N
    print(f"case stream largest n={n} N=2^24", flush=True)
    g = W.Generator(3, n, N)
    out = torch.empty(nu * 2, dtype=torch.float32, device="cuda")
    g.fill(out)
    torch.cuda.synchronize()
    ref = oracle.Gen(3, n, N).fill(nu * 2)
    assert_bits_equal(out.cpu().numpy(), ref, f"stream n={n} N=2^24")
    del out, g
    torch.cuda.empty_cache()


def test_streaming_largest_pool_n16():
    # n = 16, N = 2^22 (2^26 values, 256 MB), the largest streamed n = 16 pool
    # (4 tuples per thread): two passes word for word
    _dev()
    n, N = 16, 1 << 22
    nu = n * N
    print("case stream largest n=16 N=2^22", flush=True)
    g = W.Generator(5, n, N)
    out = torch.empty(nu * 2, dtype=torch.float32, device="cuda")
    g.fill(out)
    torch.cuda.synchronize()
    ref = oracle.Gen(5, n, N).fill(nu * 2)
    assert_bits_equal(out.cpu().numpy(), ref, "stream n=16 N=2^22")
    del out, g
    torch.cuda.empty_cache()


def test_generators_on_concurrent_streams():
    # independent generators (section 9) filled from two host threads on two
    # streams at once: two streamed pools and one on chip, each bit for bit
    _dev()
    import threading
    shapes = [(4, 1 << 15, 21), (2, 1 << 15, 22), (16, 1024, 23)]
    passes = 5
    gens, outs, streams = [], [], []
    for n, N, seed in shapes:
        gens.append(W.Generator(seed, n, N))
        outs.append(torch.empty(n * N * passes, dtype=torch.float32, device="cuda"))
        streams.append(torch.cuda.Stream())
    print("case concurrent streams", flush=True)
    torch.cuda.synchronize()
    errors = []

    def run(i):
        try:
            with torch.cuda.stream(streams[i]):
                gens[i].fill(outs[i], stream=streams[i])
        except Exception as e:  # reported below, in the test's thread
            errors.append(e)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(len(shapes))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for (n, N, seed), out in zip(shapes, outs):
        ref = oracle.Gen(seed, n, N).fill(n * N * passes)
        assert_bits_equal(out.cpu().numpy(), ref, f"concurrent n={n} N={N}")


def test_streaming_full_odd_strides():
    # any odd stride (eq. 2): the single-launch gather form of the pass
    _dev()
    n, N = 4, 1 << 14 << 1
    g = W.Generator(13, n, N, a_mode=1)
    got = gpu_stream(g, [n * N * 4 + 9])
    ref = oracle.Gen(13, n, N, a_mode=oracle.A_FULL_ODD).fill(n * N * 4 + 9)
    assert_bits_equal(got, ref, "stream a_mode 1")


@pytest.mark.parametrize("mode", [1, 2])
def test_streaming_reduce_modes(mode):
    _dev()
    g = W.Generator(8, 16, 1 << 13, reduce_mode=mode)
    got = gpu_stream(g, [16 * (1 << 13) * 4])
    ref = oracle.Gen(8, 16, 1 << 13, sum_mode=mode).fill(16 * (1 << 13) * 4)
    assert_bits_equal(got, ref, f"stream reduce {mode}")


def test_single_large_full_size():
    # n = 4, N = 2^22 (64 MB pool), seed 42, 200 passes in one call, as the
    # benchmark runs it; every pass is compared word by word with the oracle
    # (about 0.1-0.25 s of CPU per pass), then invariants that hold at any size.
    _dev()
    n, N, P = 4, 1 << 22, 200
    nu = n * N
    print("case single_large full size", flush=True)
    g = W.Generator(42, n, N)
    out = torch.empty(nu * P, dtype=torch.float32, device="cuda")
    g.fill(out)
    torch.cuda.synchronize()
    ref_gen = oracle.Gen(42, n, N)
    for p in range(P):
        ref = ref_gen.fill(nu)
        assert_bits_equal(out[p * nu:(p + 1) * nu].cpu().numpy(), ref, f"single_large pass {p + 1}")
        if (p + 1) % 50 == 0:
            print(f"single_large: {p + 1} of {P} passes bit-exact", flush=True)
    sigma, passes = g.sumsq()
    assert passes == P
    last = out[(P - 1) * nu:].double()
    assert abs((last * last).sum().item() / sigma - 1) < 1e-12
    assert abs(sigma / nu - 1) < 5 * math.sqrt(2 / nu) * 3
    assert_bits_equal(g.pool(), out[(P - 1) * nu:].cpu().numpy(), "final pool")
    del out
    torch.cuda.empty_cache()


def test_precision_shape_first_passes():
    _dev()
    n, N = 16, 1 << 20
    g = W.Generator(42, n, N)
    got = gpu_stream(g, [n * N * 3])
    ref = oracle.Gen(42, n, N).fill(n * N * 3)
    assert_bits_equal(got, ref, "precision shape")


# ---------------------------------------------------------------------------
# matrix-core transform (n = 16, accuracy variant)
# ---------------------------------------------------------------------------

def test_mfma_transform_accuracy():
    # H16 D / 4 on the matrix cores is not bit-exact; it must stay within the
    # per-variate bound against the FP64 oracle, and differ from the
    # butterflies somewhere (so the matrix-core path is the one that ran)
    _dev()
    n, N, P = 16, 1 << 13, 20
    nu = n * N
    print("case mfma n=16 N=2^13", flush=True)
    g = W.Generator(42, n, N, transform_mode=1)
    got = gpu_stream(g, [nu * P]).reshape(P, nu)
    ref64 = oracle.Gen64(42, n, N).fill(nu * P).reshape(P, nu)
    ref32 = oracle.Gen(42, n, N).fill(nu * P).reshape(P, nu)
    err = np.abs(got.astype(np.float64) - ref64) / np.maximum(1.0, np.abs(ref64))
    err32 = np.abs(ref32.astype(np.float64) - ref64) / np.maximum(1.0, np.abs(ref64))
    print(f"mfma max err {err.max():.3g}, butterflies {err32.max():.3g}", flush=True)
    assert err.max() <= 1e-5
    assert np.any(got.view(np.uint32) != ref32.view(np.uint32))


# ---------------------------------------------------------------------------
# restarts (section 5): Box-Muller refill on the GPU
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,N,R,f,counts", [
    (4, 1024, 10, 1, [4096 * 35]),
    (4, 1024, 10, 1, [4096 * 9 + 7, 4096 * 13, 4096 * 13 - 7]),
    (4, 256, 4, 2, [1024 * 9]),
    (2, 512, 6, 3, [1024 * 7]),
    (4, 1 << 15, 4, 1, [(1 << 17) * 10]),
    (16, 1 << 13, 3, 1, [(1 << 17) * 7]),
])
def test_restart_refills(n, N, R, f, counts):
    # The refill uses the GPU's FP64 log, cos and sin, the oracle the host's
    # libm: a refilled value can differ in its last bit, and the passes after
    # it then stay within FP32 rounding of the oracle. Everything else is
    # bit-exact.
    _dev()
    print(f"case restart n={n} N={N} R={R} f={f}", flush=True)
    g = W.Generator(17, n, N, restart_passes=R, f=f)
    got = gpu_stream(g, counts)
    ref_gen = oracle.Gen(17, n, N, restart=R, f=f)
    ref = ref_gen.fill(sum(counts))
    same = np.mean(got.view(np.uint32) == ref.view(np.uint32))
    err = np.abs(got.astype(np.float64) - ref) / np.maximum(1.0, np.abs(ref))
    print(f"restart: identical words {same:.6f}, max error {err.max():.3g}", flush=True)
    assert same >= 0.999 and err.max() <= 1e-5
    _, passes = g.sumsq()
    assert passes == ref_gen.passes
