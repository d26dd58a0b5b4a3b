"""GPU parity of batched generators (independent pools, section 9) against
the FP32 oracle, including the full-size uniform workload (every generator)
and the uneven one (sampled generators) in the launch configuration the
benchmark times."""
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
from paper_1004_3114_amd import wallace as W  # noqa: E402
from paper_1004_3114_amd import workloads  # noqa: E402
from tests.test_gpu_parity import assert_bits_equal  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_generator_output(seed, n, N, passes):
    return oracle.Gen(int(seed), int(n), int(N)).fill(int(n) * int(N) * int(passes))


def test_mixed_small_batch_two_launches():
    _dev()
    rng = np.random.default_rng(1)
    shapes = [(4, 4), (4, 64), (4, 256), (4, 1024), (4, 4096), (4, 16384), (16, 16),
              (16, 64), (16, 256), (16, 1024), (16, 4096), (2, 256), (2, 8192)]
    G = 40
    pick = rng.integers(0, len(shapes), size=G)
    n = np.array([shapes[i][0] for i in pick], dtype=np.int32)
    N = np.array([shapes[i][1] for i in pick], dtype=np.uint32)
    seeds = np.arange(500, 500 + G, dtype=np.uint64)
    passes = rng.integers(0, 9, size=G).astype(np.uint32)
    nu = n.astype(np.uint64) * N
    sizes = nu * passes
    off = np.zeros(G, np.uint64)
    np.cumsum(sizes[:-1], out=off[1:])
    total = int(sizes.sum())
    print(f"case mixed batch G={G} total={total}", flush=True)
    b = W.Batch(seeds, n, N)
    b.plan(off, passes)
    outs = []
    for launch in range(2):
        out = torch.full((max(total, 1),), float("nan"), dtype=torch.float32, device="cuda")
        b.fill(out)
        outs.append(out.cpu().numpy())
    for g in range(G):
        ref = oracle_generator_output(seeds[g], n[g], N[g], 2 * int(passes[g]))
        L = int(sizes[g])
        got = np.concatenate([o[int(off[g]):int(off[g]) + L] for o in outs])
        assert_bits_equal(got, ref, f"gen {g} n={n[g]} N={N[g]} passes={passes[g]}")
        s, p = b.sumsq(g)
        assert p == 2 * passes[g]
    assert b.status() == (0, 0)


def test_mixed_batch_side_stream_choices():
    # the classes of a fill run on the caller's side streams (torch's, the
    # binding's default), on streams the library creates, or on fewer side
    # streams than classes: latency-bound classes (pools of <= 8192 values)
    # first on the fill's stream, the others beside them; every choice must
    # continue each generator's stream exactly
    _dev()
    shapes = [(4, 64), (16, 64), (4, 512), (4, 4096), (16, 1024), (4, 16384), (16, 4096)]
    G = 21
    n = np.array([shapes[g % len(shapes)][0] for g in range(G)], dtype=np.int32)
    N = np.array([shapes[g % len(shapes)][1] for g in range(G)], dtype=np.uint32)
    seeds = np.arange(900, 900 + G, dtype=np.uint64)
    passes = (np.arange(G) % 3 + 1).astype(np.uint32)
    sizes = n.astype(np.uint64) * N * passes
    off = np.zeros(G, np.uint64)
    np.cumsum(sizes[:-1], out=off[1:])
    total = int(sizes.sum())
    print(f"case side streams G={G} total={total}", flush=True)
    b = W.Batch(seeds, n, N)
    b.plan(off, passes)
    refs = [oracle.Gen(int(seeds[g]), int(n[g]), int(N[g])) for g in range(G)]
    one = torch.cuda.Stream()
    for choice in ("torch", "library", "one", "torch"):
        if choice == "library":
            b.set_streams([])
        elif choice == "one":
            b.set_streams([one])
        else:
            b.set_streams(b.side_streams)
        out = torch.full((total,), float("nan"), dtype=torch.float32, device="cuda")
        b.fill(out)
        torch.cuda.synchronize()
        host = out.cpu().numpy()
        for g in range(G):
            assert_bits_equal(host[int(off[g]):int(off[g]) + int(sizes[g])],
                              refs[g].fill(int(sizes[g])), f"{choice} gen {g} n={n[g]} N={N[g]}")
    assert b.status() == (0, 0)


def test_tuning_on_the_planned_fill_keeps_state_and_bits():
    # wallace_batch_tune_planned runs every class's planned jobs under each
    # candidate schedule on a copy of the states and pools, writing into the
    # output: afterwards the generators are where they were, and the tuned
    # fill continues every stream exactly
    _dev()
    shapes = [(4, 256), (4, 4096), (16, 64), (16, 2048), (2, 1024)]
    G = 15
    n = np.array([shapes[g % len(shapes)][0] for g in range(G)], dtype=np.int32)
    N = np.array([shapes[g % len(shapes)][1] for g in range(G)], dtype=np.uint32)
    seeds = np.arange(1300, 1300 + G, dtype=np.uint64)
    passes = (np.arange(G) % 4 + 2).astype(np.uint32)
    sizes = n.astype(np.uint64) * N * passes
    off = np.zeros(G, np.uint64)
    np.cumsum(sizes[:-1], out=off[1:])
    total = int(sizes.sum())
    print(f"case tune on the planned fill G={G} total={total}", flush=True)
    b = W.Batch(seeds, n, N)
    b.plan(off, passes)
    before = [b.sumsq(g) for g in range(G)]
    out = torch.zeros(total, dtype=torch.float32, device="cuda")
    b.tune_planned(out)
    assert [b.sumsq(g) for g in range(G)] == before
    assert all(p == 0 for _, p in before)
    out.fill_(float("nan"))
    b.fill(out)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    for g in range(G):
        ref = oracle_generator_output(seeds[g], n[g], N[g], int(passes[g]))
        assert_bits_equal(host[int(off[g]):int(off[g]) + int(sizes[g])], ref,
                          f"gen {g} n={n[g]} N={N[g]}")
    assert b.status() == (0, 0)
    with pytest.raises(RuntimeError):  # not planned: refused before the library is called
        W.Batch(seeds[:2], n[:2], N[:2]).tune_planned(out)


def test_mixed_batch_graph_replays():
    # classes run on forked streams; captured in a graph, the fork and join
    # become parallel branches. Every replay continues each generator's
    # stream and must match the oracle, with eager work between replays.
    _dev()
    rng = np.random.default_rng(5)
    shapes = [(4, 16), (4, 256), (4, 1024), (4, 4096), (16, 16), (16, 256), (16, 1024),
              (2, 512)]
    G = 28
    pick = np.arange(G) % len(shapes)
    n = np.array([shapes[i][0] for i in pick], dtype=np.int32)
    N = np.array([shapes[i][1] for i in pick], dtype=np.uint32)
    seeds = np.arange(700, 700 + G, dtype=np.uint64)
    passes = rng.integers(1, 4, size=G).astype(np.uint32)
    nu = n.astype(np.uint64) * N
    sizes = nu * passes
    off = np.zeros(G, np.uint64)
    np.cumsum(sizes[:-1], out=off[1:])
    total = int(sizes.sum())
    print(f"case mixed batch graph G={G} total={total}", flush=True)
    b = W.Batch(seeds, n, N)
    b.plan(off, passes)
    out = torch.zeros(total, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        b.fill(out, stream=torch.cuda.current_stream())
    refs = [oracle.Gen(int(seeds[g]), int(n[g]), int(N[g])) for g in range(G)]
    for rep in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        host = out.cpu().numpy()
        for g in range(G):
            ref = refs[g].fill(int(sizes[g]))
            assert_bits_equal(host[int(off[g]):int(off[g]) + int(sizes[g])], ref,
                              f"replay {rep} gen {g} n={n[g]} N={N[g]}")
    assert b.status() == (0, 0)


@pytest.mark.parametrize("n,N", [(4, 256), (4, 2048), (16, 64), (16, 1024), (4, 16384),
                                 (16, 4096), (2, 1024)])
def test_every_schedule_gives_identical_bits(n, N, monkeypatch):
    # Schedules differ in lanes per pool, tuples per lane and components per
    # LDS stage; the tree order of every reduction is the same, so each one
    # must reproduce the oracle exactly. Compiled shapes: T <= 16 (n = 16:
    # T <= 4).
    _dev()
    cands = []
    for T in (1, 2, 4, 8, 16):
        if N % T or (n == 16 and T > 4):
            continue
        L = N // T
        if L < n or L > 1024:
            continue
        # one stage (C = n) while the pool fits 128 KiB, else two
        C = n if n * N * 4 <= 128 * 1024 else n // 2
        cands.append((T, L, C))
    assert cands
    G = 9
    seeds = np.arange(70, 70 + G, dtype=np.uint64)
    passes = np.full(G, 3, dtype=np.uint32)
    nu = n * N
    off = np.arange(G, dtype=np.uint64) * (nu * 3)
    refs = [oracle_generator_output(s, n, N, 3) for s in seeds]
    for T, L, C in cands:
        monkeypatch.setenv("WALLACE_SCHED", f"{n}:{N}:{T}:{L}:{C}")
        print(f"case sched n={n} N={N} T={T} L={L} C={C}", flush=True)
        b = W.Batch(seeds, [n] * G, [N] * G)
        b.plan(off, passes)
        out = torch.empty(G * nu * 3, dtype=torch.float32, device="cuda")
        b.fill(out)
        host = out.cpu().numpy()
        for g in range(G):
            assert_bits_equal(host[g * nu * 3:(g + 1) * nu * 3], refs[g],
                              f"T={T} L={L} C={C} gen {g}")


def test_undersized_output_is_rejected_before_launch():
    # An output tensor shorter than the plan writes (or of the wrong dtype)
    # never reaches a kernel: the binding raises, and the C entry point
    # returns WALLACE_EINVAL for an out_len below the planned extent.
    _dev()
    G = 4
    b = W.Batch(np.arange(3, 3 + G, dtype=np.uint64), [4] * G, [256] * G)
    off = np.arange(G, dtype=np.uint64) * (1024 * 2)
    b.plan(off, np.full(G, 2, dtype=np.uint32))
    assert b.extent == G * 1024 * 2
    guard = torch.full((G * 1024 * 2 + 64,), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        b.fill(guard[:b.extent - 1])
    with pytest.raises(TypeError):
        b.fill(torch.empty(b.extent, dtype=torch.float16, device="cuda"))
    L = W.lib()
    rc = L.wallace_fill_batched(b._h, guard.data_ptr(), b.extent - 1,
                                torch.cuda.current_stream().cuda_stream)
    assert rc == W.WALLACE_EINVAL
    torch.cuda.synchronize()
    assert bool((guard == 7.0).all())  # nothing was written
    b.fill(guard[:b.extent])
    host = guard.cpu().numpy()
    assert np.all(host[b.extent:] == 7.0)
    ref = oracle_generator_output(3, 4, 256, 2)
    assert_bits_equal(host[:2048], ref, "first generator after the rejected calls")


def test_forced_schedule_that_is_not_compiled_is_rejected(monkeypatch):
    # A WALLACE_SCHED entry naming the class must be a compiled shape; an
    # entry that is not (here two stages for a pool that fits one) makes
    # init fail instead of silently running another schedule.
    _dev()
    monkeypatch.setenv("WALLACE_SCHED", "4:256:4:64:2")
    with pytest.raises(W.WallaceError) as ei:
        W.Batch([1, 2], [4, 4], [256, 256])
    assert ei.value.code == -1
    with pytest.raises(W.WallaceError) as ei:
        W.Generator(1, 4, 256)
    assert ei.value.code == -1
    monkeypatch.setenv("WALLACE_SCHED", "4:256:4:64:4")
    W.Batch([1, 2], [4, 4], [256, 256])
    W.Generator(1, 4, 256)


def test_autotuners_keep_a_forced_schedule(tmp_path, monkeypatch):
    # A class forced through WALLACE_SCHED keeps its schedule through both
    # autotuners; the other classes are tuned as usual, and the fill stays
    # exact. Here the forced shape (2 tuples on 128 lanes) is not the
    # default one (4 on 64).
    _dev()
    monkeypatch.setenv("WALLACE_TUNE_CACHE", str(tmp_path / "tune.txt"))
    monkeypatch.setenv("WALLACE_SCHED", "4:256:2:128:4")
    G = 12
    seeds = np.arange(1500, 1500 + G, dtype=np.uint64)
    n = np.array([4] * 6 + [16] * 6, dtype=np.int32)
    N = np.array([256] * 6 + [1024] * 6, dtype=np.uint32)
    passes = np.full(G, 3, dtype=np.uint32)
    nu = n.astype(np.uint64) * N
    off = np.zeros(G, np.uint64)
    np.cumsum((nu * 3)[:-1], out=off[1:])
    total = int((nu * 3).sum())
    print(f"case forced schedule through the autotuners G={G}", flush=True)
    b = W.Batch(seeds, n, N)
    b.tune()
    b.plan(off, passes)
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    b.tune_planned(out)
    cls = {(c["n"], c["N"]): c for c in b.classes()}
    assert (cls[(4, 256)]["T"], cls[(4, 256)]["L"], cls[(4, 256)]["C"]) == (2, 128, 4)
    out.fill_(float("nan"))
    b.fill(out)
    host = out.cpu().numpy()
    for g in (0, 5, 6, 11):
        ref = oracle_generator_output(seeds[g], n[g], N[g], 3)
        assert_bits_equal(host[int(off[g]):int(off[g]) + int(nu[g]) * 3], ref, f"gen {g}")
    assert b.status() == (0, 0)


def test_tuner_runs_and_keeps_state(tmp_path, monkeypatch):
    _dev()
    monkeypatch.setenv("WALLACE_TUNE_CACHE", str(tmp_path / "tune.txt"))
    G = 64
    seeds = np.arange(900, 900 + G, dtype=np.uint64)
    n = np.array([4] * 32 + [16] * 32, dtype=np.int32)
    N = np.array([1024] * 32 + [256] * 32, dtype=np.uint32)
    b = W.Batch(seeds, n, N)
    b.tune()
    passes = np.full(G, 2, dtype=np.uint32)
    nu = n.astype(np.uint64) * N
    off = np.zeros(G, np.uint64)
    np.cumsum((nu * 2)[:-1], out=off[1:])
    b.plan(off, passes)
    out = torch.empty(int((nu * 2).sum()), dtype=torch.float32, device="cuda")
    b.fill(out)
    host = out.cpu().numpy()
    for g in (0, 31, 32, 63):
        ref = oracle_generator_output(seeds[g], n[g], N[g], 2)
        assert_bits_equal(host[int(off[g]):int(off[g]) + int(nu[g]) * 2], ref, f"gen {g}")
    text = (tmp_path / "tune.txt").read_text().split("\n")
    assert len([t for t in text if t.strip()]) == 2


def test_batch_uniform_full_size_graph():
    # 65,536 generators (n = 4, N = 256, seeds 42 + g), 64 passes per launch,
    # 4 launches captured in one HIP graph, as the benchmark runs them.
    _dev()
    spec = workloads.batch_uniform()
    per = spec.normals_per_launch()
    print(f"case batch_uniform full size per launch {per}", flush=True)
    b = W.Batch(spec.seeds, spec.n, spec.N)
    off = spec.offsets()
    b.plan(off, spec.passes)
    out = torch.empty(per * spec.launches, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for launch in range(spec.launches):
            b.fill(out[launch * per:], stream=torch.cuda.current_stream())
    graph.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    sample = sorted(set([0, 1, 4095, 65535] + [int(x) for x in rng.integers(0, spec.G, 12)]))
    nu = 1024
    for g in sample:
        ref = oracle_generator_output(spec.seeds[g], 4, 256, 64 * spec.launches)
        got = np.concatenate([
            out[launch * per + int(off[g]): launch * per + int(off[g]) + 64 * nu].cpu().numpy()
            for launch in range(spec.launches)])
        assert_bits_equal(got, ref, f"batch_uniform gen {g}")
    s, p = b.sumsq(65535)
    assert p == 256
    # Then every generator, all 256 passes, bit for bit. The oracle runs in
    # threads (its C calls release the GIL and it has no mutable global state;
    # no process is forked from this one, which holds the GPU). The output
    # comes to the host in chunks of 4096 generators (4 GiB).
    workers = max(1, min(16, os.cpu_count() or 1))
    gen_len = 64 * nu  # one generator's values per launch
    chunk = 4096
    t0 = time.time()
    with ThreadPoolExecutor(workers) as ex:
        for g0 in range(0, spec.G, chunk):
            g1 = min(spec.G, g0 + chunk)
            lo, hi = int(off[g0]), int(off[g1 - 1]) + gen_len
            host = [out[launch * per + lo:launch * per + hi].cpu().numpy().view(np.uint32)
                    for launch in range(spec.launches)]

            def differs(g, host=host, lo=lo):
                ref = oracle_generator_output(spec.seeds[g], 4, 256, 64 * spec.launches)
                ref = ref.view(np.uint32)
                base = int(off[g]) - lo
                return any(not np.array_equal(host[launch][base:base + gen_len],
                                              ref[launch * gen_len:(launch + 1) * gen_len])
                           for launch in range(spec.launches))

            bad = [g for g, d in zip(range(g0, g1), ex.map(differs, range(g0, g1))) if d]
            assert not bad, f"generators differing from the oracle: {bad[:8]} ({len(bad)})"
            del host
    print(f"batch_uniform: all {spec.G} generators bit-exact over {64 * spec.launches} passes "
          f"({time.time() - t0:.1f} s, {workers} threads)", flush=True)
    # every generator, every value: finite, and the first two moments of the
    # 2^34 outputs at N(0, 1). Each pool's sum of squares is its chi-squared
    # sample S (mean nu, standard deviation about sqrt(2 nu)), so the second
    # moment over 2^24 pools sits within about 1e-5 of 1; the mean's standard
    # error is below 1e-5.
    s1 = s2 = 0.0
    step = 1 << 28
    for i in range(0, out.numel(), step):
        x = out[i:i + step]
        assert bool(torch.isfinite(x).all()), f"non-finite output in [{i}, {i + step})"
        xd = x.double()
        s1 += float(xd.sum())
        s2 += float((xd * xd).sum())
        del xd
    m = out.numel()
    mean, second = s1 / m, s2 / m
    print(f"batch_uniform moments: mean {mean:.3e} second {second:.8f}", flush=True)
    assert abs(mean) < 1e-4
    assert abs(second - 1.0) < 1e-3
    del out
    torch.cuda.empty_cache()


def test_batch_uneven_full_size():
    # 10,000 generators of mixed n and N, tuned schedules, one launch per
    # class on forked streams, as the benchmark runs them: every generator
    # and every pass bit for bit (oracle in threads, as for the uniform batch;
    # the longest job and one generator per class are checked first, in this
    # thread, with a message naming them).
    _dev()
    spec = workloads.batch_uneven()
    per = spec.normals_per_launch()
    print(f"case batch_uneven full size {per}", flush=True)
    b = W.Batch(spec.seeds, spec.n, spec.N)
    b.tune()  # the benchmark's launch configuration
    off = spec.offsets()
    b.plan(off, spec.passes)
    out = torch.empty(per, dtype=torch.float32, device="cuda")
    b.fill(out)
    torch.cuda.synchronize()
    sizes = spec.nu * spec.passes.astype(np.uint64)
    picked = {}
    for g in range(spec.G):
        key = (int(spec.n[g]), int(spec.N[g]))
        picked.setdefault(key, [])
        if len(picked[key]) < 1 and spec.passes[g] <= 64:
            picked[key].append(g)
    picked[(-1, -1)] = [int(np.argmax(sizes))]  # the longest job
    for key, gs in sorted(picked.items()):
        for g in gs:
            L = int(sizes[g])
            ref = oracle_generator_output(spec.seeds[g], spec.n[g], spec.N[g], spec.passes[g])
            got = out[int(off[g]):int(off[g]) + L].cpu().numpy()
            assert_bits_equal(got, ref, f"uneven gen {g} n={spec.n[g]} N={spec.N[g]}")
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.time()
    limit = 1 << 30  # floats per host chunk (4 GiB)
    g0 = 0
    with ThreadPoolExecutor(workers) as ex:
        while g0 < spec.G:
            g1 = g0 + 1
            while g1 < spec.G and int(off[g1]) + int(sizes[g1]) - int(off[g0]) <= limit:
                g1 += 1
            lo, hi = int(off[g0]), int(off[g1 - 1]) + int(sizes[g1 - 1])
            host = out[lo:hi].cpu().numpy().view(np.uint32)

            def differs(g, host=host, lo=lo):
                ref = oracle_generator_output(spec.seeds[g], spec.n[g], spec.N[g],
                                              spec.passes[g]).view(np.uint32)
                base = int(off[g]) - lo
                return not np.array_equal(host[base:base + int(sizes[g])], ref)

            bad = [g for g, d in zip(range(g0, g1), ex.map(differs, range(g0, g1))) if d]
            assert not bad, f"generators differing from the oracle: {bad[:8]} ({len(bad)})"
            del host
            g0 = g1
    print(f"batch_uneven: all {spec.G} generators bit-exact ({time.time() - t0:.1f} s, "
          f"{workers} threads)", flush=True)
    del out
    torch.cuda.empty_cache()
