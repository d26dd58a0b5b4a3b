"""Benchmark of the Wallace pool-regeneration pass on one MI355X.

A step is one pass of the whole hot path over the batched uniform workload:
65,536 independent generators (n = 4, N = 256, seeds 42 + g), 64 passes per
launch, 4 launches replayed as one HIP graph: 2^34 normals written to HBM.
Inputs (the pools) are resident in HBM when the timed region starts.

Printed: one JSON line with normals/s (`value`), the HBM-write roofline of
the pass kernel (HIP events on the launch stream), the single-pool forms
beside it (4096-value pool, 1000 passes; 2^24-value pool streamed through
HBM, 200 passes), the uneven batch, a plain-store ceiling, and the CPU
oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --only headline     (profiling runs: no extras)
       python bench.py --only single_small (profiling runs: one small pool only)
       python bench.py --only single_large (profiling runs: streamed pool only)
       python bench.py --only uneven       (profiling runs: uneven batch only)
       python bench.py --only headline_candidates (every compiled schedule of the
                                           headline class, then the autotuner's pick)
       python bench.py --only precision_shape (n = 16, N = 2^20 pass: butterflies
                                           against the matrix-core transform)
       python bench.py --copy-probe BYTES  (calibration copy for counters)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_NORMAL = 4.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("wallace_pool.hpp", "wallace_devmath.hpp", "wallace_pool_inst.hip",
                 "wallace_kernels.hip", "wallace_internal.h"):
        with open(os.path.join(ROOT, "paper_1004_3114_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "pool_kernel_batch_uniform_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def timed_events(torch, stream, fn, reps):
    """Run fn() reps times between HIP events on `stream`; returns ms each."""
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return times


def headline(torch, W, workloads, steps, warmup):
    spec = workloads.batch_uniform()
    per = spec.normals_per_launch()
    total = per * spec.launches
    log(f"batch_uniform: G={spec.G} n=4 N=256 passes/launch=64 launches={spec.launches}; "
        f"init pools on host")
    t0 = time.time()
    b = W.Batch(spec.seeds, spec.n, spec.N)
    b.plan(spec.offsets(), spec.passes)
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    # the class's schedule, picked by the library's autotuner on the planned
    # launch itself (the generators' state is left as it is)
    b.tune_planned(out[:per])
    sched = {k: b.classes()[0][k] for k in ("T", "L", "C")}
    # a schedule forced through WALLACE_SCHED is kept by the autotuner
    forced = any(e.split(":")[:2] == ["4", "256"]
                 for e in os.environ.get("WALLACE_SCHED", "").split(","))
    log(f"init and tuning {time.time() - t0:.1f}s (schedule {sched}); "
        f"output {total * 4 / 2**30:.0f} GiB")
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        cur = torch.cuda.current_stream()
        for launch in range(spec.launches):
            b.fill(out[launch * per:], stream=cur)
    replay_stream = torch.cuda.current_stream()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    log(f"warmup {warmup} done; timing {steps} steps")
    # timed region: K graph replays bracketed by device synchronisation
    ev = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(replay_stream)
        graph.replay()
        e1.record(replay_stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = [a.elapsed_time(c) for a, c in ev]
    ms_per_step = wall * 1000.0 / steps
    value = total * steps / wall
    # roofline of the pass kernel: algorithmic bytes per launch over the
    # average launch duration (graph replay time / launches, on its stream)
    launch_ms = (sum(step_ms) / len(step_ms)) / spec.launches
    pool_io = 2 * 4 * 1024 / (64 * 1024)  # pool load + store per 64-pass launch, per normal
    alg_bytes = per * (BYTES_PER_NORMAL + pool_io)
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    khash = kernel_source_hash()
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": counter_traffic(khash),
            "kernel": f"k_pool<4,{sched['T']},{sched['L']}> (n=4, T tuples/lane, L lanes/pool)",
            "alg_bytes_per_launch": int(alg_bytes), "avg_launch_ms": round(launch_ms, 4),
            "kernel_source_hash": khash}
    del graph, out
    torch.cuda.empty_cache()
    return value, ms_per_step, roof, {"G": spec.G, "n": 4, "N": 256, "passes_per_launch": 64,
                                      "launches_per_step": spec.launches,
                                      "normals_per_step": total,
                                      "schedule": {**sched, "picked_by": "WALLACE_SCHED" if forced
                                                   else "autotuner"}}


def headline_candidates(torch, W, workloads, reps=5):
    """The headline workload under every compiled pool-resident schedule of
    its class (n = 4, N = 256): T tuples per lane on L = 256 / T lanes, C
    components per on-chip stage, forced through WALLACE_SCHED; ms per
    launch (median of reps graph replays of 4 launches). Then the library's
    autotuner on the planned launch, and the schedule it picks."""
    spec = workloads.batch_uniform()
    per = spec.normals_per_launch()
    alg = per * (BYTES_PER_NORMAL + 2 * 4 * 1024 / (64 * 1024))
    out = torch.empty(per * spec.launches, dtype=torch.float32, device="cuda")
    rows = []
    saved = os.environ.get("WALLACE_SCHED")
    try:
        for T in (1, 2, 4, 8, 16):
            for C in (4, 2):
                os.environ["WALLACE_SCHED"] = f"4:256:{T}:{256 // T}:{C}"
                try:
                    b = W.Batch(spec.seeds, spec.n, spec.N)
                except W.WallaceError:
                    continue  # not a compiled shape
                b.plan(spec.offsets(), spec.passes)
                graph = torch.cuda.CUDAGraph()
                stream = torch.cuda.Stream()
                with torch.cuda.graph(graph, stream=stream):
                    cur = torch.cuda.current_stream()
                    for launch in range(spec.launches):
                        b.fill(out[launch * per:], stream=cur)
                graph.replay()
                torch.cuda.synchronize()
                rs = torch.cuda.current_stream()
                ms = sorted(timed_events(torch, rs, graph.replay, reps))
                launch_ms = ms[len(ms) // 2] / spec.launches
                rows.append({"T": T, "L": 256 // T, "C": C, "ms_per_launch": round(launch_ms, 4),
                             "GBps": round(alg / (launch_ms * 1e-3) / 1e9, 1)})
                log(f"candidate T={T} L={256 // T} C={C}: {launch_ms:.4f} ms per launch")
                del graph, b
    finally:
        if saved is None:
            os.environ.pop("WALLACE_SCHED", None)
        else:
            os.environ["WALLACE_SCHED"] = saved
    b = W.Batch(spec.seeds, spec.n, spec.N)
    default = b.classes()[0]
    b.plan(spec.offsets(), spec.passes)
    b.tune_planned(out[:per])
    tuned = b.classes()[0]
    del b, out
    torch.cuda.empty_cache()
    return {"workload": "batch_uniform", "candidates": rows,
            "default": {k: default[k] for k in ("T", "L", "C")},
            "tuner_pick": {k: tuned[k] for k in ("T", "L", "C")}}


def precision_shape(torch, W, workloads, passes=50, reps=3):
    """The long-run precision workload's pass (n = 16, N = 2^20, seed 42) with
    the butterflies and with the matrix-core transform: microseconds per pass
    over a fill of `passes` returned pools (best of reps, fresh generator
    each time)."""
    spec = workloads.PRECISION
    out = torch.empty(passes * spec.nu, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {"workload": spec.name, "n": spec.n, "N": spec.N, "passes_timed": passes}
    for tm, name in ((0, "butterflies"), (1, "matrix_cores")):
        best = None
        for r in range(reps + 1):
            g = W.Generator(spec.seed, spec.n, spec.N, transform_mode=tm)
            torch.cuda.synchronize()
            ms = timed_events(torch, stream, lambda: g.fill(out), 1)[0]
            if r > 0:
                best = ms if best is None else min(best, ms)
            del g
        res[f"{name}_us_per_pass"] = round(best * 1e3 / passes, 2)
    del out
    torch.cuda.empty_cache()
    return res


def single_pool(torch, W, workloads, which, reps=3, keep=None):
    """Times one fill of the whole workload on a fresh generator (best of
    reps after one untimed run). keep: receives the last generator's final
    pool, sum of squares and pass count."""
    spec = workloads.SINGLE_SMALL if which == "small" else workloads.SINGLE_LARGE
    log(f"single pool {spec.name}: n={spec.n} N={spec.N} passes={spec.passes}")
    out = torch.empty(spec.normals, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    best = None
    for r in range(reps + 1):
        g = W.Generator(spec.seed, spec.n, spec.N)  # fresh generator each time
        torch.cuda.synchronize()
        ms = timed_events(torch, stream, lambda: g.fill(out), 1)[0]
        if r > 0:
            best = ms if best is None else min(best, ms)
        if r == reps and keep is not None:
            keep["pool"] = g.pool()
            keep["sigma"], keep["passes"] = g.sumsq()
        del g
    del out
    torch.cuda.empty_cache()
    rate = spec.normals / (best * 1e-3)
    res = {"workload": spec.name, "n": spec.n, "N": spec.N, "passes": spec.passes,
           "normals": spec.normals, "ms": round(best, 3), "normals_per_s": rate,
           "write_GBps": round(rate * 4 / 1e9, 1),
           "frac_hbm": round(rate * 4 / 1e9 / HBM_PEAK_GBPS, 4)}
    if which == "large":
        # algorithmic: each pass writes the returned pool and reads the old
        # one once (8 bytes per value)
        nu = spec.n * spec.N
        alg = 8 * nu * spec.passes
        res["hbm_alg_bytes"] = alg
        res["hbm_alg_GBps"] = round(alg / (best * 1e-3) / 1e9, 1)
        res["hbm_alg_frac"] = round(alg / (best * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
        # moved by this design (n = 2, 4): a permute of the starting pool
        # (read and write), then per pass one fused launch that reads the
        # permuted pool and writes the output and the next permuted pool; the
        # last pass writes the workspace pool instead of a permuted one
        moved = 8 * nu + 12 * nu * spec.passes
        res["hbm_moved_bytes"] = moved
        res["hbm_moved_GBps"] = round(moved / (best * 1e-3) / 1e9, 1)
    return res


def uneven(torch, W, workloads, reps=3):
    spec = workloads.batch_uneven()
    total = spec.normals_per_launch()
    log(f"batch_uneven: G={spec.G} normals={total}")
    b = W.Batch(spec.seeds, spec.n, spec.N)
    b.plan(spec.offsets(), spec.passes)
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    t0 = time.time()
    b.tune_planned(out)  # per (n, N) class: the fastest schedule on its planned jobs
    log(f"batch_uneven tuned in {time.time() - t0:.1f}s")
    stream = torch.cuda.current_stream()
    b.fill(out)
    ms = min(timed_events(torch, stream, lambda: b.fill(out), reps))
    # the same fill captured in a HIP graph (its side streams become parallel
    # branches), replayed
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    with torch.cuda.graph(graph, stream=cap):
        b.fill(out, stream=torch.cuda.current_stream())
    graph.replay()
    torch.cuda.synchronize()
    gms = min(timed_events(torch, torch.cuda.current_stream(), graph.replay, reps))
    classes = b.classes()
    del graph, out, b
    torch.cuda.empty_cache()
    rate = total / (ms * 1e-3)
    return {"workload": "batch_uneven", "G": spec.G, "normals": total, "ms": round(ms, 3),
            "normals_per_s": rate, "write_GBps": round(rate * 4 / 1e9, 1),
            "frac_hbm": round(rate * 4 / 1e9 / HBM_PEAK_GBPS, 4),
            "graph_ms": round(gms, 3), "graph_normals_per_s": total / (gms * 1e-3),
            "classes": classes}


def store_ceilings(torch, nbytes=16 << 30, reps=5):
    """Plain store streams on the same GPU, GB/s (best of reps over 16 GiB):
    torch's fill kernel; the store-ceiling kernels of libwallace_check.so in
    one-shot form (one 16-byte chunk per thread, blocks in address order,
    nontemporal and plain); and long-lived waves writing the headline's own
    pattern with no arithmetic (65,536 waves, each 64 consecutive 4 KB
    pools)."""
    from paper_1004_3114_amd import check as CK
    t = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    t.fill_(1.0)

    def rate(fn):
        fn()
        ms = min(timed_events(torch, stream, fn, reps))
        return round(nbytes / (ms * 1e-3) / 1e9, 1)

    waves, chunks = 65536, 64
    assert waves * chunks * 1024 * 4 == nbytes
    res = {"torch_fill": rate(lambda: t.fill_(0.5)),
           "oneshot_nontemporal": rate(lambda: CK.store_oneshot(t, 0.25, True)),
           "oneshot": rate(lambda: CK.store_oneshot(t, 0.25, False)),
           "longlived_headline_pattern": rate(
               lambda: CK.store_longlived(t, waves, chunks, chunks * 1024, 1024))}
    del t
    torch.cuda.empty_cache()
    return res


def precision_report(small, large):
    """Precision of the single pools after their full pass counts, from the
    GPU's final pools (small/large: the kept pool, sum of squares and pass
    count) and the oracle results the CPU-baseline leg kept: bit-equality
    with the FP32 oracle (SHA-256 of the pool), the drift of the pool's
    exact sum of squares from the chi-squared target S of its last pass
    (section 4), the library's sum of squares against that exact sum, and
    for the small pool the per-variate error e = |x32 - x64| / max(1, |x64|)
    against the FP64 oracle (bound 1e-5)."""
    out = {}
    for name, got in (("single_small", small), ("single_large", large)):
        if not got or f"{name}_fp32_S" not in PRECISION_REF:
            continue
        pool = got["pool"]
        d = pool.astype(np.float64)
        exact = float(np.sum(d * d))
        S = PRECISION_REF[f"{name}_fp32_S"]
        rec = {"passes": int(got["passes"]),
               "bit_exact_vs_fp32_oracle":
                   hashlib.sha256(pool.tobytes()).hexdigest() == PRECISION_REF[f"{name}_fp32_sha"],
               "sigma_drift": abs(exact - S) / S,
               "sigma_lib_rel_err": abs(got["sigma"] - exact) / exact}
        x64 = PRECISION_REF.get(f"{name}_fp64_pool")
        if x64 is not None:
            e = np.abs(d - x64) / np.maximum(1.0, np.abs(x64))
            rec.update({"vs": "FP64 oracle", "err_max": float(e.max()),
                        "err_rms": float(np.sqrt(np.mean(e * e))), "bound": 1e-5,
                        "within_bound": bool(e.max() <= 1e-5)})
        out[name] = rec
    return out


# Host cores the CPU baseline uses at most: one GPU's share of the host on
# the MI355X machines measured (16 cores per GPU, whatever the host reports
# in total).
CPU_SHARE = 16


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "affinity": affinity}


def cpu_baseline(workloads):
    """The oracle as it is, on the host cores: the headline workload
    (batch_uniform) and the uneven batch in full, one generator per worker
    process on the job's core share; the two single pools in full on one
    thread; the FP64 oracle of the single small pool, whose last pool is kept
    for the precision report."""
    import multiprocessing as mp

    import oracle  # the CPU-baseline leg may use the oracle
    oracle.lib()
    info = host_info()
    cores = max(1, min(CPU_SHARE, info["affinity"]))
    res = {}
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_cpu_warm, range(cores))
        for spec in (workloads.batch_uniform(), workloads.batch_uneven()):
            passes = spec.passes.astype(np.uint64) * spec.launches
            work = spec.nu * passes
            order = np.argsort(-work.astype(np.float64), kind="stable")  # largest first
            args = [(int(spec.seeds[g]), int(spec.n[g]), int(spec.N[g]), int(passes[g]))
                    for g in order]
            t0 = time.perf_counter()
            pool.map(_cpu_one, args, chunksize=max(1, len(args) // (cores * 64)))
            wall = time.perf_counter() - t0
            total = int(work.sum())
            res[spec.name] = {"normals_per_s": total / wall, "normals": total,
                              "wall_s": round(wall, 2),
                              "sample": f"all {spec.G} generators in full, largest first, "
                                        f"one generator per task on {cores} processes"}
    res.update(cpu_single_thread(workloads))
    head = res["batch_uniform"]
    return {"value": head["normals_per_s"], "unit": "normals/s", "cores": cores,
            "kind": "oracle",
            "sample": f"batch_uniform in full ({head['normals']} normals), {head['sample']}, "
                      f"{head['wall_s']} s wall",
            "host": {**info, "core_share": CPU_SHARE},
            "workloads": res}


def cpu_single_thread(workloads):
    """The oracle on one thread of this process: both single pools in full
    (the initial pool not timed), batch_uniform generators one after another,
    and the FP64 oracle of the single small pool (its last pool is kept)."""
    import oracle
    oracle.lib()
    res = {}
    for spec in (workloads.SINGLE_SMALL, workloads.SINGLE_LARGE):
        g = oracle.Gen(spec.seed, spec.n, spec.N)
        t0 = time.perf_counter()
        for _ in range(spec.passes):
            g.fill(spec.nu)  # one pass and its returned pool
        dt = time.perf_counter() - t0
        res[spec.name] = {"normals_per_s": spec.normals / dt, "normals": spec.normals,
                          "wall_s": round(dt, 2),
                          "sample": f"all {spec.passes} passes on 1 thread"}
        PRECISION_REF[f"{spec.name}_fp32_S"] = g.last_S
        PRECISION_REF[f"{spec.name}_fp32_sha"] = hashlib.sha256(g.pool.tobytes()).hexdigest()
        del g
    uni = workloads.batch_uniform()
    passes = 64 * uni.launches
    gens = 64
    t0 = time.perf_counter()
    for s in uni.seeds[:gens]:
        oracle.Gen(int(s), 4, 256).fill(1024 * passes)
    dt = time.perf_counter() - t0
    res["batch_uniform_1thread"] = {"normals_per_s": gens * 1024 * passes / dt,
                                    "sample": f"{gens} of {uni.G} generators, {passes} passes "
                                              "each, initial pools included, 1 thread"}
    spec = workloads.SINGLE_SMALL
    g64 = oracle.Gen64(spec.seed, spec.n, spec.N)
    t0 = time.perf_counter()
    for _ in range(spec.passes):
        g64.fill(spec.nu)
    dt = time.perf_counter() - t0
    res["single_small_fp64"] = {"normals_per_s": spec.normals / dt,
                                "sample": f"FP64 variant, all {spec.passes} passes, 1 thread"}
    PRECISION_REF["single_small_fp64_pool"] = g64.pool
    return res


# FP64 oracle results kept by the CPU-baseline leg for the precision report
PRECISION_REF = {}


def _cpu_warm(_):
    import oracle
    oracle.lib()
    return 0


def _cpu_one(arg):
    import oracle
    seed, n, N, passes = arg
    g = oracle.Gen(seed, n, N)
    for _ in range(passes):
        g.fill(n * N)  # one pass and its returned pool
    return 0


def copy_probe(torch, nbytes):
    """Calibration for the HBM counters: one plain copy of nbytes."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", choices=["headline", "single_small", "single_large", "uneven",
                                       "headline_candidates", "precision_shape", "all"],
                    default="all")
    ap.add_argument("--copy-probe", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the batched generators are independent "
              "(no exchange between pools), so a multi-GPU run would be N copies of this "
              "one; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_1004_3114_amd import workloads

    # the CPU leg runs first, in worker processes started before this
    # process loads the HIP runtime or touches the GPU
    cpu = None
    if args.only == "all" and not args.copy_probe:
        log("cpu baseline (the oracle on the host cores)")
        cpu = cpu_baseline(workloads)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return
    from paper_1004_3114_amd import wallace as W
    W.lib()  # fails loudly if the HIP library is missing
    if args.only in ("single_small", "single_large"):
        which = "small" if args.only == "single_small" else "large"
        print(json.dumps(single_pool(torch, W, workloads, which)), flush=True)
        return
    if args.only == "uneven":
        print(json.dumps(uneven(torch, W, workloads)), flush=True)
        return
    if args.only == "precision_shape":
        print(json.dumps(precision_shape(torch, W, workloads)), flush=True)
        return
    if args.only == "headline_candidates":
        print(json.dumps(headline_candidates(torch, W, workloads)), flush=True)
        return
    value, ms_per_step, roof, cfg = headline(torch, W, workloads, args.steps, args.warmup)
    line = {"metric": "normals/sec at 1 GPU (FP32) + % HBM-write roofline; batched vs single-pool",
            "value": value, "unit": "normals/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic (seeded splitmix64 + Box-Muller initial pools)",
            "config": {"workload": "batch_uniform", **cfg},
            "roofline": roof}
    if args.only == "all":
        small, large = {}, {}
        line["single_pool"] = {
            "single_small": single_pool(torch, W, workloads, "small", keep=small),
            "single_large": single_pool(torch, W, workloads, "large", keep=large)}
        line["batch_uneven"] = uneven(torch, W, workloads)
        line["precision"] = precision_report(small, large)
        line["precision"]["n16_transform"] = precision_shape(torch, W, workloads)
        ceil = store_ceilings(torch)
        line["store_ceilings_GBps"] = ceil
        line["frac_of_store_ceiling"] = {k: round(roof["achieved"] / v, 4) for k, v in ceil.items()}
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
