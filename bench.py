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
    log(f"init {time.time() - t0:.1f}s; output {total * 4 / 2**30:.0f} GiB")
    out = torch.empty(total, dtype=torch.float32, device="cuda")
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
            "kernel": "k_pool<4,4> (n=4, T=4 tuples/lane, L=64 lanes/pool)",
            "alg_bytes_per_launch": int(alg_bytes), "avg_launch_ms": round(launch_ms, 4),
            "kernel_source_hash": khash}
    del graph, out
    torch.cuda.empty_cache()
    return value, ms_per_step, roof, {"G": spec.G, "n": 4, "N": 256, "passes_per_launch": 64,
                                      "launches_per_step": spec.launches,
                                      "normals_per_step": total}


def single_pool(torch, W, workloads, which, reps=3):
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
    t0 = time.time()
    b.tune()  # per (n, N) class: the fastest pool-resident schedule
    log(f"batch_uneven tuned in {time.time() - t0:.1f}s")
    b.plan(spec.offsets(), spec.passes)
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    b.fill(out)
    ms = min(timed_events(torch, stream, lambda: b.fill(out), reps))
    del out, b
    torch.cuda.empty_cache()
    rate = total / (ms * 1e-3)
    return {"workload": "batch_uneven", "G": spec.G, "normals": total, "ms": round(ms, 3),
            "normals_per_s": rate, "write_GBps": round(rate * 4 / 1e9, 1),
            "frac_hbm": round(rate * 4 / 1e9 / HBM_PEAK_GBPS, 4)}


def store_ceiling(torch, nbytes=16 << 30, reps=5):
    """Plain streaming-store reference on the same GPU (torch fill kernel)."""
    t = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    t.fill_(1.0)
    ms = min(timed_events(torch, stream, lambda: t.fill_(0.5), reps))
    del t
    torch.cuda.empty_cache()
    return round(nbytes / (ms * 1e-3) / 1e9, 1)


def cpu_baseline(workloads, budget_s=12.0):
    """The oracle as it is, one generator per worker process, on a bounded
    sample of the batched uniform workload (full 256 passes per generator)."""
    import multiprocessing as mp

    import oracle  # the CPU-baseline leg may use the oracle
    oracle.lib()
    cores = max(1, min(16, os.cpu_count() or 1))
    spec = workloads.batch_uniform()
    passes = 64 * spec.launches
    per_gen = 1024 * passes
    chunk = cores * 4
    done = 0
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        g0 = 0
        while time.perf_counter() - t0 < budget_s and g0 < spec.G:
            seeds = [int(s) for s in spec.seeds[g0:g0 + chunk]]
            pool.map(_cpu_one, [(s, passes) for s in seeds])
            done += len(seeds)
            g0 += chunk
    wall = time.perf_counter() - t0
    return {"value": done * per_gen / wall, "unit": "normals/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{done} of {spec.G} batch_uniform generators (n=4, N=256, seeds 42+g), "
                      f"{passes} passes each = {done * per_gen} normals, one generator per "
                      f"process on {cores} processes, {wall:.1f} s wall",
            "single_thread": cpu_single_thread(workloads)}


def cpu_single_thread(workloads):
    """The oracle on one thread of this process: the single small pool in
    full, the single large pool on a sample of its passes (its initial pool
    not timed), and batch_uniform generators one after another."""
    import oracle
    oracle.lib()
    res = {}
    for spec, sample_passes in ((workloads.SINGLE_SMALL, None), (workloads.SINGLE_LARGE, 5)):
        P = spec.passes if sample_passes is None else sample_passes
        g = oracle.Gen(spec.seed, spec.n, spec.N)
        t0 = time.perf_counter()
        g.fill(spec.n * spec.N * P)
        dt = time.perf_counter() - t0
        res[spec.name] = {"normals_per_s": spec.n * spec.N * P / dt,
                          "sample": f"{P} of {spec.passes} passes"}
    uni = workloads.batch_uniform()
    passes = 64 * uni.launches
    gens = 64
    t0 = time.perf_counter()
    for s in uni.seeds[:gens]:
        oracle.Gen(int(s), 4, 256).fill(1024 * passes)
    dt = time.perf_counter() - t0
    res["batch_uniform"] = {"normals_per_s": gens * 1024 * passes / dt,
                            "sample": f"{gens} of {uni.G} generators, {passes} passes each, "
                                      "initial pools included"}
    return res


def _cpu_one(arg):
    import oracle
    seed, passes = arg
    g = oracle.Gen(seed, 4, 256)
    g.fill(1024 * passes)
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
    ap.add_argument("--only", choices=["headline", "single_small", "single_large", "uneven", "all"],
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
        log("cpu baseline (oracle, bounded sample)")
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
    value, ms_per_step, roof, cfg = headline(torch, W, workloads, args.steps, args.warmup)
    line = {"metric": "normals/sec at 1 GPU (FP32) + % HBM-write roofline; batched vs single-pool",
            "value": value, "unit": "normals/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic (seeded splitmix64 + Box-Muller initial pools)",
            "config": {"workload": "batch_uniform", **cfg},
            "roofline": roof}
    if args.only == "all":
        line["single_pool"] = {"single_small": single_pool(torch, W, workloads, "small"),
                               "single_large": single_pool(torch, W, workloads, "large")}
        line["batch_uneven"] = uneven(torch, W, workloads)
        line["store_ceiling_GBps"] = store_ceiling(torch)
        line["frac_of_store_ceiling"] = round(roof["achieved"] / line["store_ceiling_GBps"], 4)
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
