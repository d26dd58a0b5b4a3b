"""Oracle side of the precision study (runs on the CPU, no GPU).

Four trajectories in parallel processes: the FP32 oracle with each
reduction mode, and the FP64 oracle. At every checkpoint the pool is saved
to --dir (FP32 64 MB, FP64 128 MB), with its SHA-256, the generator's sum
of squares, the exact sum of squares of the pool and the chi-squared target
S of the pass that produced it.

    python tests/precision/study_cpu.py --dir /some/scratch
"""
import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from tests.precision import common as C  # noqa: E402


def run(kind, mode, outdir):
    import oracle
    g = oracle.Gen64(C.SEED, C.N_COMP, C.N) if kind == "fp64" else \
        oracle.Gen(C.SEED, C.N_COMP, C.N, sum_mode=mode)
    tag = "fp64" if kind == "fp64" else "fp32_" + C.REDUCE_MODES[mode]
    log = []
    t0 = time.time()
    done = 0
    for cp in C.CHECKPOINTS:
        while done < cp:
            g.do_pass()
            done += 1
        pool = g.pool
        np.save(os.path.join(outdir, f"{tag}_{cp}.npy"), pool)
        sq = pool.astype(np.float64) ** 2
        rec = {"pass": cp, "sigma": g.sigma, "S": g.last_S, "sigma_exact": math.fsum(sq),
               "sha256": hashlib.sha256(pool.tobytes()).hexdigest() if kind != "fp64" else None,
               "elapsed_s": time.time() - t0}
        log.append(rec)
        print(tag, json.dumps(rec), flush=True)
    with open(os.path.join(outdir, f"{tag}.json"), "w") as fh:
        json.dump(log, fh, indent=1)
    return tag


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", required=True)
    args = ap.parse_args()
    os.makedirs(args.dir, exist_ok=True)
    jobs = [("fp64", 0)] + [("fp32", m) for m in C.REDUCE_MODES]
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        print(pool.starmap(run, [(k, m, args.dir) for k, m in jobs]))


if __name__ == "__main__":
    main()
