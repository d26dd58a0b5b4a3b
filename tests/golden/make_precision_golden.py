"""Write precision_n16_oracle.json from the CPU oracle only.

The long-run precision workload: n = 16, N = 2^20, seed 42, 10,000 passes.
For each reduction mode of the sum of squares (FP64 tree, FP32 tree,
compensated FP32 tree) the FP32 oracle's pool is hashed (SHA-256 of its
little-endian bytes) every 1000 passes, with the oracle's sum of squares and
the chi-squared target S of the pass (section 4, eq. 3) as exact hex floats.
The FP64 oracle records its pool at SAMPLE fixed positions every 1000
passes, and its S. Four trajectories in four processes; about 1.5 h on a
2.7 GHz Xeon.

    python tests/golden/make_precision_golden.py            # all four
    python tests/golden/make_precision_golden.py fp32:0     # one, into the file
"""
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SEED, N_COMP, N = 42, 16, 1 << 20
PASSES, EVERY = 10000, 1000
SAMPLE = 256
MODES = {0: "fp64", 1: "fp32", 2: "fp32c"}


def positions():
    # fixed pool positions of the FP64 record: every component, spread over j
    rng = np.random.default_rng(1004)
    return np.sort(rng.choice(N_COMP * N, SAMPLE, replace=False)).astype(np.int64)


def run(kind, mode):
    import oracle
    if kind == "fp64":
        g = oracle.Gen64(SEED, N_COMP, N)
    else:
        g = oracle.Gen(SEED, N_COMP, N, sum_mode=mode)
    pos = positions()
    recs = []
    t0 = time.time()
    for p in range(1, PASSES + 1):
        g.do_pass()
        if p % EVERY:
            continue
        pool = g.pool
        rec = {"pass": p, "S_hex": float(g.last_S).hex(), "sigma_hex": float(g.sigma).hex()}
        if kind == "fp64":
            rec["sample_hex"] = [float(v).hex() for v in pool[pos]]
        else:
            rec["sha256"] = hashlib.sha256(np.ascontiguousarray(pool).tobytes()).hexdigest()
        recs.append(rec)
        print(kind, mode, p, f"{time.time() - t0:.0f}s", flush=True)
    return (kind, mode), recs


def main():
    """Computes every trajectory, or those named on the command line
    (fp32:0, fp32:1, fp32:2, fp64) into the existing file."""
    path = os.path.join(HERE, "precision_n16_oracle.json")
    jobs = [("fp32", 0), ("fp32", 1), ("fp32", 2), ("fp64", 0)]
    if len(sys.argv) > 1:
        jobs = [(a.split(":")[0], int(a.split(":")[1]) if ":" in a else 0) for a in sys.argv[1:]]
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        res = dict(pool.starmap(run, jobs))
    if os.path.exists(path) and len(sys.argv) > 1:
        with open(path) as fh:
            out = json.load(fh)
    else:
        out = {"source": "written by tests/golden/make_precision_golden.py from the CPU oracle "
                         "only",
               "seed": SEED, "n": N_COMP, "N": N, "passes": PASSES, "every": EVERY,
               "sample_positions": [int(v) for v in positions()],
               "fp32_oracle": {}, "fp64_oracle": None}
    for (kind, mode), recs in res.items():
        if kind == "fp64":
            out["fp64_oracle"] = recs
        else:
            out["fp32_oracle"][MODES[mode]] = recs
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
