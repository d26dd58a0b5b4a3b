"""GPU side of the precision study: the library's n = 16, N = 2^20
generator (seed 42) for 10,000 passes in each of the six variants
{butterflies, matrix cores} x {FP64, FP32, compensated FP32 sum of squares}.

At every checkpoint it records the pool's SHA-256 (compared with the FP32
oracle's, which must match bit for bit for the butterfly variants), the
library's sum of squares, the exact sum of squares of the pool, the
chi-squared target S of the pass, and for the matrix-core variants the pool
values at fixed sampled positions. Over the final 60 passes (1.007e9
outputs) of the FP64-sum variants it computes the first four moments and a
100-bin equiprobable chi-squared test.

    python tests/precision/study_gpu.py --out DIR
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from tests.precision import common as C  # noqa: E402

CHUNK = 50  # passes per fill call


def normal_stats(torch, x):
    """Moments and 100-bin equiprobable chi^2 of a float32 CUDA tensor."""
    from scipy.special import ndtri
    M = x.numel()
    xd = x.double()
    ev = {1: 0.0, 2: 1.0, 3: 0.0, 4: 3.0}
    var = {1: 1.0, 2: 2.0, 3: 15.0, 4: 96.0}
    mom = {}
    p = torch.ones_like(xd)
    for k in range(1, 5):
        p = p * xd
        m = p.mean().item()
        mom[f"m{k}"] = m
        mom[f"z{k}"] = (m - ev[k]) / math.sqrt(var[k] / M)
    del p, xd
    edges = torch.tensor(ndtri(np.arange(1, 100) / 100.0), dtype=torch.float64, device=x.device)
    counts = torch.zeros(100, dtype=torch.int64, device=x.device)
    step = 1 << 26
    for i in range(0, M, step):
        idx = torch.bucketize(x[i:i + step].double(), edges)
        counts += torch.bincount(idx, minlength=100)
    counts = counts.cpu().numpy().astype(np.float64)
    E = M / 100.0
    X2 = float(((counts - E) ** 2 / E).sum())
    return {"count": M, **mom, "chi2_100bins": X2, "chi2_dof": 99,
            "chi2_ok": abs(X2 - 99) <= 5 * math.sqrt(198)}


def run_variant(torch, W, tm, rm, outdir, positions):
    r_nu = math.sqrt(2 * C.NU - 1)
    g = W.Generator(C.SEED, C.N_COMP, C.N, reduce_mode=rm, transform_mode=tm)
    buf = torch.empty(C.NU * CHUNK, dtype=torch.float32, device="cuda")
    tag = f"{C.TRANSFORMS[tm]}_{C.REDUCE_MODES[rm]}"
    recs, samples = [], []
    done = 0
    stats = None
    t0 = time.time()
    for cp in C.CHECKPOINTS:
        # the pool after pass cp and the previous pool's last value x*
        final = cp == C.PASSES and rm == 0
        lead = C.STAT_PASSES if final else 2
        while done < cp - lead:
            k = min(CHUNK, cp - lead - done)
            g.fill(buf, C.NU * k)
            done += k
        if final:
            stat_buf = torch.empty(C.NU * C.STAT_PASSES, dtype=torch.float32, device="cuda")
            g.fill(stat_buf)
            done += C.STAT_PASSES
            xstar = float(stat_buf[C.NU * (C.STAT_PASSES - 1) - 1].item())
            stats = normal_stats(torch, stat_buf)
            del stat_buf
        else:
            g.fill(buf, 2 * C.NU)
            done += 2
            xstar = float(buf[C.NU - 1].item())
        pool = g.pool()
        sig_lib, passes = g.sumsq()
        assert passes == cp, (passes, cp)
        t = xstar + r_nu
        S = (t * t) * 0.5
        sq = pool.astype(np.float64) ** 2
        rec = {"pass": cp, "sigma_lib": sig_lib, "S": S, "sigma_exact": math.fsum(sq),
               "sha256": hashlib.sha256(pool.tobytes()).hexdigest()}
        rec["drift"] = abs(rec["sigma_exact"] - S) / S
        recs.append(rec)
        if tm == 1:
            samples.append(pool[positions])
        print(tag, json.dumps(rec), f"{time.time() - t0:.1f}s", flush=True)
    status = g.status()
    del buf, g
    torch.cuda.empty_cache()
    if samples:
        np.save(os.path.join(outdir, f"samples_{tag}.npy"), np.stack(samples))
    return {"variant": tag, "checkpoints": recs, "stats": stats, "status": list(status)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    import torch
    from paper_1004_3114_amd import wallace as W
    W.lib()
    positions = C.sample_positions()
    res = []
    for tm in C.TRANSFORMS:
        for rm in C.REDUCE_MODES:
            print(f"variant transform={C.TRANSFORMS[tm]} reduce={C.REDUCE_MODES[rm]}", flush=True)
            res.append(run_variant(torch, W, tm, rm, args.out, positions))
            with open(os.path.join(args.out, "precision_gpu.json"), "w") as fh:
                json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
