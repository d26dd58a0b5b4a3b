"""Merge the two sides of the precision study into one report.

    python tests/precision/report.py --cpu-dir DIR --gpu-dir DIR --out FILE.json

For each checkpoint (every 1000 passes) and reduction mode:
  - whether the GPU butterfly run's pool is bit-identical to the FP32
    oracle's (SHA-256 of the pool);
  - the per-variate error of the FP32 pool against the FP64 oracle, over the
    whole pool (valid for the GPU butterfly runs when the hashes match) and
    over the sampled positions (the matrix-core runs);
  - the sum-of-squares drift |sum(y^2) - S| / S of the GPU pool and the
    error of the library's own sum of squares.
Prints a markdown table of the same figures.
"""
import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from tests.precision import common as C  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cpu-dir", required=True)
    ap.add_argument("--gpu-dir", required=True)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    gpu = {r["variant"]: r for r in json.load(open(os.path.join(args.gpu_dir, "precision_gpu.json")))}
    cpu = {}
    for tag in ["fp64"] + ["fp32_" + m for m in C.REDUCE_MODES.values()]:
        cpu[tag] = {r["pass"]: r for r in json.load(open(os.path.join(args.cpu_dir, f"{tag}.json")))}
    pos = C.sample_positions()
    samples = {m: np.load(os.path.join(args.gpu_dir, f"samples_mfma_{m}.npy"))
               for m in C.REDUCE_MODES.values()}
    rows = []
    for ci, cp in enumerate(C.CHECKPOINTS):
        x64 = np.load(os.path.join(args.cpu_dir, f"fp64_{cp}.npy"))
        for m in C.REDUCE_MODES.values():
            x32 = np.load(os.path.join(args.cpu_dir, f"fp32_{m}_{cp}.npy"))
            g_valu = gpu[f"valu_{m}"]["checkpoints"][ci]
            g_mfma = gpu[f"mfma_{m}"]["checkpoints"][ci]
            assert g_valu["pass"] == cp and g_mfma["pass"] == cp
            e_max, e_rms = C.variate_error(x32, x64)
            s_max, s_rms = C.variate_error(x32[pos], x64[pos])
            m_max, m_rms = C.variate_error(samples[m][ci], x64[pos])
            rows.append({
                "pass": cp, "reduce": m,
                "valu_bit_exact_vs_fp32_oracle": g_valu["sha256"] == cpu["fp32_" + m][cp]["sha256"],
                "valu_err_max": e_max, "valu_err_rms": e_rms,
                "valu_err_max_sampled": s_max, "valu_err_rms_sampled": s_rms,
                "mfma_err_max_sampled": m_max, "mfma_err_rms_sampled": m_rms,
                "valu_sigma_drift": g_valu["drift"], "mfma_sigma_drift": g_mfma["drift"],
                "valu_sigma_lib_err": abs(g_valu["sigma_lib"] - g_valu["sigma_exact"]) / g_valu["sigma_exact"],
                "mfma_sigma_lib_err": abs(g_mfma["sigma_lib"] - g_mfma["sigma_exact"]) / g_mfma["sigma_exact"],
            })
            print(cp, m, "done", flush=True)
    stats = {v: gpu[v]["stats"] for v in gpu if gpu[v]["stats"]}
    res = {"config": {"n": C.N_COMP, "N": C.N, "seed": C.SEED, "passes": C.PASSES,
                      "sampled_positions": C.SAMPLE},
           "checkpoints": rows, "final_stats": stats,
           "status": {v: gpu[v]["status"] for v in gpu}}
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print("| pass | Σ mode | butterflies = FP32 oracle | butterflies max e / RMS e | "
          "matrix cores max e / RMS e (sampled) | Σ drift (butterflies / matrix) | "
          "library Σ rel. error |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['pass']} | {r['reduce']} | {'yes' if r['valu_bit_exact_vs_fp32_oracle'] else 'NO'} | "
              f"{r['valu_err_max']:.2e} / {r['valu_err_rms']:.2e} | "
              f"{r['mfma_err_max_sampled']:.2e} / {r['mfma_err_rms_sampled']:.2e} | "
              f"{r['valu_sigma_drift']:.1e} / {r['mfma_sigma_drift']:.1e} | "
              f"{r['valu_sigma_lib_err']:.1e} |")


if __name__ == "__main__":
    main()
