"""Shared settings of the long-run precision study (n = 16, N = 2^20, seed
42, 10,000 passes): checkpoints, the sampled pool positions compared for
the matrix-core variant, and the error measure. No part of the generator is
computed here."""
import numpy as np

N_COMP = 16
N = 1 << 20
NU = N_COMP * N
SEED = 42
PASSES = 10000
EVERY = 1000
CHECKPOINTS = list(range(EVERY, PASSES + 1, EVERY))
STAT_PASSES = 60          # final passes whose outputs feed the moments and chi^2 (1.007e9)
SAMPLE = 131072           # pool positions kept per checkpoint for the matrix-core runs
REDUCE_MODES = {0: "fp64", 1: "fp32", 2: "fp32c"}
TRANSFORMS = {0: "valu", 1: "mfma"}


def sample_positions() -> np.ndarray:
    return np.sort(np.random.default_rng(20241202).choice(NU, SAMPLE, replace=False))


def variate_error(x32, x64):
    """Per-variate error |x32 - x64| / max(1, |x64|) (relative error is not
    defined near zero): returns (max, rms)."""
    x64 = np.asarray(x64, dtype=np.float64)
    e = np.abs(np.asarray(x32, dtype=np.float64) - x64) / np.maximum(1.0, np.abs(x64))
    return float(e.max()), float(np.sqrt(np.mean(e * e)))
