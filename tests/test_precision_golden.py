"""Consistency of tests/golden/precision_n16_oracle.json (written by
tests/golden/make_precision_golden.py from the oracle only), checked on the
CPU without recomputing the 10,000-pass trajectories:

- every trajectory has a record at every 1000th pass up to 10,000;
- after each pass the pool's sum of squares is the chi-squared target S of
  that pass (section 4, eq. 3): to FP64 rounding for the FP64 oracle, to
  FP32 pool rounding for the FP32 oracle in each reduction mode;
- the FP32 trajectories' targets stay within the FP32-versus-FP64 error of
  the FP64 oracle's (S is (x* + sqrt(2 nu - 1))^2 / 2 with x* one pool
  value, so a per-variate error e moves S by about sqrt(2 nu) e);
- the sampled positions are the script's fixed draw, inside the pool.
"""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "golden", "precision_n16_oracle.json")


@pytest.fixture(scope="module")
def golden():
    with open(PATH) as fh:
        return json.load(fh)


def test_records_at_every_checkpoint(golden):
    want = list(range(golden["every"], golden["passes"] + 1, golden["every"]))
    assert [r["pass"] for r in golden["fp64_oracle"]] == want
    assert set(golden["fp32_oracle"]) == {"fp64", "fp32", "fp32c"}
    for recs in golden["fp32_oracle"].values():
        assert [r["pass"] for r in recs] == want
        assert all(len(r["sha256"]) == 64 for r in recs)
    assert all(len(r["sample_hex"]) == len(golden["sample_positions"]) for r in golden["fp64_oracle"])


def test_sum_of_squares_reaches_chi2_target(golden):
    for r in golden["fp64_oracle"]:
        S, sig = float.fromhex(r["S_hex"]), float.fromhex(r["sigma_hex"])
        assert abs(sig - S) / S <= 1e-13
    for mode, recs in golden["fp32_oracle"].items():
        for r in recs:
            S, sig = float.fromhex(r["S_hex"]), float.fromhex(r["sigma_hex"])
            # FP32 pool values round the scaled sum by a few ulp in relative terms
            assert abs(sig - S) / S <= 1e-6, (mode, r["pass"])


def test_fp32_targets_track_fp64_targets(golden):
    nu = golden["n"] * golden["N"]
    s64 = {r["pass"]: float.fromhex(r["S_hex"]) for r in golden["fp64_oracle"]}
    for mode, recs in golden["fp32_oracle"].items():
        for r in recs:
            S = float.fromhex(r["S_hex"])
            # |dS| ~ sqrt(2 nu) |dx*| with |dx*| well below 1e-4 after 10,000 passes
            assert abs(S - s64[r["pass"]]) <= math.sqrt(2 * nu) * 1e-4, (mode, r["pass"])


def test_sample_positions(golden):
    pos = np.asarray(golden["sample_positions"])
    rng = np.random.default_rng(1004)
    ref = np.sort(rng.choice(golden["n"] * golden["N"], len(pos), replace=False))
    assert np.array_equal(pos, ref)
    assert pos.min() >= 0 and pos.max() < golden["n"] * golden["N"]
