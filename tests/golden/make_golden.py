"""Write oracle_stream_heads.json from the CPU oracle only.

The file freezes the head of the oracle's output stream for a few seeds and
shapes, so that any later change to the oracle's arithmetic shows up in a test
and has to be made on purpose. Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

CASES = [
    {"seed": 42, "n": 4, "N": 1024, "passes": 1000},
    {"seed": 42, "n": 4, "N": 256, "passes": 64},
    {"seed": 7, "n": 16, "N": 64, "passes": 200},
    {"seed": 42, "n": 16, "N": 16, "passes": 50},
]


def record(case):
    g = oracle.Gen(case["seed"], case["n"], case["N"])
    nu = case["n"] * case["N"]
    x = g.fill(nu * case["passes"])
    head = x[:32].view(np.uint32)
    tail = x[-32:].view(np.uint32)
    return dict(case, head_bits=[f"{int(v):08x}" for v in head],
                tail_bits=[f"{int(v):08x}" for v in tail],
                sigma_hex=float(g.sigma).hex(), rng=str(g.rng))


def main():
    out = {"source": "written by tests/golden/make_golden.py from the CPU oracle only",
           "cases": [record(c) for c in CASES]}
    with open(os.path.join(HERE, "oracle_stream_heads.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
