"""Host-side pin of the near-midpoint inputs used to check the GPU's FP64
divide and square root (tests/test_gpu_devmath.py): every constructed case
really lies within a tiny fraction of an ulp of a rounding midpoint, and the
host's IEEE arithmetic (the oracle's C code and Python floats) rounds it
correctly, by exact rational arithmetic."""
import math
from fractions import Fraction

import numpy as np

import oracle
from tests import near_ties


def _ulp_distance_to_midpoint(exact: Fraction, rounded: float) -> float:
    u = Fraction(math.ulp(rounded))
    return float(abs(abs(exact - Fraction(rounded)) - u / 2) / u)


def test_division_cases_are_near_midpoints_and_host_rounds_them():
    cases = near_ties.division_cases(400, seed=5)
    x = np.zeros(len(cases))
    sigma = np.array([c[0] for c in cases])
    r = np.array([c[1] for c in cases])
    S, c = oracle.chi2_many(x, sigma, r)
    for i, (sg, rr, qexp) in enumerate(cases):
        assert S[i] == (rr * rr) * 0.5
        exact = Fraction(float(S[i])) / Fraction(sg)
        assert _ulp_distance_to_midpoint(exact, qexp) < 2.0 ** -40
        assert float(S[i]) / sg == qexp
        assert near_ties.check_rounding(float(S[i]), sg, qexp, float(c[i]))


def test_sqrt_cases_are_near_midpoints_and_host_rounds_them():
    cases = near_ties.sqrt_cases(400)
    x = np.zeros(len(cases))
    sigma = np.array([c[0] for c in cases])
    r = np.array([c[1] for c in cases])
    S, c = oracle.chi2_many(x, sigma, r)
    below = above = 0
    for i, (sg, rr, cexp) in enumerate(cases):
        q = float(S[i]) / sg
        assert q == float(Fraction(float(S[i])) / Fraction(sg))  # exact quotient
        assert c[i] == cexp
        u = Fraction(math.ulp(cexp))
        mid = Fraction(cexp) + u / 2
        lower_mid = Fraction(cexp) - u / 2
        d = min(abs(Fraction(q) - mid * mid), abs(Fraction(q) - lower_mid * lower_mid))
        assert d / (u * Fraction(cexp)) < Fraction(1, 2 ** 40)
        if Fraction(q) < mid * mid and Fraction(q) > lower_mid * lower_mid:
            below += Fraction(q) > Fraction(cexp) ** 2
            above += Fraction(q) < Fraction(cexp) ** 2
        assert near_ties.check_rounding(float(S[i]), sg, q, float(c[i]))
    assert below > 100 and above > 100
