"""Statistical checks of the oracle's output stream (section 8 of the paper).

Moments within 5 sigma, a 100-bin chi-squared test against the normal CDF,
and the paper's (u, v) test: for a pair (x, y) of N(0,1) values,
u = exp(-(x^2 + y^2)/2) is uniform on [0, 1] and v = arctan(x / y) is uniform
on [-pi/2, pi/2]; 1000 equal bins give a chi-squared statistic with 999
degrees of freedom.
"""
import math

import numpy as np
import pytest
from scipy.special import ndtr

import oracle


def _moments_ok(x):
    M = x.size
    x = x.astype(np.float64)
    z = [x.mean() / math.sqrt(1 / M),
         ((x ** 2).mean() - 1) / math.sqrt(2 / M),
         (x ** 3).mean() / math.sqrt(15 / M),
         ((x ** 4).mean() - 3) / math.sqrt(96 / M)]
    return z


def _chi2_normal_100(x):
    # 100 equiprobable cells of N(0,1): edges where Phi = i/100.
    edges = np.empty(101)
    edges[0], edges[-1] = -np.inf, np.inf
    for i in range(1, 100):
        lo, hi = -10.0, 10.0
        for _ in range(200):  # bisection on Phi
            mid = 0.5 * (lo + hi)
            if ndtr(mid) < i / 100:
                lo = mid
            else:
                hi = mid
        edges[i] = 0.5 * (lo + hi)
    counts, _ = np.histogram(x, bins=edges)
    e = x.size / 100
    return ((counts - e) ** 2 / e).sum()


def _chi2_uniform(u, lo, hi, bins=1000):
    counts, _ = np.histogram(u, bins=bins, range=(lo, hi))
    e = u.size / bins
    return ((counts - e) ** 2 / e).sum()


@pytest.mark.parametrize("n,N,passes", [(4, 1024, 1000), (16, 4096, 64), (2, 2048, 1000)])
def test_moments_and_chi2(n, N, passes):
    x = oracle.Gen(42, n, N).fill(n * N * passes)
    z = _moments_ok(x)
    assert all(abs(v) < 5 for v in z), z
    X2 = _chi2_normal_100(x)
    assert abs(X2 - 99) <= 5 * math.sqrt(2 * 99), X2


def test_paper_uv_test():
    x = oracle.Gen(7, 4, 1 << 14).fill(1 << 22).astype(np.float64)
    p, q = x[0::2], x[1::2]
    u = np.exp(-(p * p + q * q) / 2)
    v = np.arctan(p / q)
    for X2 in (_chi2_uniform(u, 0.0, 1.0), _chi2_uniform(v, -math.pi / 2, math.pi / 2)):
        assert abs(X2 - 999) <= 5 * math.sqrt(2 * 999), X2


def test_stats_detect_a_broken_generator():
    # The battery must reject a plausible mistake: dropping the chi-squared
    # rescaling leaves every pool with the same sum of squares, and a pool of
    # fixed norm whose entries all have magnitude 1 fails the chi2 test.
    x = np.tile(np.array([1.0, -1.0, 1.0, 1.0]), 4096)
    assert abs(_chi2_normal_100(x) - 99) > 5 * math.sqrt(198)
