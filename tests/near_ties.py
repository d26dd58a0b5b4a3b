"""Inputs of the chi-squared scale c = sqrt(S / sigma) (section 4, eq. 3)
whose FP64 quotient or square root lies extremely close to a rounding
midpoint: the cases where a divide or square root that is not correctly
rounded gives the other neighbour. Built with integer arithmetic, so the
correctly rounded results are known exactly.

Every case is (x*, sigma, r) with x* = 0, so S = RN(r * r) / 2; the scale
functions then see S / sigma and its square root.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _sqrt_mod_pow2(x: int, k: int) -> int:
    """An odd y with y*y = x (mod 2^k), for x = 1 (mod 8) (Hensel lifting)."""
    assert x % 8 == 1
    y = 1
    for i in range(3, k):
        if (y * y - x) % (1 << (i + 1)):
            y += 1 << (i - 1)
    assert (y * y - x) % (1 << k) == 0
    return y


def _as_target(S: float):
    """An r with RN(r*r) * 0.5 == S exactly (so x* = 0, r gives target S),
    or None."""
    r = math.sqrt(2.0 * S)
    for cand in (r, math.nextafter(r, 0.0), math.nextafter(r, math.inf)):
        if (cand * cand) * 0.5 == S:
            return cand
    return None


def division_cases(count: int, seed: int = 1):
    """(sigma, r, q_expected) where S / sigma is within 2^-52 of a midpoint
    between two doubles (just below or just above it, alternately)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        b = int(rng.integers(1 << 52, 1 << 53)) | 1
        for sign in (1, -1):
            inv = pow(b, -1, 1 << 54)
            m = inv if sign > 0 else (-inv) % (1 << 54)
            if m < (1 << 53):
                continue  # m must have 54 bits: a midpoint of 53-bit values
            num = b * m - sign  # = T 2^54: a / b = m - sign / b
            T = num >> 54
            if num % (1 << 54) or T >= (1 << 53):
                continue
            # S = T 2^e1 and sigma = b 2^e2, scaled to S ~ 2^20, S / sigma ~ 1
            e1 = 20 - T.bit_length()
            e2 = 20 - b.bit_length()
            S = math.ldexp(float(T), e1)
            sigma = math.ldexp(float(b), e2)
            r = _as_target(S)
            if r is None:
                continue
            # correctly rounded quotient: m - 1 (below the midpoint) or m + 1
            qexp = math.ldexp(float(m - sign), e1 - e2 - 54)
            exact = Fraction(S) / Fraction(sigma)
            other = math.ldexp(float(m + sign), e1 - e2 - 54)
            assert abs(Fraction(qexp) - exact) < abs(Fraction(other) - exact)
            out.append((sigma, r, qexp))
    return out[:count]


def sqrt_cases(count: int):
    """(sigma, r, c_expected) where S / sigma is exact and its square root
    lies within 2^-50 of a midpoint (below it for r = 1 mod 8, above it for
    r = 7 mod 8)."""
    out = []
    j = 0
    while len(out) < count:
        for resid, sign in ((1 + 8 * j, 1), (7 + 8 * j, -1)):
            # M^2 = Q 2^55 + resid (sign +1) or Q 2^55 + 2^55 - resid (sign -1)
            target = resid if sign > 0 else (1 << 55) - resid
            y = _sqrt_mod_pow2(target, 55)
            M = None
            for cand in (y, (1 << 55) - y, (y + (1 << 54)) % (1 << 55),
                         ((1 << 55) - y + (1 << 54)) % (1 << 55)):
                if (1 << 53) <= cand < (1 << 54) and cand % 2 == 1:
                    M = cand
                    break
            if M is None:
                continue
            sq = M * M
            Q = (sq - resid) >> 55 if sign > 0 else (sq + resid) >> 55
            if Q >= (1 << 53):
                continue
            # q = Q 2^55 = M^2 -/+ resid; scale by 2^-2s so q ~ 1..4, then
            # S = q 2^20 and sigma = 2^20
            s = 54
            q = math.ldexp(float(Q), 55 - 2 * s)
            S = math.ldexp(q, 20)
            sigma = math.ldexp(1.0, 20)
            r = _as_target(S)
            if r is None:
                continue
            cexp = math.ldexp(float(M - sign), -s)  # sqrt just below/above M
            out.append((sigma, r, cexp))
        j += 1
    return out[:count]


def check_rounding(S: float, sigma: float, q: float, c: float) -> bool:
    """True if q = RN(S / sigma) and c = RN(sqrt(q)), by exact arithmetic."""
    exact = Fraction(S) / Fraction(sigma)
    lo, hi = math.nextafter(q, -math.inf), math.nextafter(q, math.inf)
    if not (abs(Fraction(q) - exact) < abs(Fraction(lo) - exact) and
            abs(Fraction(q) - exact) < abs(Fraction(hi) - exact)):
        return False
    qq = Fraction(q)
    lo, hi = math.nextafter(c, 0.0), math.nextafter(c, math.inf)
    mid_lo = (Fraction(lo) + Fraction(c)) / 2
    mid_hi = (Fraction(c) + Fraction(hi)) / 2
    return mid_lo * mid_lo < qq < mid_hi * mid_hi
