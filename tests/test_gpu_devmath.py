"""The GPU's FP64 arithmetic behind bit-exactness.

The pass kernels compute the chi-squared scale c = sqrt(S / sigma) with
S = (x* + r)^2 / 2 (section 4, eq. 3) and the n = 2 rotation's cos and sin
by divisions (section 8) in FP64 on the GPU, and the FP32 pool depends on
RN32(c). These tests run the very device functions the kernels call
(libwallace_check.so, built from the same header with the same flags) and
compare every result bit with host IEEE arithmetic (the oracle's C code):
about 1e8 random inputs each, plus constructed cases whose quotient or
square root lies within 2^-50 ulp of a rounding midpoint, where an
incorrectly rounded divide or square root shows.
"""
import math

import numpy as np
import pytest

import oracle
from tests import near_ties

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CHUNK = 1 << 24
CHUNKS = 6  # 1.007e8 inputs


def _check():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1004_3114_amd import check
    check.lib()
    return check


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def test_chi2_scale_near_midpoints():
    ck = _check()
    div = near_ties.division_cases(3000)
    sq = near_ties.sqrt_cases(3000)
    cases = div + sq
    sigma = np.array([c[0] for c in cases])
    r = np.array([c[1] for c in cases])
    x = np.zeros(len(cases))
    print(f"case chi2 near midpoints: {len(div)} divisions, {len(sq)} square roots", flush=True)
    S_d = torch.empty(len(cases), dtype=torch.float64, device="cuda")
    q_d = torch.empty_like(S_d)
    c_d = ck.chi2(_dev(x), _dev(sigma), _dev(r), S=S_d, q=q_d)
    S_h, c_h = oracle.chi2_many(x, sigma, r)
    q_h = S_h / sigma
    # the host itself is correctly rounded on these inputs (exact arithmetic)
    for i in range(0, len(cases), 97):
        assert near_ties.check_rounding(float(S_h[i]), float(sigma[i]), float(q_h[i]),
                                        float(c_h[i]))
    qexp = np.array([c[2] for c in div])
    cexp = np.array([c[2] for c in sq])
    assert np.array_equal(_bits(q_h[:len(div)]), _bits(qexp))
    assert np.array_equal(_bits(c_h[len(div):]), _bits(cexp))
    S_g, q_g, c_g = S_d.cpu().numpy(), q_d.cpu().numpy(), c_d.cpu().numpy()
    assert np.array_equal(_bits(S_g), _bits(S_h))
    bad_q = np.nonzero(_bits(q_g) != _bits(q_h))[0]
    bad_c = np.nonzero(_bits(c_g) != _bits(c_h))[0]
    assert bad_q.size == 0, f"{bad_q.size} quotients differ, first {bad_q[:5]}"
    assert bad_c.size == 0, f"{bad_c.size} square roots differ, first {bad_c[:5]}"


def test_chi2_scale_matches_host_on_1e8_inputs():
    # x* an FP32 pool value, nu = 2^k (k = 3..26) with r = RN(sqrt(2 nu - 1)),
    # sigma a sum of squares near nu: the values the pass kernels see
    ck = _check()
    rng = np.random.default_rng(20261203)
    total = 0
    for ch in range(CHUNKS):
        x = rng.standard_normal(CHUNK).astype(np.float32).astype(np.float64)
        k = rng.integers(3, 27, CHUNK)
        nu = np.ldexp(1.0, k)
        r = np.sqrt(2.0 * nu - 1.0)
        sigma = nu * (1.0 + 0.02 * rng.standard_normal(CHUNK))
        S_d = torch.empty(CHUNK, dtype=torch.float64, device="cuda")
        c_d = ck.chi2(_dev(x), _dev(sigma), _dev(r), S=S_d)
        S_h, c_h = oracle.chi2_many(x, sigma, r)
        bad_S = int(np.count_nonzero(_bits(S_d.cpu().numpy()) != _bits(S_h)))
        bad_c = int(np.count_nonzero(_bits(c_d.cpu().numpy()) != _bits(c_h)))
        total += CHUNK
        print(f"chi2 chunk {ch}: {total} inputs, {bad_S} S and {bad_c} c differ", flush=True)
        assert bad_S == 0 and bad_c == 0


def test_rotation_matches_host_on_1e8_draws():
    ck = _check()
    rng = np.random.default_rng(7)
    total = 0
    for ch in range(CHUNKS):
        w = rng.integers(0, np.iinfo(np.int64).max, CHUNK, dtype=np.int64, endpoint=True)
        w ^= rng.integers(0, 2, CHUNK, dtype=np.int64) << 63  # both halves of uint64
        cs_d, sn_d = ck.rotation(_dev(w, torch.int64))
        cs_h, sn_h = oracle.rotation_many(w.view(np.uint64))
        bad = int(np.count_nonzero(_bits(cs_d.cpu().numpy()) != _bits(cs_h)) +
                  np.count_nonzero(_bits(sn_d.cpu().numpy()) != _bits(sn_h)))
        total += CHUNK
        print(f"rotation chunk {ch}: {total} draws, {bad} values differ", flush=True)
        assert bad == 0
    # and the rotation is what section 8 asks: cos^2 + sin^2 = 1, min >= 1/2
    assert np.all(np.minimum(np.abs(cs_h), np.abs(sn_h)) >= 0.5 - 1e-15)
    assert np.max(np.abs(cs_h * cs_h + sn_h * sn_h - 1.0)) < 1e-15
