"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks one oracle function against something other than the oracle
itself: published test vectors, brute force on tiny inputs, closed forms,
exact invariants, or hand-derived worked examples under tests/golden/.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------------------
# Uniform source: splitmix64 against its published vectors
# ---------------------------------------------------------------------------

def test_splitmix64_published_vectors():
    g = _golden("splitmix64_vectors.json")
    s = 1234567
    got = []
    for _ in range(5):
        s, z = oracle.splitmix64(s)
        got.append(str(z))
    assert got == g["seed_1234567_first5"]
    _, z0 = oracle.splitmix64(0)
    assert z0 == int(g["seed_0_first"], 16)


def test_splitmix64_published_bucket_counts():
    g = _golden("splitmix64_vectors.json")
    s = 987654321
    counts = [0] * 5
    for _ in range(100000):
        s, z = oracle.splitmix64(s)
        counts[(z * 5) >> 64] += 1
    assert counts == g["seed_987654321_buckets5_of_100000"]


# ---------------------------------------------------------------------------
# Strides and offsets (eq. 1, eq. 2, sections 3 and 8)
# ---------------------------------------------------------------------------

def test_stride_pairs_start_with_rann4_sets():
    # Section 8: alpha in {3, 5}, beta in {7, 11}.
    assert oracle.stride_pair(0) == (3, 5)
    assert oracle.stride_pair(1) == (7, 11)


def test_stride_pairs_odd_distinct_greater_than_one():
    # Sections 3 and 7: strides odd, distinct and greater than 1.
    flat = [x for k in range(16) for x in oracle.stride_pair(k)]
    assert len(set(flat)) == 32
    assert all(x % 2 == 1 and x > 1 for x in flat)
    for x in flat:
        assert all(x % d for d in range(2, int(math.isqrt(x)) + 1))


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32, 64])
def test_affine_index_map_is_permutation_iff_gcd_one(N):
    # eq. 2 by brute force: j -> (a j + b) mod N is a bijection exactly when
    # GCD(a, N) = 1, i.e. for every odd a when N is a power of two.
    for a in range(N):
        for b in range(N):
            image = {(a * j + b) % N for j in range(N)}
            assert (len(image) == N) == (math.gcd(a, N) == 1)


def _draw_tops(state, n):
    """Top bits of the n component draws of one pass (oracle.splitmix64 is
    pinned against the published vectors above)."""
    tops = []
    for _ in range(n):
        state, w = oracle.splitmix64(state)
        tops.append(w >> 63)
    return tops


@pytest.mark.parametrize("n,N", [(4, 4), (4, 8), (4, 16), (4, 256), (16, 16), (16, 32),
                                 (16, 64), (16, 128), (16, 1024), (4, 1 << 22), (2, 4),
                                 (2, 8)])
@pytest.mark.parametrize("a_mode", [oracle.A_PAIRS, oracle.A_FULL_ODD])
def test_pass_params_ranges(n, N, a_mode):
    # Strides odd (eq. 2), above one and distinct (sections 3, 6, 9) as far
    # as the N/2 - 1 odd residues above one allow; a table stride that is
    # already acceptable is kept as drawn.
    s = 99
    seen_hi = [set() for _ in range(n)]
    free_odd = N // 2 - 1
    for _ in range(300):
        tops = _draw_tops(s, n)
        a, b, signs, s = oracle.pass_params(s, n, N, a_mode)
        assert signs == 0 if n != 16 else signs < (1 << 16)
        assert np.all(a % 2 == 1) and np.all(a < N) and np.all(b < N)
        assert np.all(a > 1)
        m = min(n, free_odd)
        assert len(set(int(x) for x in a[:m])) == m
        if a_mode == oracle.A_PAIRS:
            for k in range(n):
                drawn = oracle.stride_pair(k)[tops[k]] % N
                if drawn > 1 and (k >= free_odd or drawn not in a[:k]):
                    assert a[k] == drawn
                if N > 137:
                    assert a[k] == oracle.stride_pair(k)[tops[k]]
                seen_hi[k].add(int(a[k]))
    if a_mode == oracle.A_PAIRS and N > 137:
        assert all(len(x) == 2 for x in seen_hi)  # both members get picked


@pytest.mark.parametrize("n", [2, 4, 16])
def test_strides_above_one_and_distinct_for_every_pool_size(n):
    # Every N the library accepts for this n (N >= n, N >= 4): over many
    # passes no stride is 1 and the first min(n, N/2 - 1) strides of a pass
    # differ; from N = 256 on the strides are the table's primes unchanged.
    for logN in range(2, 25 if n != 16 else 23):
        N = 1 << logN
        if N < n:
            continue
        s = 1234 + logN
        for _ in range(64):
            tops = _draw_tops(s, n)
            a, _, _, s = oracle.pass_params(s, n, N)
            assert np.all(a > 1) and np.all(a % 2 == 1)
            m = min(n, N // 2 - 1)
            assert len(set(int(x) for x in a[:m])) == m, (n, N, a)
            if N >= 256:
                assert [int(x) for x in a] == [oracle.stride_pair(k)[tops[k]] for k in range(n)]


def test_pass_params_consume_one_draw_per_component():
    s0 = 12345
    _, _, _, s = oracle.pass_params(s0, 16, 64)
    assert s == (s0 + 16 * 0x9E3779B97F4A7C15) % (1 << 64)


def test_offsets_uniform():
    # Section 8: offsets uniform on {0..N-1}. Chi-squared over 16 cells.
    s = 7
    N = 16
    counts = np.zeros(N)
    for _ in range(4000):
        _, b, _, s = oracle.pass_params(s, 4, N)
        np.add.at(counts, b.astype(int), 1)
    expect = counts.sum() / N
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 15 + 5 * math.sqrt(30)


# ---------------------------------------------------------------------------
# Matrices: orthogonal, rows with at least two non-small entries (section 3)
# ---------------------------------------------------------------------------

def _sylvester(n):
    H = np.array([[1]])
    while H.shape[0] < n:
        H = np.kron(H, np.array([[1, 1], [1, -1]]))
    return H


def test_sylvester_hadamard_matches_library():
    # the Hadamard matrices behind A0 and H16 (section 3), against scipy's
    # Sylvester construction
    import scipy.linalg
    for n in (2, 4, 16):
        assert np.array_equal(_sylvester(n), scipy.linalg.hadamard(n))
    assert np.array_equal(oracle.matrix(16, 0) * 4.0, scipy.linalg.hadamard(16))
    assert np.array_equal(oracle.matrix(4, 0) * 2.0, scipy.linalg.hadamard(4))


def _expected_matrix(n, mat):
    if n == 4 and mat == 1:
        return 0.5 * np.ones((4, 4)) - np.eye(4)
    return _sylvester(n) / math.sqrt(n)


@pytest.mark.parametrize("n,mat", [(4, 0), (4, 1), (16, 0)])
def test_dense_matrix_definition_and_orthogonality(n, mat):
    M = oracle.matrix(n, mat)
    assert np.array_equal(M, _expected_matrix(n, mat))
    assert np.array_equal(M @ M.T, np.eye(n))  # exact in binary
    for row in M:
        nz = np.abs(row[row != 0])
        assert nz.size >= 2 and nz.min() >= 0.25


def test_a0_a1_generate_a_finite_group():
    # The paper's footnote asks for multiplicatively independent matrices;
    # A0 and A1 are involutions and A0 A1 has order 6 (a dihedral group of
    # order 12). This records that reading; the per-pass permutations carry
    # the mixing.
    A0, A1 = oracle.matrix(4, 0), oracle.matrix(4, 1)
    assert np.array_equal(A0 @ A0, np.eye(4))
    assert np.array_equal(A1 @ A1, np.eye(4))
    P = A0 @ A1
    Q = np.eye(4)
    orders = []
    for m in range(1, 13):
        Q = Q @ P
        if np.allclose(Q, np.eye(4), atol=1e-12):
            orders.append(m)
    assert orders[0] == 6


# ---------------------------------------------------------------------------
# One pass: brute-force impulse responses pin gather, matrix and write-back
# ---------------------------------------------------------------------------

def _preimage(a, b, x, N):
    hits = [j for j in range(N) if (a * j + b) % N == x]
    assert len(hits) == 1
    return hits[0]


@pytest.mark.parametrize("n,N,mat", [(4, 8, 0), (4, 8, 1), (4, 32, 0),
                                     (4, 32, 1), (16, 4, 0), (16, 16, 0)])
def test_pass32_impulse_response(n, N, mat):
    # eq. 1: new tuple j takes component k from old X_k[(a_k j + b_k) mod N].
    # An impulse at X_k[x] must land in exactly one new tuple, j*, carrying
    # column k of the matrix (h folds in the 1/2 or 1/4 factor; for n = 16
    # the column is negated when bit k of the sign mask is set).
    rng = np.random.default_rng(n * 1000 + N + mat)
    A = _expected_matrix(n, mat)
    h = np.float32(0.5 if n == 4 else 0.25)
    for _ in range(3):
        a = (rng.integers(0, N, size=n) | 1).astype(np.uint32)
        b = rng.integers(0, N, size=n).astype(np.uint32)
        signs = int(rng.integers(0, 1 << 16)) if n == 16 else 0
        for k in range(n):
            for x in range(N):
                X = np.zeros(n * N, dtype=np.float32)
                X[k * N + x] = 1.0
                Y = oracle.pass32(n, N, mat, a, b, h, X, signs).reshape(n, N)
                js = _preimage(int(a[k]), int(b[k]), x, N)
                expect = np.zeros((n, N))
                expect[:, js] = A[:, k] * (-1.0 if (signs >> k) & 1 else 1.0)
                assert np.array_equal(Y.astype(np.float64), expect)
                Z = oracle.pass64(n, N, mat, a, b, 1.0,
                                  X.astype(np.float64), signs).reshape(n, N)
                assert np.array_equal(Z, expect)


@pytest.mark.parametrize("n,N,mat", [(4, 64, 0), (4, 64, 1), (16, 32, 0)])
def test_pass32_equals_dense_product_on_dyadic_inputs(n, N, mat):
    # With dyadic inputs every partial sum is exact, so the FP32 butterfly
    # order must reproduce the dense FP64 product bit for bit.
    rng = np.random.default_rng(5)
    X = (rng.integers(-64, 65, size=n * N) / 8.0).astype(np.float32)
    a = (rng.integers(0, N, size=n) | 1).astype(np.uint32)
    b = rng.integers(0, N, size=n).astype(np.uint32)
    h = np.float32(0.5 if n == 4 else 0.25)
    signs = 0xA5C3 if n == 16 else 0
    Y32 = oracle.pass32(n, N, mat, a, b, h, X, signs)
    Y64 = oracle.pass64(n, N, mat, a, b, 1.0, X.astype(np.float64), signs)
    assert np.array_equal(Y32.astype(np.float64), Y64)


@pytest.mark.parametrize("n,N,mat", [(4, 256, 0), (4, 256, 1), (16, 256, 0)])
def test_pass_preserves_sum_of_squares_when_unscaled(n, N, mat):
    # Section 2: an orthogonal A keeps the sum of squares, up to rounding.
    rng = np.random.default_rng(11)
    X = rng.standard_normal(n * N).astype(np.float32)
    a = (rng.integers(0, N, size=n) | 1).astype(np.uint32)
    b = rng.integers(0, N, size=n).astype(np.uint32)
    h = np.float32(0.5 if n == 4 else 0.25)
    Y = oracle.pass32(n, N, mat, a, b, h, X)
    s0, s1 = oracle.sumsq_f64(X), oracle.sumsq_f64(Y)
    assert abs(s1 - s0) <= 8 * 2.0 ** -24 * s0
    # every old value is used exactly once: the multiset of |values| of the
    # gathered tuples is the old pool (checked via the impulse test), and the
    # pass is not a per-tuple map (per-component permutations mix tuples)
    norms_old = np.sort((X.reshape(n, N) ** 2).sum(0))
    norms_new = np.sort((Y.reshape(n, N) ** 2).sum(0))
    assert not np.allclose(norms_old, norms_new, rtol=1e-3)


# ---------------------------------------------------------------------------
# Sum of squares: canonical tree against exact sums and worked examples
# ---------------------------------------------------------------------------

def test_canonical_tree_worked_examples():
    g = _golden("canonical_tree.json")
    c0, c1, c2 = g["cases"]
    y = np.array(c0["y"], dtype=np.float32)
    assert oracle.sumsq_f64(y) == float(int(c0["f64_tree"]))
    y = np.array(c1["y"], dtype=np.float32)
    assert float(oracle.sumsq_f32(y)) == float(int(c1["f32_tree"]))
    y = np.array(c2["y"], dtype=np.float32)
    assert oracle.sumsq_f32c(y) == float(int(c2["f32c_tree"]))


@pytest.mark.parametrize("nu", [2, 16, 1024, 4096])
def test_sumsq_within_error_bound_of_exact(nu):
    rng = np.random.default_rng(nu)
    y = (rng.standard_normal(nu) * np.exp(rng.uniform(-3, 3, nu))).astype(np.float32)
    exact = sum(Fraction(float(v)) ** 2 for v in y)
    levels = int(math.log2(nu))
    t64 = Fraction(oracle.sumsq_f64(y))
    assert abs(t64 - exact) <= Fraction(levels * 2.0 ** -53) * exact
    t32 = Fraction(float(oracle.sumsq_f32(y)))
    assert abs(t32 - exact) <= Fraction((levels + 1) * 2.0 ** -24) * exact
    tc = Fraction(oracle.sumsq_f32c(y))
    assert abs(tc - exact) <= Fraction(2.0 ** -40) * exact
    td = Fraction(oracle.sumsq_d(y.astype(np.float64)))
    assert abs(td - exact) <= Fraction(levels * 2.0 ** -53) * exact


def test_sumsq_tree_is_aligned_block_decomposable():
    # The canonical tree over a power-of-two block is the join of the trees
    # over its two halves.
    rng = np.random.default_rng(3)
    y = rng.standard_normal(4096).astype(np.float32)
    assert oracle.sumsq_f64(y) == oracle.sumsq_f64(y[:2048]) + oracle.sumsq_f64(y[2048:])
    assert oracle.sumsq_f32(y) == np.float32(oracle.sumsq_f32(y[:2048]) + oracle.sumsq_f32(y[2048:]))


# ---------------------------------------------------------------------------
# Chi-squared rescaling (section 4, eq. 3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nu", [16, 256])
def test_chi2_sample_closed_form_moments(nu):
    # S = (x + sqrt(2 nu - 1))^2 / 2 with x ~ N(0,1): E[S] = nu and
    # Var[S] = 2 nu - 1/2 (chi2_nu has nu and 2 nu). One independent sample
    # per seed: the first pass uses the Box-Muller pool's last value.
    S = []
    for seed in range(4000):
        g = oracle.Gen(seed, 4, nu // 4)
        g.do_pass()
        S.append(g.last_S)
    S = np.array(S)
    m = len(S)
    var = 2 * nu - 0.5
    assert abs(S.mean() - nu) <= 5 * math.sqrt(var / m)
    # variance of the sample variance for this law ~ (mu4 - var^2)/m; use a
    # generous 10% band, still far from the 2 nu + 1/2 or 4 nu of a wrong S
    assert abs(S.var() / var - 1) < 0.1


@pytest.mark.parametrize("nu", [4, 16, 256, 4096, 1 << 16, 1 << 20, 1 << 24])
def test_chi2_target_closed_form_by_quadrature(nu):
    # eq. 3: 2 chi2_nu ~ (x + sqrt(2 nu - 1))^2 with x ~ N(0,1), so the
    # target is S(x) = (x + r)^2 / 2 with r^2 = 2 nu - 1. Deterministic pins:
    #   S(0) = (2 nu - 1) / 2;
    #   (S(x) - S(-x)) / (2x) = r;
    #   E[S] = nu exactly by two-point Gauss-Hermite quadrature (nodes +-1,
    #   weights 1/2; exact for polynomials of degree <= 3);
    #   Var[S] = 2 nu - 1/2 by the three-point rule (nodes 0, +-sqrt 3,
    #   weights 2/3, 1/6, 1/6; exact for degree <= 5).
    # A wrong constant (say r^2 = 2 nu) moves E[S] by 1/2.
    def S_of(x):
        return oracle.scale32(x, 1.0, nu)[1]
    assert abs(S_of(0.0) - (2 * nu - 1) / 2) <= 4 * 2.0 ** -53 * nu
    for x in (1.0, 0.5, 3.0):
        assert abs((S_of(x) - S_of(-x)) / (2 * x) - math.sqrt(2 * nu - 1)) <= 1e-15 * nu
    mean = (Fraction(S_of(1.0)) + Fraction(S_of(-1.0))) / 2
    assert abs(float(mean) - nu) <= 8 * 2.0 ** -53 * nu
    if nu <= 1 << 16:  # beyond, FP64 rounding of S^2 blurs the 1/2
        nodes = [(Fraction(2, 3), 0.0), (Fraction(1, 6), math.sqrt(3)),
                 (Fraction(1, 6), -math.sqrt(3))]
        e1 = sum(w * Fraction(S_of(x)) for w, x in nodes)
        e2 = sum(w * Fraction(S_of(x)) ** 2 for w, x in nodes)
        var = float(e2 - e1 * e1)
        assert abs(var - (2 * nu - 0.5)) <= 1e-9 * nu * nu + 1e-6


@pytest.mark.parametrize("nu", [16, 4096, 1 << 20])
def test_chi2_scale_direction_exact(nu):
    # c = sqrt(S / sigma): sigma = S gives exactly 1, sigma = S/4 exactly 2,
    # sigma = 4 S exactly 1/2 (powers of two scale exactly); the FP32 scale
    # is RN32 of the FP64 one.
    for x in (0.0, 0.7, -1.3):
        _, S, _ = oracle.scale32(x, 1.0, nu)
        for sigma, want in ((S, 1.0), (S / 4, 2.0), (4 * S, 0.5)):
            c32, S2, c64 = oracle.scale32(x, sigma, nu)
            assert S2 == S and c64 == want and c32 == np.float32(want)
        c32, _, c64 = oracle.scale32(x, 3.0, nu)
        assert c64 == math.sqrt(S / 3.0) and c32 == np.float32(c64)


def test_chi2_many_matches_scale32():
    # the array form used to check the GPU's arithmetic is the same eq. 3
    rng = np.random.default_rng(3)
    for nu in (16, 1 << 10, 1 << 22):
        x = rng.standard_normal(200).astype(np.float32).astype(np.float64)
        sig = nu * (1 + 0.01 * rng.standard_normal(200))
        S, c = oracle.chi2_many(x, sig, np.full(200, math.sqrt(2 * nu - 1)))
        for i in range(200):
            _, S1, c1 = oracle.scale32(float(x[i]), float(sig[i]), nu)
            assert S[i] == S1 and c[i] == c1
    w = rng.integers(0, 2 ** 63, 300, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    cs, sn = oracle.rotation_many(w)
    for i in range(300):
        assert (cs[i], sn[i]) == oracle.rotation(int(w[i]))


def test_scaled_pass_hits_chi2_target():
    # After a pass the pool's sum of squares equals S up to rounding.
    g = oracle.Gen(1, 4, 1024)
    for _ in range(20):
        g.do_pass()
        assert abs(g.sigma / g.last_S - 1) < 1e-6


def test_chi2_target_depends_only_on_driver():
    # The new sum of squares depends on the old pool only through its last
    # flat value (the driver), whatever the rest holds.
    rng = np.random.default_rng(8)
    n, N = 4, 64
    nu = n * N
    a = np.array([3, 7, 13, 19], dtype=np.uint32)
    b = np.array([1, 2, 3, 4], dtype=np.uint32)
    results = []
    for trial in range(3):
        X = rng.standard_normal(nu).astype(np.float32)
        X[-1] = np.float32(0.75)
        c32, S, _ = oracle.scale32(float(X[-1]), oracle.sumsq_f64(X), nu)
        Y = oracle.pass32(n, N, 0, a, b, np.float32(c32 * np.float32(0.5)), X)
        results.append(oracle.sumsq_f64(Y))
    assert max(results) / min(results) - 1 < 1e-6
    X[-1] = np.float32(-0.75)
    c32, S2, _ = oracle.scale32(float(X[-1]), oracle.sumsq_f64(X), nu)
    assert abs(S2 - S) > 1.0


def test_outlier_bound_generalised():
    # Section 8 bounds the pool maximum across a pass by M/sqrt(2) <= M' <=
    # sqrt(2) M for n = 2. With entries +-1/2 (n = 4) the same argument gives
    # c M / 2 <= M' <= 2 c M, and with H16/4, c M / 4 <= M' <= 4 c M.
    for n, N, lo, hi in ((4, 256, 0.5, 2.0), (16, 64, 0.25, 4.0)):
        g = oracle.Gen(3, n, N)
        M = np.abs(g.pool).max()
        for _ in range(50):
            g.do_pass()
            M2 = np.abs(g.pool).max()
            c = g.last_c64
            assert c * M * lo * (1 - 1e-6) <= M2 <= c * M * hi * (1 + 1e-6)
            M = M2


# ---------------------------------------------------------------------------
# Initial pool (section 5: Box-Muller)
# ---------------------------------------------------------------------------

def test_box_muller_polar_form():
    seed = 42
    pool, _ = oracle.initial_pool64(seed, 4, 64)
    s = seed
    for m in range(pool.size // 2):
        s, w1 = oracle.splitmix64(s)
        s, w2 = oracle.splitmix64(s)
        u1 = ((w1 >> 11) + 1) * 2.0 ** -53
        u2 = (w2 >> 11) * 2.0 ** -53
        x, y = pool[2 * m], pool[2 * m + 1]
        assert math.isclose(x * x + y * y, -2.0 * math.log(u1), rel_tol=1e-12, abs_tol=1e-300)
        ang = math.atan2(y, x) % (2 * math.pi)
        d = abs(ang - 2 * math.pi * u2)
        assert min(d, 2 * math.pi - d) < 1e-9


def test_initial_pool_state_and_moments():
    pool, s = oracle.initial_pool64(42, 4, 1 << 16)
    assert s == (42 + pool.size * 0x9E3779B97F4A7C15) % (1 << 64)
    M = pool.size
    assert abs(pool.mean()) < 5 * math.sqrt(1 / M)
    assert abs((pool ** 2).mean() - 1) < 5 * math.sqrt(2 / M)
    assert abs((pool ** 4).mean() - 3) < 5 * math.sqrt(96 / M)


# ---------------------------------------------------------------------------
# Generator-level properties
# ---------------------------------------------------------------------------

def test_stream_independent_of_call_splitting():
    ref = oracle.Gen(42, 4, 64).fill(5000)
    rng = np.random.default_rng(0)
    g = oracle.Gen(42, 4, 64)
    parts, left = [], 5000
    while left:
        m = int(min(left, rng.integers(0, 700)))
        parts.append(g.fill(m))
        left -= m
    assert np.array_equal(np.concatenate(parts), ref)


def test_throwaway_factor_keeps_every_fth_pool():
    nu = 4 * 32
    full = oracle.Gen(9, 4, 32).fill(6 * nu).reshape(6, nu)
    f2 = oracle.Gen(9, 4, 32, f=2).fill(3 * nu).reshape(3, nu)
    assert np.array_equal(f2, full[1::2])


def test_withheld_driver_is_not_emitted():
    nu = 4 * 32
    full = oracle.Gen(9, 4, 32).fill(4 * nu).reshape(4, nu)
    w = oracle.Gen(9, 4, 32, withhold=1).fill(4 * (nu - 1)).reshape(4, nu - 1)
    assert np.array_equal(w, full[:, :-1])


def test_generator_composes_documented_steps():
    # The generator is params -> scale from the old pool -> pass with
    # A_{(p-1) mod 2} -> new sum of squares.
    n, N = 4, 128
    g = oracle.Gen(77, n, N)
    X = g.pool
    sigma, s = g.sigma, 77 + n * N * 0x9E3779B97F4A7C15
    s %= 1 << 64
    assert sigma == oracle.sumsq_f64(X)
    for p in range(1, 5):
        a, b, _, s = oracle.pass_params(s, n, N)
        c32, _, _ = oracle.scale32(float(X[-1]), sigma, n * N)
        X = oracle.pass32(n, N, (p - 1) % 2, a, b, np.float32(c32 * np.float32(0.5)), X)
        sigma = oracle.sumsq_f64(X)
        g.do_pass()
        assert np.array_equal(g.pool, X)
        assert g.sigma == sigma and g.rng == s


@pytest.mark.parametrize("n,N", [(4, 128), (16, 64), (2, 256)])
def test_fp64_variant_composes_documented_steps(n, N):
    # The FP64 variant is params -> c64 from the old pool (unrounded) ->
    # dense FP64 product c64 A v (or the rotation) -> FP64 sum of squares.
    seed = 123
    g = oracle.Gen64(seed, n, N)
    X, s = oracle.initial_pool64(seed, n, N)
    assert np.array_equal(g.pool, X)
    sigma = oracle.sumsq_d(X)
    assert g.sigma == sigma
    for p in range(1, 6):
        a, b, signs, (cs, sn), s = oracle.pass_params_rot(s, n, N)
        _, S, c64 = oracle.scale32(float(X[-1]), sigma, n * N)
        if n == 2:
            X = oracle.pass64_rot(N, a, b, cs, sn, c64, X)
        else:
            X = oracle.pass64(n, N, (p - 1) % 2 if n == 4 else 0, a, b, c64, X, signs)
        sigma = oracle.sumsq_d(X)
        g.do_pass()
        assert np.array_equal(g.pool, X), p
        assert g.sigma == sigma and g.rng == s and g.last_S == S and g.last_c64 == c64


@pytest.mark.parametrize("n,N", [(4, 1024), (16, 256), (2, 2048)])
def test_fp64_variant_hits_chi2_target_to_fp64_rounding(n, N):
    # In exact arithmetic the scaled pass gives the new pool the sum of
    # squares S exactly (A orthogonal, c^2 = S / sigma). The FP64 variant
    # must reach it to FP64 rounding: a scale rounded to FP32 anywhere would
    # leave errors near 1e-7.
    g = oracle.Gen64(9, n, N)
    worst = 0.0
    for _ in range(30):
        g.do_pass()
        worst = max(worst, abs(g.sigma - g.last_S) / g.last_S)
    assert worst < 1e-13, worst


def test_fp32_variant_within_1e5_of_fp64_variant():
    # Accuracy bound of the bit-exact variant against the FP64 variant after
    # 1000 passes of the 4096-value pool.
    x = oracle.Gen(42, 4, 1024).fill(4096 * 1000)
    y = oracle.Gen64(42, 4, 1024).fill(4096 * 1000)
    e = np.abs(x.astype(np.float64) - y) / np.maximum(1.0, np.abs(y))
    assert e.max() <= 1e-5
    assert math.sqrt((e ** 2).mean()) < 3e-6


@pytest.mark.parametrize("mode", [oracle.SUM_F32, oracle.SUM_F32_COMP])
def test_fp32_sum_modes_close_to_fp64(mode):
    a = oracle.Gen(5, 16, 256, sum_mode=mode).fill(4096 * 50)
    b = oracle.Gen(5, 16, 256).fill(4096 * 50)
    assert np.max(np.abs(a - b)) < 1e-4


def test_n16_sign_draws_and_composition():
    # n = 16: the column signs come from bit 62 of each component's draw, and
    # the generator applies them (H16 D / 4).
    n, N = 16, 32
    g = oracle.Gen(5, n, N)
    X, sigma = g.pool, g.sigma
    s = (5 + n * N * 0x9E3779B97F4A7C15) % (1 << 64)
    seen = set()
    for p in range(1, 6):
        t = s
        expect_signs = 0
        for k in range(n):
            t, w = oracle.splitmix64(t)
            expect_signs |= ((w >> 62) & 1) << k
        a, b, signs, s = oracle.pass_params(s, n, N)
        assert signs == expect_signs
        seen.add(signs)
        c32, _, _ = oracle.scale32(float(X[-1]), sigma, n * N)
        X = oracle.pass32(n, N, 0, a, b, np.float32(c32 * np.float32(0.25)), X, signs)
        sigma = oracle.sumsq_f64(X)
        g.do_pass()
        assert np.array_equal(g.pool, X)
    assert len(seen) == 5


def test_fixed_h16_conserves_pool_total_every_second_pass():
    # Why n = 16 draws column signs: with the same H16/4 every pass the pool
    # total T obeys T'' = c c' T (the all-ones row of H16), so the output
    # mean cannot average out. Random column signs break the recurrence.
    n, N = 16, 64
    rng = np.random.default_rng(2)
    X = rng.standard_normal(n * N).astype(np.float32)
    a = np.array([3] * n, dtype=np.uint32)
    T0 = float(X.astype(np.float64).sum())
    Y = X
    for _ in range(2):
        b = rng.integers(0, N, size=n).astype(np.uint32)
        Y = oracle.pass32(n, N, 0, a, b, np.float32(0.25), Y, 0)
    assert abs(float(Y.astype(np.float64).sum()) - T0) < 1e-3
    Z = X
    for signs in (0x1234, 0x8421):
        b = rng.integers(0, N, size=n).astype(np.uint32)
        Z = oracle.pass32(n, N, 0, a, b, np.float32(0.25), Z, signs)
    assert abs(float(Z.astype(np.float64).sum()) - T0) > 1.0


def test_oracle_matches_frozen_stream_heads():
    # Regression guard: any change to the oracle's arithmetic must be made on
    # purpose (tests/golden/make_golden.py rewrites the file).
    g = _golden("oracle_stream_heads.json")
    for case in g["cases"]:
        gen = oracle.Gen(case["seed"], case["n"], case["N"])
        nu = case["n"] * case["N"]
        x = gen.fill(nu * case["passes"])
        assert [f"{int(v):08x}" for v in x[:32].view(np.uint32)] == case["head_bits"]
        assert [f"{int(v):08x}" for v in x[-32:].view(np.uint32)] == case["tail_bits"]
        assert float(gen.sigma).hex() == case["sigma_hex"]
        assert str(gen.rng) == case["rng"]


# ---------------------------------------------------------------------------
# n = 2: RANN4's random rotation (section 8)
# ---------------------------------------------------------------------------

_GAMMA = 0x9E3779B97F4A7C15


def _theta_ok(theta):
    # section 8: pi/6 <= |theta| <= pi/3 or 2pi/3 <= theta <= 5pi/6
    a = abs(theta)
    eps = 1e-12
    return (math.pi / 6 - eps <= a <= math.pi / 3 + eps or
            2 * math.pi / 3 - eps <= theta <= 5 * math.pi / 6 + eps)


def test_rotation_matches_trigonometry_and_ranges():
    # sin and cos from t = tan(theta/2) by rational formulas must equal the
    # trigonometric functions of theta = 2 atan(t), lie in the printed
    # ranges, keep min(|sin|, |cos|) >= 1/2 and hit all three intervals.
    rng = np.random.default_rng(11)
    hits = [0, 0, 0]
    for w in rng.integers(0, 1 << 63, size=3000, dtype=np.uint64):
        w = int(w) ^ (int(rng.integers(0, 2)) << 63)
        cs, sn = oracle.rotation(w)
        i = (w >> 32) % 3
        hits[i] += 1
        u = (w & 0xFFFFFFFF) / 2.0 ** 32
        lo_hi = {0: (math.tan(math.pi / 12), math.tan(math.pi / 6)),
                 1: (-math.tan(math.pi / 6), -math.tan(math.pi / 12)),
                 2: (math.tan(math.pi / 3), math.tan(5 * math.pi / 12))}[i]
        t = lo_hi[0] + (lo_hi[1] - lo_hi[0]) * u
        theta = 2 * math.atan(t)
        assert abs(cs - math.cos(theta)) < 1e-14 and abs(sn - math.sin(theta)) < 1e-14
        assert _theta_ok(math.atan2(sn, cs))
        assert min(abs(cs), abs(sn)) >= 0.5 - 1e-14
        assert abs(cs * cs + sn * sn - 1.0) < 1e-15
    assert min(hits) > 800


def test_rotation_interval_endpoints():
    # u = 0 gives the interval's first end: theta = pi/6, -pi/3, 2pi/3
    for i, theta in ((0, math.pi / 6), (1, -math.pi / 3), (2, 2 * math.pi / 3)):
        w = i << 32
        cs, sn = oracle.rotation(w)
        assert abs(cs - math.cos(theta)) < 1e-15 and abs(sn - math.sin(theta)) < 1e-15


def test_n2_pass_params_are_rann4_sets_plus_one_draw():
    # alpha in {3,5}, beta in {7,11}, offsets below N, three draws per pass
    s0 = 99
    seen = set()
    s = s0
    for _ in range(200):
        a, b, _, rot, s = oracle.pass_params_rot(s, 2, 1024)
        assert a[0] in (3, 5) and a[1] in (7, 11) and (b < 1024).all()
        assert min(abs(rot[0]), abs(rot[1])) >= 0.5 - 1e-14
        seen.add((int(a[0]), int(a[1])))
    assert seen == {(3, 7), (3, 11), (5, 7), (5, 11)}
    assert s == (s0 + 3 * 200 * _GAMMA) % (1 << 64)


def test_n2_pass32_exact_on_dyadic_inputs():
    # with dyadic p, q and small dyadic pool values every FP32 product and
    # sum is exact, so the FP32 pass equals the exact rotation-type map
    N = 16
    rng = np.random.default_rng(3)
    X = (rng.integers(-64, 64, size=2 * N) / 8.0).astype(np.float32)
    a = np.array([3, 7], np.uint32)
    b = np.array([5, 2], np.uint32)
    p, q = np.float32(0.75), np.float32(-0.625)
    Y = oracle.pass32_rot(N, a, b, p, q, X)
    for j in range(N):
        x = Fraction(float(X[(3 * j + 5) % N]))
        y = Fraction(float(X[N + (7 * j + 2) % N]))
        assert Fraction(float(Y[j])) == Fraction(0.75) * x + Fraction(-0.625) * y
        assert Fraction(float(Y[N + j])) == Fraction(0.75) * y - Fraction(-0.625) * x


def test_n2_rotation_preserves_sum_of_squares():
    # unscaled (c = 1): per tuple x'^2 + y'^2 = x^2 + y^2 up to rounding
    N = 512
    X = oracle.initial_pool64(5, 2, N)[0].astype(np.float32)
    a, b, _, (cs, sn), _ = oracle.pass_params_rot(5, 2, N)
    Y = oracle.pass32_rot(N, a, b, np.float32(cs), np.float32(sn), X)
    j = np.arange(N)
    x = X[(a[0].astype(np.int64) * j + b[0]) % N].astype(np.float64)
    y = X[N + (a[1].astype(np.int64) * j + b[1]) % N].astype(np.float64)
    before = x * x + y * y
    after = Y[:N].astype(np.float64) ** 2 + Y[N:].astype(np.float64) ** 2
    assert np.all(np.abs(after - before) <= 8 * 2.0 ** -24 * before + 1e-30)


def test_n2_generator_composes_documented_steps():
    # params (3 draws) -> c from the old pool -> p = RN32(c cos), q = RN32(c sin)
    # -> rotation pass -> new sum of squares
    n, N = 2, 256
    g = oracle.Gen(31, n, N)
    X = g.pool
    sigma = g.sigma
    s = (31 + n * N * _GAMMA) % (1 << 64)
    for _ in range(5):
        a, b, _, (cs, sn), s = oracle.pass_params_rot(s, n, N)
        _, _, c64 = oracle.scale32(float(X[-1]), sigma, n * N)
        X = oracle.pass32_rot(N, a, b, np.float32(c64 * cs), np.float32(c64 * sn), X)
        sigma = oracle.sumsq_f64(X)
        g.do_pass()
        assert np.array_equal(g.pool, X) and g.sigma == sigma and g.rng == s


def test_n2_fp32_within_1e5_of_fp64_and_dense_matrix():
    x = oracle.Gen(42, 2, 2048).fill(4096 * 500)
    y = oracle.Gen64(42, 2, 2048).fill(4096 * 500)
    e = np.abs(x.astype(np.float64) - y) / np.maximum(1.0, np.abs(y))
    assert e.max() <= 1e-5
    # the FP64 pass is the dense product c [[cos, sin], [-sin, cos]] v
    N = 64
    X = np.random.default_rng(2).standard_normal(2 * N)
    a = np.array([5, 11], np.uint32)
    b = np.array([1, 60], np.uint32)
    Y = oracle.pass64_rot(N, a, b, 0.6, 0.8, 1.5, X)
    j = np.arange(N)
    v0 = X[(5 * j + 1) % N]
    v1 = X[N + (11 * j + 60) % N]
    assert np.allclose(Y[:N], 1.5 * (0.6 * v0 + 0.8 * v1), rtol=0, atol=1e-15)
    assert np.allclose(Y[N:], 1.5 * (-0.8 * v0 + 0.6 * v1), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# Restarts (section 5)
# ---------------------------------------------------------------------------

def test_restart_refills_by_box_muller_from_the_stream():
    # after R passes the pool is replaced by Box-Muller from the generator's
    # own stream (nu draws, as at initialisation), its sum of squares is
    # recomputed, and the next pass transforms the refilled pool
    n, N, R = 4, 64, 3
    nu = n * N
    g = oracle.Gen(123, n, N, restart=R)
    plain = oracle.Gen(123, n, N)
    for _ in range(R):
        g.do_pass()
        plain.do_pass()
    assert np.array_equal(g.pool, plain.pool)
    s = g.rng
    X64, s2 = oracle.initial_pool64(s, n, N)
    assert s2 == (s + nu * _GAMMA) % (1 << 64)
    X = X64.astype(np.float32)
    sigma = oracle.sumsq_f64(X)
    a, b, _, s3 = oracle.pass_params(s2, n, N)
    c32, _, _ = oracle.scale32(float(X[-1]), sigma, nu)
    Y = oracle.pass32(n, N, R % 2, a, b, np.float32(c32 * np.float32(0.5)), X)
    g.do_pass()
    assert np.array_equal(g.pool, Y) and g.rng == s3
    assert g.sigma == oracle.sumsq_f64(Y)


def test_restart_stream_statistics_and_fp64_agreement():
    x = oracle.Gen(8, 4, 1024, restart=50).fill(4096 * 400)
    y = oracle.Gen64(8, 4, 1024, restart=50).fill(4096 * 400)
    e = np.abs(x.astype(np.float64) - y) / np.maximum(1.0, np.abs(y))
    assert e.max() <= 1e-5
    M = x.size
    xd = x.astype(np.float64)
    assert abs(xd.mean()) * math.sqrt(M) < 5
    assert abs((xd ** 2).mean() - 1) / math.sqrt(2 / M) < 5
