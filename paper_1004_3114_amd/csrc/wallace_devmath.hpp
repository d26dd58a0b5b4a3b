// Per-pass parameter and scale arithmetic of the Wallace generator library,
// shared by every pass kernel (pool-resident and streamed) so that all of
// them draw the same strides, offsets, signs and rotations and compute the
// same chi-squared scale. Host code may call the __host__ __device__ parts.
//
//   splitmix64 (Steele, Lea and Flood 2014): the uniform source of the pass
//   parameters; draw m of a generator is a function of its state + m gamma.
//   Strides (eq. 2; sections 3, 6, 8, 9): component k picks one of a pair of
//   odd primes; the reduced stride must differ from 1 and from the strides
//   of earlier components (distinct_stride).
//   Chi-squared scale (section 4, eq. 3): c = sqrt(S / sigma) with
//   S = (x* + sqrt(2 nu - 1))^2 / 2, one correctly rounded FP64 operation
//   per step.
//   n = 2 rotation (section 8): cos and sin of theta from t = tan(theta/2)
//   by rational formulas.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wallace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

// splitmix64 output for state value z (after the Weyl step): two
// xor-shift-multiply rounds and a final xor-shift.
__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One splitmix64 step: Weyl increment of the state, then the mix.
__host__ __device__ __forceinline__ uint64_t sm64_next(uint64_t &s)
{
    s += kGamma;
    return sm64_mix(s);
}

// Stride pair of component k: RANN4's {3,5} and {7,11} (section 8), then
// further disjoint pairs of odd primes. `top` (the draw's top bit) picks one.
__host__ __device__ __forceinline__ uint32_t stride_pick(int k, uint32_t top)
{
    constexpr uint32_t lo[16] = {3, 7, 13, 19, 29, 37, 43, 53,
                                 61, 71, 79, 89, 101, 107, 113, 131};
    constexpr uint32_t hi[16] = {5, 11, 17, 23, 31, 41, 47, 59,
                                 67, 73, 83, 97, 103, 109, 127, 137};
    return top ? hi[k] : lo[k];
}

// Largest prime of the pairs used by n components: with N above it, every
// reduced table stride is the prime itself, so no two components share one
// and none is 1.
__host__ __device__ constexpr uint32_t max_table_stride(int n)
{
    return n == 2 ? 11u : (n == 4 ? 23u : 137u);
}

// Distinct strides above one (sections 3, 6 and 9). A stride acts modulo N,
// so for small pools a table prime can reduce to 1 or to the stride of an
// earlier component of the same pass. Such a candidate moves up by 2 (mod N,
// so it stays odd and eq. 2 holds) until it is neither 1 nor, while some of
// the N/2 - 1 odd residues above one are still unused by components
// 0 .. K-1, one of theirs. `prev` holds the strides of components 0 .. K-1.
// Terminates: with K < N/2 - 1 an unused residue exists; otherwise only 1 is
// skipped, and N >= 4 leaves 3.
template <int K, int NP>
__host__ __device__ __forceinline__ uint32_t distinct_stride(uint32_t cand, const uint32_t (&prev)[NP],
                                                             uint32_t N)
{
    static_assert(K <= NP, "earlier components");
    const uint32_t free_odd = N / 2u - 1u;
    const bool need_distinct = (uint32_t)K < free_odd;
    for (;;) {
        bool clash = cand == 1u;
        if (need_distinct) {
#pragma unroll
            for (int i = 0; i < K; ++i) clash = clash || prev[i] == cand;
        }
        if (!clash || free_odd == 0u) return cand;
        cand = (cand + 2u) & (N - 1u);
    }
}

// Chi-squared target (section 4, eq. 3) from the old pool's last flat value
// x* and r_nu = RN64(sqrt(2 nu - 1)): t = x* + r_nu, S = (t t) / 2.
__host__ __device__ __forceinline__ double chi2_target(double xstar, double r_nu)
{
    const double t = xstar + r_nu;
    return (t * t) * 0.5;
}

// Scale that gives the new pool the target S from the old pool's sum of
// squares sigma: q = S / sigma, c = sqrt(q).
__host__ __device__ __forceinline__ double chi2_scale_from_S(double S, double sigma)
{
    const double q = S / sigma;
    return __builtin_sqrt(q);
}

// Both steps: c = sqrt(((x* + r_nu)^2 / 2) / sigma), each step one correctly
// rounded FP64 operation (no contraction: built with -ffp-contract=off).
__host__ __device__ __forceinline__ double chi2_scale64(double xstar, double sigma, double r_nu)
{
    return chi2_scale_from_S(chi2_target(xstar, r_nu), sigma);
}

// n = 2 rotation of a pass from its draw w (section 8): theta in one of
// [pi/6, pi/3], [-pi/3, -pi/6], [2pi/3, 5pi/6] picked by (w >> 32) mod 3,
// t = tan(theta/2) uniform on that interval's image with u = (w mod 2^32)
// 2^-32 (the ends are 2 - sqrt 3, 1/sqrt 3, sqrt 3 and 2 + sqrt 3),
// cos = (1 - t^2)/(1 + t^2), sin = 2t/(1 + t^2), one FP64 operation per step.
__host__ __device__ __forceinline__ void rotation(uint64_t w, double &cs, double &sn)
{
    const double r3 = __builtin_sqrt(3.0);
    const double tA = 2.0 - r3, tB = 1.0 / r3, tC = r3, tD = 2.0 + r3;
    const uint32_t i = (uint32_t)((w >> 32) % 3u);
    const double lo = i == 0 ? tA : (i == 1 ? -tB : tC);
    const double hi = i == 0 ? tB : (i == 1 ? -tA : tD);
    const double u = (double)(uint32_t)w * (1.0 / 4294967296.0);
    const double t = lo + (hi - lo) * u;
    const double t2 = t * t;
    const double den = 1.0 + t2;
    cs = (1.0 - t2) / den;
    sn = (t + t) / den;
}

}  // namespace wallace
