/*
 * Oracle for Wallace's normal generator (Brent 1997, "A fast vectorised
 * implementation of Wallace's normal random number generator").
 *
 * TEST INFRASTRUCTURE. This is a plain, slow, single-threaded CPU
 * implementation written from the paper, used only to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does. It shares no code,
 * header, table or constant with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared (x86-64 SSE
 * arithmetic, round to nearest even, no flush-to-zero).
 *
 * Parity status of each part is stated beside it below.
 */
#ifndef WALLACE_ORACLE_H
#define WALLACE_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Summation modes for the pool's sum of squares (section 4, and section 8's
 * drift monitor). */
enum { WO_SUM_F64 = 0, WO_SUM_F32 = 1, WO_SUM_F32_COMP = 2 };

/* Stride modes for the per-pass permutation (section 3, section 8). */
enum { WO_A_PAIRS = 0, WO_A_FULL_ODD = 1 };

/* ---- uniform source -------------------------------------------------- */

/* splitmix64: advance *state by the golden-ratio increment and return the
 * mixed 64-bit output. Pinned by published test vectors. */
uint64_t wo_splitmix64(uint64_t *state);

/* The k-th stride pair: the (2k+2)-th and (2k+3)-th primes (k < 16).
 * k = 0, 1 give RANN4's alpha in {3,5} and beta in {7,11} (section 8). */
void wo_stride_pair(int k, uint32_t out[2]);

/* ---- initial pool (section 5: uniform generator + Box-Muller) ---------- */

/* Draws nu = n*N uniforms in pairs and returns the unrounded FP64 pool in
 * flat order f = k*N + j. Consumes nu draws from *state. */
void wo_initial_pool64(uint64_t *state, int n, uint32_t N, double *pool);

/* ---- per-pass parameters (eq. 1, eq. 2, sections 3 and 8) -------------- */

/* One draw per component k = 0..n-1: a[k] (odd stride), b[k] (offset);
 * for n = 16 also bit k of *signs (column sign of the matrix). For n = 2
 * (RANN4, section 8) a third draw gives the rotation; see wo_rotation. */
void wo_pass_params(uint64_t *state, int n, uint32_t N, int a_mode,
                    uint32_t *a, uint32_t *b, uint32_t *signs);
/* The same, also returning the n = 2 rotation (rot[0] = cos theta,
 * rot[1] = sin theta; untouched for other n). */
void wo_pass_params_rot(uint64_t *state, int n, uint32_t N, int a_mode,
                        uint32_t *a, uint32_t *b, uint32_t *signs, double *rot);

/* Rotation of an n = 2 pass from one draw w (section 8): theta in one of
 * [pi/6, pi/3], [-pi/3, -pi/6], [2pi/3, 5pi/6], picked by (w >> 32) mod 3;
 * t = tan(theta/2) uniform in that interval's image with u = (w mod 2^32)
 * 2^-32; cos theta = (1 - t^2)/(1 + t^2), sin theta = 2t/(1 + t^2), each
 * step one FP64 operation. */
void wo_rotation(uint64_t w, double *cs, double *sn);

/* Array forms for checking the GPU's FP64 arithmetic against the host's:
 * wo_rotation for each w[i]; and the chi-squared scale of eq. 3 from an
 * explicit r = RN64(sqrt(2 nu - 1)): S[i] = (xstar[i] + r[i])^2 / 2,
 * c[i] = sqrt(S[i] / sigma[i]), each step one IEEE operation. */
void wo_rotation_many(const uint64_t *w, size_t count, double *cs, double *sn);
void wo_chi2_many(const double *xstar, const double *sigma, const double *r,
                  size_t count, double *S, double *c);

/* ---- sum of squares (section 4) ----------------------------------------- */

/* Canonical pairwise tree over flat index: leaves y_f^2, then pairs
 * (2i, 2i+1), then pairs of pairs. nu must be a power of two. */
double wo_sumsq_f64(const float *y, size_t nu);       /* FP64 nodes, exact leaves */
float wo_sumsq_f32(const float *y, size_t nu);        /* FP32 nodes (naive)       */
double wo_sumsq_f32c(const float *y, size_t nu);      /* FP32 pairs + error terms */
double wo_sumsq_mode(const float *y, size_t nu, int mode);
double wo_sumsq_d(const double *y, size_t nu);        /* FP64 pool (FP64 variant) */

/* ---- chi-squared rescaling (section 4, eq. 3) ----------------------------- */

/* S = ((xstar + sqrt(2 nu - 1))^2) / 2; returns RN32(sqrt(S / sigma)). */
float wo_scale32(double xstar, double sigma, size_t nu, double *S_out,
                 double *c64_out);

/* ---- one pass (eq. 1) ------------------------------------------------------ */

/* FP32 pass: Y_k[j] = (A v)_k * h with v_k = X_k[(a_k j + b_k) mod N].
 * n = 4: mat 0 -> A0 = H4/2, mat 1 -> A1 = J/2 - I; n = 16: H16 D/4 with
 * D = diag((-1)^(bit k of signs)). h includes the power-of-two factor. */
void wo_pass32(int n, uint32_t N, int mat, const uint32_t *a,
               const uint32_t *b, uint32_t signs, float h, const float *X,
               float *Y);

/* FP64 pass with an explicit dense matrix: Y_k[j] = c * sum_i (M D)[k][i] v_i. */
void wo_pass64(int n, uint32_t N, int mat, const uint32_t *a,
               const uint32_t *b, uint32_t signs, double c, const double *X,
               double *Y);

/* Dense n x n matrix used by wo_pass64 (row-major), for tests. */
void wo_matrix(int n, int mat, double *M);

/* n = 2 passes (RANN4). FP32: with p = RN32(c cos theta), q = RN32(c sin
 * theta), x'_j = p x + q y and y'_j = p y - q x, each product and the sum
 * rounded once (two multiplies and one add per number, section 7).
 * FP64: Y = c [[cs, sn], [-sn, cs]] v. */
void wo_pass32_rot(uint32_t N, const uint32_t *a, const uint32_t *b, float p, float q,
                   const float *X, float *Y);
void wo_pass64_rot(uint32_t N, const uint32_t *a, const uint32_t *b, double cs,
                   double sn, double c, const double *X, double *Y);

/* ---- generators ------------------------------------------------------------- */

typedef struct wo_gen wo_gen;

/* FP32 generator (bit-exact variant). f = throw-away factor (>= 1),
 * withhold = 1 keeps the chi-squared driver (flat index nu-1) out of the
 * output (section 4). */
wo_gen *wo_gen_create(uint64_t seed, int n, uint32_t N, int sum_mode,
                      int a_mode, int f, int withhold);
/* FP64 generator (accuracy variant): same draws, unrounded pool, dense
 * FP64 matrices, FP64 sum of squares. */
wo_gen *wo_gen64_create(uint64_t seed, int n, uint32_t N, int a_mode);
/* Section 5 restarts: before pass p + 1 with p a positive multiple of
 * `passes`, refill the pool by Box-Muller from the generator's stream (nu
 * draws, as at initialisation) and recompute its sum of squares. 0: never. */
void wo_gen_set_restart(wo_gen *g, uint64_t passes);
void wo_gen_destroy(wo_gen *g);

/* One pass (eq. 1 plus the section-4 rescaling). */
void wo_gen_pass(wo_gen *g);
/* Emit `count` values of the output stream (pools after every f-th pass,
 * flat order) into out32 (FP32 generator) or out64 (FP64 generator). */
void wo_gen_fill(wo_gen *g, float *out32, double *out64, uint64_t count);

/* State accessors. */
const float *wo_gen_pool32(const wo_gen *g);
const double *wo_gen_pool64(const wo_gen *g);
double wo_gen_sigma(const wo_gen *g);
uint64_t wo_gen_passes(const wo_gen *g);
uint64_t wo_gen_rng(const wo_gen *g);
double wo_gen_last_S(const wo_gen *g);
double wo_gen_last_c64(const wo_gen *g);

#ifdef __cplusplus
}
#endif
#endif
