/*
 * Oracle for Wallace's normal generator as described by Brent (1997).
 *
 * TEST INFRASTRUCTURE: a plain single-threaded CPU implementation that the
 * test suite, the smoke check and the benchmark's CPU-baseline leg use to
 * check the GPU library. Nothing in the product path loads it. Every step is
 * written the slow, obvious way, in the paper's order and notation.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes of the repository):
 *   - uniform source: splitmix64 (the paper's RANU4 is not available);
 *   - initial pool: Box-Muller on pairs of uniforms, cos to even flat index,
 *     sin to odd (section 5 names Box-Muller for (re)filling the pool);
 *   - strides: per component k a pair of primes, one picked per pass by the
 *     top bit of a draw; k = 0, 1 are RANN4's {3,5} and {7,11} (section 8);
 *     reduced mod N, a stride that lands on 1 or on an earlier component's
 *     stride moves to the next free odd residue (sections 3, 6 and 9 want
 *     distinct strides above one; see distinct_stride);
 *     offsets uniform on {0..N-1} (section 8);
 *   - n = 2 (RANN4, section 8): a rotation by theta drawn each pass, with
 *     sin and cos from t = tan(theta/2) (see wo_rotation);
 *   - matrices: n = 4 alternates A0 = H4/2 and A1 = J/2 - I (section 3 says
 *     Wallace picks among two predefined 4x4 matrices); n = 16 uses H16 D/4
 *     with D a diagonal of random signs drawn each pass (section 3 asks for a
 *     different matrix at each pass; with a fixed H16 the pool total returns
 *     every second pass and the output mean drifts);
 *   - chi-squared driver: the old pool's last flat value (section 4, eq. 3);
 *     the scale for a pass comes from the old pool's sum of squares and is
 *     folded into the matrix (section 4);
 *   - sum of squares: canonical pairwise tree over the flat index.
 */
#include "wallace_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Uniform source                                                            */
/* ------------------------------------------------------------------------ */

/* splitmix64 (Steele, Lea and Flood, OOPSLA 2014; Vigna's public-domain
 * reference): the state advances by 0x9E3779B97F4A7C15 and the output is the
 * state passed through two xor-shift-multiply rounds and a final xor-shift.
 * All arithmetic is modulo 2^64. */
uint64_t wo_splitmix64(uint64_t *state)
{
    uint64_t z;
    *state = *state + 0x9E3779B97F4A7C15ull;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Primes by trial division, so the stride table is derived rather than typed
 * in. The k-th pair is (p[2k+1], p[2k+2]) with p[0] = 2. */
static int is_prime(uint32_t x)
{
    uint32_t d;
    if (x < 2) return 0;
    for (d = 2; d * d <= x; ++d)
        if (x % d == 0) return 0;
    return 1;
}

/* The first 34 primes by trial division, filled once when the library is
 * loaded, so that threads calling the oracle concurrently only read them. */
static uint32_t g_primes[34];

__attribute__((constructor)) static void fill_primes(void)
{
    int count = 0;
    uint32_t x;
    for (x = 2; count < 34; ++x)
        if (is_prime(x)) g_primes[count++] = x;
}

void wo_stride_pair(int k, uint32_t out[2])
{
    out[0] = g_primes[2 * k + 1];
    out[1] = g_primes[2 * k + 2];
}

/* ------------------------------------------------------------------------ */
/* Initial pool: Box-Muller (section 5)                                      */
/* ------------------------------------------------------------------------ */

void wo_initial_pool64(uint64_t *state, int n, uint32_t N, double *pool)
{
    size_t nu = (size_t)n * N;
    size_t m;
    double two_pi = 2.0 * M_PI;
    for (m = 0; m < nu / 2; ++m) {
        /* u1 in (0, 1] so that log(u1) is finite; u2 in [0, 1). */
        double u1 = (double)((wo_splitmix64(state) >> 11) + 1) * 0x1.0p-53;
        double u2 = (double)(wo_splitmix64(state) >> 11) * 0x1.0p-53;
        double rho = sqrt(-2.0 * log(u1));
        double theta = two_pi * u2;
        pool[2 * m] = rho * cos(theta);
        pool[2 * m + 1] = rho * sin(theta);
    }
}

/* ------------------------------------------------------------------------ */
/* Per-pass parameters (eq. 1; eq. 2: odd strides give permutations when N   */
/* is a power of two; section 8: alpha in {3,5}, beta in {7,11}, offsets     */
/* uniform on {0..N-1}, chosen once per pool)                                */
/* ------------------------------------------------------------------------ */

void wo_pass_params(uint64_t *state, int n, uint32_t N, int a_mode,
                    uint32_t *a, uint32_t *b, uint32_t *signs)
{
    wo_pass_params_rot(state, n, N, a_mode, a, b, signs, NULL);
}

/* Section 8: RANN4 rotates by theta with min(|sin|, |cos|) >= 1/2, choosing
 * t = tan(theta/2) with a uniform generator and getting sin and cos from t
 * by a few arithmetic operations (no trigonometric functions). Readings:
 * the three theta intervals as printed are equally likely; t is uniform on
 * the image of the chosen interval; tan(pi/12) = 2 - sqrt 3,
 * tan(pi/6) = 1/sqrt 3, tan(pi/3) = sqrt 3, tan(5pi/12) = 2 + sqrt 3. */
void wo_rotation(uint64_t w, double *cs, double *sn)
{
    double r3 = sqrt(3.0);
    double tA = 2.0 - r3, tB = 1.0 / r3, tC = r3, tD = 2.0 + r3;
    double lo, hi, u, t, t2, den;
    unsigned i = (unsigned)((w >> 32) % 3u);
    if (i == 0) {        /* theta in [pi/6, pi/3] */
        lo = tA; hi = tB;
    } else if (i == 1) { /* theta in [-pi/3, -pi/6] */
        lo = -tB; hi = -tA;
    } else {             /* theta in [2pi/3, 5pi/6] */
        lo = tC; hi = tD;
    }
    u = (double)(w & 0xFFFFFFFFull) * (1.0 / 4294967296.0);
    t = lo + (hi - lo) * u;
    t2 = t * t;
    den = 1.0 + t2;
    *cs = (1.0 - t2) / den;
    *sn = (t + t) / den;
}

/* Sections 3, 6 and 9 ask for strides that are distinct and greater than
 * one. A stride acts modulo N, so for small pools a prime of the table can
 * reduce to 1 (unit stride) or to another component's stride. Reading: the
 * reduced stride of component k moves up by 2 (mod N, staying odd) while it
 * is 1, or while it equals the stride of an earlier component of the same
 * pass and some odd residue above one is still unused (there are N/2 - 1 of
 * them; when k of them are taken by earlier components and k < N/2 - 1, a
 * free one exists). For N above the largest prime of the table nothing
 * moves and the strides are the primes themselves. */
static uint32_t distinct_stride(uint32_t cand, const uint32_t *earlier, int k,
                                uint32_t N)
{
    uint32_t free_odd = N / 2 - 1; /* odd residues mod N other than 1 */
    for (;;) {
        int clash = (cand == 1u);
        if (!clash && (uint32_t)k < free_odd) {
            int i;
            for (i = 0; i < k; ++i)
                if (earlier[i] == cand) clash = 1;
        }
        if (!clash || free_odd == 0) return cand;
        cand = (cand + 2u) % N;
    }
}

void wo_rotation_many(const uint64_t *w, size_t count, double *cs, double *sn)
{
    size_t i;
    for (i = 0; i < count; ++i) wo_rotation(w[i], &cs[i], &sn[i]);
}

void wo_chi2_many(const double *xstar, const double *sigma, const double *r,
                  size_t count, double *S, double *c)
{
    size_t i;
    for (i = 0; i < count; ++i) {
        double t = xstar[i] + r[i];
        double s = (t * t) * 0.5;
        S[i] = s;
        c[i] = sqrt(s / sigma[i]);
    }
}

void wo_pass_params_rot(uint64_t *state, int n, uint32_t N, int a_mode,
                        uint32_t *a, uint32_t *b, uint32_t *signs, double *rot)
{
    int k;
    *signs = 0;
    for (k = 0; k < n; ++k) {
        uint64_t w = wo_splitmix64(state);
        uint32_t cand;
        if (a_mode == WO_A_PAIRS) {
            uint32_t pair[2];
            wo_stride_pair(k, pair);
            cand = pair[w >> 63] % N;
        } else {
            cand = (uint32_t)((w >> 32) % N) | 1u;
        }
        a[k] = distinct_stride(cand, a, k, N);
        b[k] = (uint32_t)(w % N);
        /* n = 16: a fresh column sign per component and pass, so that the
         * matrix differs at each pass (section 3). */
        if (n == 16 && ((w >> 62) & 1u)) *signs |= 1u << k;
    }
    if (n == 2) { /* the pass's rotation: one more draw */
        uint64_t w = wo_splitmix64(state);
        double cs, sn;
        wo_rotation(w, &cs, &sn);
        if (rot) { rot[0] = cs; rot[1] = sn; }
    }
}

/* ------------------------------------------------------------------------ */
/* Sum of squares (section 4): canonical pairwise tree over the flat index   */
/* ------------------------------------------------------------------------ */

double wo_sumsq_f64(const float *y, size_t nu)
{
    double *t = (double *)malloc(nu * sizeof(double));
    size_t f, w;
    double s;
    for (f = 0; f < nu; ++f) t[f] = (double)y[f] * (double)y[f]; /* exact */
    for (w = nu; w > 1; w /= 2)
        for (f = 0; f < w / 2; ++f) t[f] = t[2 * f] + t[2 * f + 1];
    s = t[0];
    free(t);
    return s;
}

float wo_sumsq_f32(const float *y, size_t nu)
{
    float *t = (float *)malloc(nu * sizeof(float));
    size_t f, w;
    float s;
    for (f = 0; f < nu; ++f) t[f] = y[f] * y[f];
    for (w = nu; w > 1; w /= 2)
        for (f = 0; f < w / 2; ++f) t[f] = t[2 * f] + t[2 * f + 1];
    s = t[0];
    free(t);
    return s;
}

/* Compensated FP32 tree: every node is a pair (s, e) with s + e carrying the
 * node's sum. Leaves: s = RN(y*y), e = fma(y, y, -s) (exact remainder).
 * Join: s = RN(s1 + s2) with Knuth's TwoSum error, e = (e1 + e2) + err. */
double wo_sumsq_f32c(const float *y, size_t nu)
{
    float *s = (float *)malloc(nu * sizeof(float));
    float *e = (float *)malloc(nu * sizeof(float));
    size_t f, w;
    double out;
    for (f = 0; f < nu; ++f) {
        s[f] = y[f] * y[f];
        e[f] = fmaf(y[f], y[f], -s[f]);
    }
    for (w = nu; w > 1; w /= 2) {
        for (f = 0; f < w / 2; ++f) {
            float s1 = s[2 * f], s2 = s[2 * f + 1];
            float e1 = e[2 * f], e2 = e[2 * f + 1];
            float sum = s1 + s2;
            float bb = sum - s1;
            float err = (s1 - (sum - bb)) + (s2 - bb);
            s[f] = sum;
            e[f] = (e1 + e2) + err;
        }
    }
    out = (double)s[0] + (double)e[0];
    free(s);
    free(e);
    return out;
}

double wo_sumsq_mode(const float *y, size_t nu, int mode)
{
    if (mode == WO_SUM_F32) return (double)wo_sumsq_f32(y, nu);
    if (mode == WO_SUM_F32_COMP) return wo_sumsq_f32c(y, nu);
    return wo_sumsq_f64(y, nu);
}

double wo_sumsq_d(const double *y, size_t nu)
{
    double *t = (double *)malloc(nu * sizeof(double));
    size_t f, w;
    double s;
    for (f = 0; f < nu; ++f) t[f] = y[f] * y[f];
    for (w = nu; w > 1; w /= 2)
        for (f = 0; f < w / 2; ++f) t[f] = t[2 * f] + t[2 * f + 1];
    s = t[0];
    free(t);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Chi-squared rescaling (section 4, eq. 3)                                  */
/* ------------------------------------------------------------------------ */

/* eq. 3: 2 chi2_nu ~ (x + sqrt(2 nu - 1))^2 with x ~ N(0,1), so a chi2_nu
 * sample is S = (x + sqrt(2 nu - 1))^2 / 2. The pool is scaled so that its
 * sum of squares becomes S: c = sqrt(S / sigma). */
float wo_scale32(double xstar, double sigma, size_t nu, double *S_out,
                 double *c64_out)
{
    double r = sqrt((double)(2 * nu - 1));
    double t = xstar + r;
    double S = (t * t) * 0.5;
    double c64 = sqrt(S / sigma);
    if (S_out) *S_out = S;
    if (c64_out) *c64_out = c64;
    return (float)c64;
}

/* ------------------------------------------------------------------------ */
/* Transforms                                                                */
/* ------------------------------------------------------------------------ */

/* In-place fast Walsh-Hadamard transform on n = 2^m values, stage s pairing
 * i and i + 2^s for every i with bit s clear. Gives the natural-order
 * Sylvester matrix H_n (entry (i,j) = (-1)^popcount(i & j)). */
static void fwht32(float *v, int n)
{
    int s, i;
    for (s = 1; s < n; s <<= 1) {
        for (i = 0; i < n; ++i) {
            if (i & s) continue;
            {
                float lo = v[i], hi = v[i + s];
                v[i] = lo + hi;
                v[i + s] = lo - hi;
            }
        }
    }
}

/* y = A v (unscaled by h) for the FP32 pass. Bit k of `signs` negates v_k
 * first (the column signs of the n = 16 matrix). */
static void transform32(int n, int mat, uint32_t signs, const float *v_in,
                        float *y)
{
    float v[16];
    int k;
    for (k = 0; k < n; ++k) v[k] = ((signs >> k) & 1u) ? -v_in[k] : v_in[k];
    if (n == 4 && mat == 1) {
        /* A1 = J/2 - I = D_r P (H4/2) D_c with D_c = diag(-1,1,1,1),
         * P swapping rows 1 and 2, D_r = diag(1,-1,-1,-1). */
        v[0] = -v[0];
        fwht32(v, 4);
        y[0] = v[0];
        y[1] = -v[2];
        y[2] = -v[1];
        y[3] = -v[3];
        return;
    }
    fwht32(v, n);
    for (k = 0; k < n; ++k) y[k] = v[k];
}

void wo_pass32(int n, uint32_t N, int mat, const uint32_t *a,
               const uint32_t *b, uint32_t signs, float h, const float *X,
               float *Y)
{
    uint32_t j;
    int k;
    for (j = 0; j < N; ++j) {
        float v[16], u[16];
        for (k = 0; k < n; ++k) {
            uint64_t idx = ((uint64_t)a[k] * j + b[k]) % N; /* eq. 1 */
            v[k] = X[(size_t)k * N + idx];
        }
        transform32(n, mat, signs, v, u);
        for (k = 0; k < n; ++k) Y[(size_t)k * N + j] = u[k] * h;
    }
}

static int popcount_u(unsigned x)
{
    int c = 0;
    while (x) { c += (int)(x & 1u); x >>= 1; }
    return c;
}

/* Dense matrices, written from their definitions. */
void wo_matrix(int n, int mat, double *M)
{
    int i, j;
    for (i = 0; i < n; ++i) {
        for (j = 0; j < n; ++j) {
            double hij = (popcount_u((unsigned)(i & j)) & 1) ? -1.0 : 1.0;
            if (n == 4 && mat == 1)
                M[i * n + j] = 0.5 - (i == j ? 1.0 : 0.0);
            else
                M[i * n + j] = hij / sqrt((double)n);
        }
    }
}

void wo_pass64(int n, uint32_t N, int mat, const uint32_t *a,
               const uint32_t *b, uint32_t signs, double c, const double *X,
               double *Y)
{
    double M[256];
    uint32_t j;
    int k, i;
    wo_matrix(n, mat, M);
    for (k = 0; k < n; ++k) /* M <- M D, D = diag of the column signs */
        if ((signs >> k) & 1u)
            for (i = 0; i < n; ++i) M[i * n + k] = -M[i * n + k];
    for (j = 0; j < N; ++j) {
        double v[16];
        for (k = 0; k < n; ++k) {
            uint64_t idx = ((uint64_t)a[k] * j + b[k]) % N;
            v[k] = X[(size_t)k * N + idx];
        }
        for (k = 0; k < n; ++k) {
            double acc = 0.0;
            for (i = 0; i < n; ++i) acc += M[k * n + i] * v[i];
            Y[(size_t)k * N + j] = c * acc;
        }
    }
}

void wo_pass32_rot(uint32_t N, const uint32_t *a, const uint32_t *b, float p, float q,
                   const float *X, float *Y)
{
    uint32_t j;
    for (j = 0; j < N; ++j) {
        uint64_t ix = ((uint64_t)a[0] * j + b[0]) % N; /* eq. 1 */
        uint64_t iy = ((uint64_t)a[1] * j + b[1]) % N;
        float x = X[ix], y = X[(size_t)N + iy];
        float px = p * x, qy = q * y, py = p * y, qx = q * x;
        Y[j] = px + qy;
        Y[(size_t)N + j] = py - qx;
    }
}

void wo_pass64_rot(uint32_t N, const uint32_t *a, const uint32_t *b, double cs,
                   double sn, double c, const double *X, double *Y)
{
    double M[4];
    uint32_t j;
    int k, i;
    M[0] = cs; M[1] = sn; M[2] = -sn; M[3] = cs;
    for (j = 0; j < N; ++j) {
        double v[2];
        v[0] = X[((uint64_t)a[0] * j + b[0]) % N];
        v[1] = X[(size_t)N + ((uint64_t)a[1] * j + b[1]) % N];
        for (k = 0; k < 2; ++k) {
            double acc = 0.0;
            for (i = 0; i < 2; ++i) acc += M[k * 2 + i] * v[i];
            Y[(size_t)k * N + j] = c * acc;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Generators                                                                */
/* ------------------------------------------------------------------------ */

struct wo_gen {
    int n, fp64, sum_mode, a_mode, f, withhold;
    uint32_t N;
    size_t nu;
    uint64_t rng;      /* splitmix64 state */
    uint64_t restart;  /* refill the pool every `restart` passes (0: never) */
    double sigma;      /* sum of squares of the current pool */
    uint64_t passes;   /* passes done */
    size_t cursor;     /* values of the current output pool already emitted */
    float *X32, *Y32;  /* FP32 pool and its double buffer (section 2) */
    double *X64, *Y64; /* FP64 pool and its double buffer */
    double last_S, last_c64;
};

static size_t emit_len(const wo_gen *g)
{
    return g->withhold ? g->nu - 1 : g->nu;
}

static wo_gen *gen_alloc(uint64_t seed, int n, uint32_t N, int fp64)
{
    wo_gen *g = (wo_gen *)calloc(1, sizeof(wo_gen));
    g->n = n;
    g->N = N;
    g->nu = (size_t)n * N;
    g->fp64 = fp64;
    g->f = 1;
    g->rng = seed;
    g->X64 = (double *)malloc(g->nu * sizeof(double));
    g->Y64 = (double *)malloc(g->nu * sizeof(double));
    g->X32 = (float *)malloc(g->nu * sizeof(float));
    g->Y32 = (float *)malloc(g->nu * sizeof(float));
    wo_initial_pool64(&g->rng, n, N, g->X64);
    return g;
}

wo_gen *wo_gen_create(uint64_t seed, int n, uint32_t N, int sum_mode,
                      int a_mode, int f, int withhold)
{
    wo_gen *g = gen_alloc(seed, n, N, 0);
    size_t i;
    g->sum_mode = sum_mode;
    g->a_mode = a_mode;
    g->f = f < 1 ? 1 : f;
    g->withhold = withhold;
    for (i = 0; i < g->nu; ++i) g->X32[i] = (float)g->X64[i];
    g->sigma = wo_sumsq_mode(g->X32, g->nu, sum_mode);
    g->cursor = emit_len(g); /* the initial pool is not emitted */
    return g;
}

wo_gen *wo_gen64_create(uint64_t seed, int n, uint32_t N, int a_mode)
{
    wo_gen *g = gen_alloc(seed, n, N, 1);
    g->a_mode = a_mode;
    g->sigma = wo_sumsq_d(g->X64, g->nu);
    g->cursor = emit_len(g);
    return g;
}

void wo_gen_destroy(wo_gen *g)
{
    if (!g) return;
    free(g->X64);
    free(g->Y64);
    free(g->X32);
    free(g->Y32);
    free(g);
}

/* Section 5: restart after a fixed amount of output by refilling the pool
 * from the uniform generator with Box-Muller, as at initialisation. The
 * refilled pool is not output; the next pass transforms it. */
void wo_gen_set_restart(wo_gen *g, uint64_t passes) { g->restart = passes; }

static void gen_refill(wo_gen *g)
{
    size_t i;
    wo_initial_pool64(&g->rng, g->n, g->N, g->X64);
    if (g->fp64) {
        g->sigma = wo_sumsq_d(g->X64, g->nu);
    } else {
        for (i = 0; i < g->nu; ++i) g->X32[i] = (float)g->X64[i];
        g->sigma = wo_sumsq_mode(g->X32, g->nu, g->sum_mode);
    }
}

void wo_gen_pass(wo_gen *g)
{
    uint32_t a[16], b[16], signs;
    double rot[2];
    uint64_t p = g->passes + 1;
    if (g->restart && g->passes > 0 && g->passes % g->restart == 0) gen_refill(g);
    int mat = (g->n == 4) ? (int)((p - 1) % 2) : 0;
    wo_pass_params_rot(&g->rng, g->n, g->N, g->a_mode, a, b, &signs, rot);
    if (g->n == 2) {
        /* section 4: the chi-squared scale folds into the rotation */
        if (!g->fp64) {
            float *t;
            wo_scale32((double)g->X32[g->nu - 1], g->sigma, g->nu, &g->last_S,
                       &g->last_c64);
            wo_pass32_rot(g->N, a, b, (float)(g->last_c64 * rot[0]),
                          (float)(g->last_c64 * rot[1]), g->X32, g->Y32);
            t = g->X32; g->X32 = g->Y32; g->Y32 = t;
            g->sigma = wo_sumsq_mode(g->X32, g->nu, g->sum_mode);
        } else {
            double *t;
            wo_scale32(g->X64[g->nu - 1], g->sigma, g->nu, &g->last_S, &g->last_c64);
            wo_pass64_rot(g->N, a, b, rot[0], rot[1], g->last_c64, g->X64, g->Y64);
            t = g->X64; g->X64 = g->Y64; g->Y64 = t;
            g->sigma = wo_sumsq_d(g->X64, g->nu);
        }
        g->passes = p;
        return;
    }
    if (!g->fp64) {
        float c32 = wo_scale32((double)g->X32[g->nu - 1], g->sigma, g->nu,
                               &g->last_S, &g->last_c64);
        float h = c32 * (g->n == 4 ? 0.5f : 0.25f);
        float *t;
        wo_pass32(g->n, g->N, mat, a, b, signs, h, g->X32, g->Y32);
        t = g->X32; g->X32 = g->Y32; g->Y32 = t;
        g->sigma = wo_sumsq_mode(g->X32, g->nu, g->sum_mode);
    } else {
        double *t;
        wo_scale32(g->X64[g->nu - 1], g->sigma, g->nu, &g->last_S,
                   &g->last_c64);
        wo_pass64(g->n, g->N, mat, a, b, signs, g->last_c64, g->X64,
                  g->Y64);
        t = g->X64; g->X64 = g->Y64; g->Y64 = t;
        g->sigma = wo_sumsq_d(g->X64, g->nu);
    }
    g->passes = p;
}

void wo_gen_fill(wo_gen *g, float *out32, double *out64, uint64_t count)
{
    size_t len = emit_len(g);
    while (count > 0) {
        size_t m;
        if (g->cursor == len) {
            int i;
            for (i = 0; i < g->f; ++i) wo_gen_pass(g);
            g->cursor = 0;
        }
        m = len - g->cursor;
        if ((uint64_t)m > count) m = (size_t)count;
        if (out32) memcpy(out32, g->X32 + g->cursor, m * sizeof(float));
        if (out64) memcpy(out64, g->X64 + g->cursor, m * sizeof(double));
        if (out32) out32 += m;
        if (out64) out64 += m;
        g->cursor += m;
        count -= m;
    }
}

const float *wo_gen_pool32(const wo_gen *g) { return g->X32; }
const double *wo_gen_pool64(const wo_gen *g) { return g->X64; }
double wo_gen_sigma(const wo_gen *g) { return g->sigma; }
uint64_t wo_gen_passes(const wo_gen *g) { return g->passes; }
uint64_t wo_gen_rng(const wo_gen *g) { return g->rng; }
double wo_gen_last_S(const wo_gen *g) { return g->last_S; }
double wo_gen_last_c64(const wo_gen *g) { return g->last_c64; }
