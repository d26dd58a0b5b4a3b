// Streaming pass for pools too large to stay on chip (tens of MB). With the
// prime-pair strides (section 8) a pass is two launches:
//   permute: G_k[j] = X_k[(a_k j + b_k) mod N] (section 2, eq. 1). A block
//     loads a contiguous run of a*R values of X_k into LDS with coalesced
//     reads; the j whose source lies in that run form a+1 strands of R
//     consecutive j each, which the block writes as coalesced runs of G_k.
//   combine: reads G_k contiguously, applies the scaled transform, writes
//     the new pool in place of G and, when it is a returned pool, the
//     caller's output, plus one partial sum of squares (section 4) per
//     component and block.
// The partials are reduced, and the generator state advanced, by one extra
// block of the next pass's permute launch, or by a one-block finish launch
// after a call's last pass. The host passes each pass's splitmix64 state, so
// no permute block depends on the state that block rewrites.
// For n = 2 and 4 the combine of one pass and the permute of the next are
// one launch (k_stream_fuse), and a small launch forms the sum-of-squares
// component nodes between them; only the first pass of a call, or of the
// passes after a refill, runs the permute on its own.
// Arbitrary odd strides (eq. 2) use one launch that gathers from HBM, then
// the finish launch.
#include <mutex>
#include <type_traits>
#include <utility>
#include "wallace_devmath.hpp"
#include "wallace_runtime.h"

namespace wallace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

namespace {

struct F64 {
    double v;
    __device__ static F64 leaf(float y) { return {(double)y * (double)y}; }
    __device__ static F64 zero() { return {0.0}; }
    __device__ static F64 join(F64 a, F64 b) { return {a.v + b.v}; }
    __device__ static F64 xr(F64 a, int m) { return {__shfl_xor(a.v, m, 64)}; }
    __device__ static F64 sel(bool c, F64 a, F64 b) { return c ? a : b; }
    __device__ double value() const { return v; }
    __device__ double2 pack() const { return make_double2(v, 0.0); }
    __device__ static F64 unpack(double2 d) { return {d.x}; }
};

struct F32 {
    float v;
    __device__ static F32 leaf(float y) { return {y * y}; }
    __device__ static F32 zero() { return {0.0f}; }
    __device__ static F32 join(F32 a, F32 b) { return {a.v + b.v}; }
    __device__ static F32 xr(F32 a, int m) { return {__shfl_xor(a.v, m, 64)}; }
    __device__ static F32 sel(bool c, F32 a, F32 b) { return c ? a : b; }
    __device__ double value() const { return (double)v; }
    __device__ double2 pack() const { return make_double2((double)v, 0.0); }
    __device__ static F32 unpack(double2 d) { return {(float)d.x}; }
};

struct F32C {
    float s, e;
    __device__ static F32C leaf(float y)
    {
        float p = y * y;
        return {p, __builtin_fmaf(y, y, -p)};
    }
    __device__ static F32C zero() { return {0.0f, 0.0f}; }
    __device__ static F32C join(F32C a, F32C b)
    {
        float sum = a.s + b.s;
        float bb = sum - a.s;
        float err = (a.s - (sum - bb)) + (b.s - bb);
        return {sum, (a.e + b.e) + err};
    }
    __device__ static F32C xr(F32C a, int m)
    {
        return {__shfl_xor(a.s, m, 64), __shfl_xor(a.e, m, 64)};
    }
    __device__ static F32C sel(bool c, F32C a, F32C b) { return c ? a : b; }
    __device__ double value() const { return (double)s + (double)e; }
    __device__ double2 pack() const { return make_double2((double)s, (double)e); }
    __device__ static F32C unpack(double2 d) { return {(float)d.x, (float)d.y}; }
};

// Compile-time loop: f(integral_constant<int, I>) for I in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void static_for_k(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        static_for_k<B + 1, E>(f);
    }
}

template <int V>
struct Lg {
    static constexpr int value = 1 + Lg<V / 2>::value;
};
template <>
struct Lg<1> {
    static constexpr int value = 0;
};

constexpr int kThreads = 256;

// A thread's T consecutive values of one component (16-, 8- or 4-byte
// accesses). NT: nontemporal loads. The n = 4 fused pass reads its
// permuted components with them (read once; the caches are left to the next
// pass's permuted components, written in the same pass and read in the
// next): at N = 2^22 that took the pass from 44.6 to 40.6 us on MI355X. The
// permute kernel reads its source runs the same way.
template <int T, bool NT>
__device__ __forceinline__ void load_run(float (&x)[T], const float *p)
{
    if constexpr (T % 4 == 0) {
#pragma unroll
        for (int i = 0; i < T; i += 4) {
            const v4f *src = reinterpret_cast<const v4f *>(p + i);
            v4f q;
            if constexpr (NT)
                q = __builtin_nontemporal_load(src);
            else
                q = *src;
            x[i] = q.x;
            x[i + 1] = q.y;
            x[i + 2] = q.z;
            x[i + 3] = q.w;
        }
    } else if constexpr (T == 2) {
        const v2f *src = reinterpret_cast<const v2f *>(p);
        v2f q;
        if constexpr (NT)
            q = __builtin_nontemporal_load(src);
        else
            q = *src;
        x[0] = q.x;
        x[1] = q.y;
    } else {
        if constexpr (NT)
            x[0] = __builtin_nontemporal_load(p);
        else
            x[0] = p[0];
    }
}

// A lane's T consecutive values to global memory; NT: nontemporal stores
// (the returned pools, written once and never read back). NT is a template
// parameter: with a run-time flag the compiler merged the two forms into
// one store and dropped the nontemporal hint (3.8% of the batched store
// rate on MI355X).
template <int T, bool NT>
__device__ __forceinline__ void store_run(float *p, const float (&x)[T])
{
    if constexpr (T % 4 == 0) {
#pragma unroll
        for (int i = 0; i < T; i += 4) {
            const v4f q = {x[i], x[i + 1], x[i + 2], x[i + 3]};
            if constexpr (NT)
                __builtin_nontemporal_store(q, reinterpret_cast<v4f *>(p + i));
            else
                *reinterpret_cast<v4f *>(p + i) = q;
        }
    } else if constexpr (T == 2) {
        const v2f q = {x[0], x[1]};
        if constexpr (NT)
            __builtin_nontemporal_store(q, reinterpret_cast<v2f *>(p));
        else
            *reinterpret_cast<v2f *>(p) = q;
    } else {
        if constexpr (NT)
            __builtin_nontemporal_store(x[0], p);
        else
            p[0] = x[0];
    }
}

struct Pass {
    const float *X;   // old pool
    const float *G;   // permuted components (PERM kernels), else unused
    float *Y;         // new pool
    float *out;       // returned copy of the new pool (NULL: not returned)
    uint32_t emit_cnt;
    uint32_t affine;
    float mu, sig;
    GenState *state;
    double2 *partials;  // [n][nblocks]
    double r_nu;
    uint64_t rng;       // splitmix64 state the pass draws from
    const double2 *comp;  // non-null: the old pool's sum of squares is the tree
                          // over these per-component nodes (else state.sigma)
    uint64_t passes;    // passes done once this pass is complete
    uint32_t mat;       // n = 4: 1 for A1 (the pass after an odd count of passes)
    uint32_t N;
    uint32_t a_mode;
    uint32_t nblocks;
};

// Per-block partial sums for every component: the block's tuples
// [j0, j0 + 256 T) form an aligned subtree of each component's part of the
// canonical tree over the flat index.
template <class Nd, int NC, int T, int NW = kThreads / 64>
__device__ void block_partials(const float (&X)[NC][T], double2 *dst,
                               uint32_t nblocks, double2 *red, uint32_t bid)
{
    constexpr int LOG_NC = Lg<NC>::value;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    Nd v[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        Nd t[T];
#pragma unroll
        for (int i = 0; i < T; ++i) t[i] = Nd::leaf(X[k][i]);
#pragma unroll
        for (int w = T; w > 1; w >>= 1) {
#pragma unroll
            for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
        }
        v[k] = t[0];
    }
#pragma unroll
    for (int m = 0; m < LOG_NC; ++m) {
        const int V = NC >> m;
        const bool hi = (lane >> m) & 1;
#pragma unroll
        for (int t = 0; t < V / 2; ++t) {
            Nd keep = Nd::sel(hi, v[t + V / 2], v[t]);
            Nd send = Nd::sel(hi, v[t], v[t + V / 2]);
            v[t] = Nd::join(keep, Nd::xr(send, 1 << m));
        }
    }
    Nd acc = v[0];
#pragma unroll
    for (int m = LOG_NC; m < 6; ++m) acc = Nd::join(acc, Nd::xr(acc, 1 << m));
    int kappa = 0;
#pragma unroll
    for (int m = 0; m < LOG_NC; ++m) kappa |= ((lane >> m) & 1) << (LOG_NC - 1 - m);
    if (lane < NC) red[wave * NC + kappa] = acc.pack();
    __syncthreads();
    if (threadIdx.x < NC) {
        // the block's NW wave nodes of component k, in tree order
        const int k = threadIdx.x;
        Nd t[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) t[w] = Nd::unpack(red[w * NC + k]);
#pragma unroll
        for (int w = NW; w > 1; w >>= 1) {
#pragma unroll
            for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
        }
        dst[(size_t)k * nblocks + bid] = t[0].pack();
    }
}

// Tree over PB consecutive partial nodes.
template <class Nd, int PB>
__device__ __forceinline__ Nd run_tree(const double2 *p)
{
    Nd t[PB];
#pragma unroll
    for (int i = 0; i < PB; ++i) t[i] = Nd::unpack(p[i]);
#pragma unroll
    for (int w = PB; w > 1; w >>= 1) {
#pragma unroll
        for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
    }
    return t[0];
}

// Canonical tree over the n*nblocks partial nodes (nblocks a power of two,
// at most 16 per thread): per component over its blocks, then over the
// components. A thread's run of nodes is joined four at a time in tree
// order; missing nodes are zeros, which join exactly. NT threads.
template <class Nd, int NT>
__device__ __forceinline__ Nd thread_run(const double2 *p, uint32_t per)
{
    if (per == 1) return run_tree<Nd, 1>(p);
    if (per == 2) return run_tree<Nd, 2>(p);
    if (per == 4) return run_tree<Nd, 4>(p);
    const Nd q0 = run_tree<Nd, 4>(p), q1 = run_tree<Nd, 4>(p + 4);
    const Nd h0 = Nd::join(q0, q1);
    if (per == 8) return h0;
    const Nd q2 = run_tree<Nd, 4>(p + 8), q3 = run_tree<Nd, 4>(p + 12);
    return Nd::join(h0, Nd::join(q2, q3));
}

template <class Nd, int NC, int NT>
__device__ double final_tree(const double2 *partials, uint32_t nblocks)
{
    constexpr int NW = NT / 64;
    __shared__ double2 wv[NC][NW];
    __shared__ double2 comp[NC];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t per = nblocks > NT ? nblocks / NT : 1u;
    const uint32_t b0 = threadIdx.x * per;
    for (int k = 0; k < NC; ++k) {
        Nd acc = Nd::zero();
        if (b0 < nblocks) acc = thread_run<Nd, NT>(partials + (size_t)k * nblocks + b0, per);
#pragma unroll
        for (int m = 0; m < 6; ++m) acc = Nd::join(acc, Nd::xr(acc, 1 << m));
        if (lane == 0) wv[k][wave] = acc.pack();
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        const int k = threadIdx.x;
        Nd t[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) t[w] = Nd::unpack(wv[k][w]);
#pragma unroll
        for (int w = NW; w > 1; w >>= 1) {
#pragma unroll
            for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
        }
        comp[k] = t[0].pack();
    }
    __syncthreads();
    double out = 0.0;
    if (threadIdx.x == 0) {
        Nd t[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) t[k] = Nd::unpack(comp[k]);
#pragma unroll
        for (int w = NC; w > 1; w >>= 1) {
#pragma unroll
            for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
        }
        out = t[0].value();
    }
    return out;
}

// Completes a call's pass from its partials: the new sum of squares, the
// pass count and the splitmix64 state after the pass's draws (both known to
// the host). NONFINITE was already set by the pass kernel; CORRUPT stops
// everything.
template <class Nd, int NC, int NT>
__device__ void finish_pass(GenState *state, const double2 *partials, uint32_t nblocks,
                            uint64_t passes, uint64_t rng_next)
{
    if (state->flags & WALLACE_FLAG_CORRUPT) return;
    const double sigma = final_tree<Nd, NC, NT>(partials, nblocks);
    if (threadIdx.x == 0) {
        state->sigma = sigma;
        state->passes = passes;
        state->rng = rng_next;
    }
}

// One component's node of the canonical tree: the tree over its nblocks
// partial nodes (a power of two, at most 16 per thread), by one block of NT
// threads. Thread 0 returns it.
template <class Nd, int NT>
__device__ Nd comp_sum(const double2 *p, uint32_t nblocks)
{
    constexpr int NW = NT / 64;
    __shared__ double2 wv[NW];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t per = nblocks > NT ? nblocks / NT : 1u;
    const uint32_t b0 = threadIdx.x * per;
    Nd acc = Nd::zero();
    if (b0 < nblocks) acc = thread_run<Nd, NT>(p + b0, per);
#pragma unroll
    for (int m = 0; m < 6; ++m) acc = Nd::join(acc, Nd::xr(acc, 1 << m));
    if (lane == 0) wv[wave] = acc.pack();
    __syncthreads();
    Nd t[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) t[w] = Nd::unpack(wv[w]);
#pragma unroll
    for (int w = NW; w > 1; w >>= 1) {
#pragma unroll
        for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
    }
    return t[0];
}

// LDS run of the permute kernel: at most run_floats(n) source values. Runs
// of 4096 values (16 KB) gave n = 4 the most blocks in flight; n = 16, with
// strides up to 137, needs 8192 to keep its strands at 64 values or more.
constexpr uint32_t kRunFloatsMax = 8192;
__host__ __device__ constexpr uint32_t run_floats(int n) { return n == 16 ? 8192u : 4096u; }

// Splitmix64 draws per pass: one per component, one more for the n = 2
// rotation (section 8).
__host__ __device__ constexpr uint32_t draws_per_pass(int n) { return n == 2 ? 3u : (uint32_t)n; }
constexpr int kMaxStrands = 160;  // a + 1 for the largest prime-pair stride

struct Perm {
    const float *X;        // old pool
    float *G;              // permuted components
    GenState *state;
    uint64_t rng;          // splitmix64 state the pass draws from
    const double2 *partials;  // previous pass's partial sums [n][fin_nblocks]
    double2 *comp;         // its per-component nodes, written by the finish blocks
    uint32_t fin_nblocks;
    uint32_t fin;          // 1: the grid's last n blocks reduce the previous pass
    uint32_t N;
    uint32_t first[17];    // first block of component k; first[n] = grid
    uint32_t logR[16];     // strand length R_k = 2^logR[k]
    float *xs;             // non-null: receives the old pool's last flat value
};

// Permute kernel (see the file comment). Block (k, c) covers source values
// x in [c a R, c a R + a R) of component k; strand w holds the j with
// a j + b - w N in that run, j = c R + s_w + t (t < R) and
// x = c a R + r_w + a t, where s_w = ceil((w N - b) / a) and
// r_w = a s_w + b - w N lies in [0, a).
template <class Nd, int NC>
__global__ __launch_bounds__(kThreads) void k_stream_permute(Perm P)
{
    extern __shared__ __attribute__((aligned(16))) float run[];
    __shared__ int32_t s_tab[kMaxStrands];
    __shared__ int32_t r_tab[kMaxStrands];
    if (P.fin && blockIdx.x >= P.first[NC]) {
        // previous pass, component k: its node for the next pass kernel
        const uint32_t k = blockIdx.x - P.first[NC];
        const Nd r = comp_sum<Nd, kThreads>(P.partials + (size_t)k * P.fin_nblocks, P.fin_nblocks);
        if (threadIdx.x == 0) P.comp[k] = r.pack();
        return;
    }
    if (P.state->flags & WALLACE_FLAG_CORRUPT) return;
    const uint32_t N = P.N;
    if (P.xs && blockIdx.x == 0 && threadIdx.x == 0) *P.xs = P.X[(size_t)NC * N - 1];
    int k = 0;
#pragma unroll
    for (int q = 1; q < NC; ++q) k += blockIdx.x >= P.first[q] ? 1 : 0;
    const uint32_t c = blockIdx.x - P.first[k];
    // draw k + 1 of the pass (the same draw the combine kernel makes)
    uint64_t rng = P.rng + (uint64_t)k * 0x9E3779B97F4A7C15ull;
    const uint64_t w64 = sm64_next(rng);
    const uint32_t a = stride_pick(k, (uint32_t)(w64 >> 63)) & (N - 1u);
    const uint32_t b = (uint32_t)w64 & (N - 1u);
    const uint32_t logR = P.logR[k];
    const uint32_t R = 1u << logR;
    const uint64_t X0 = (uint64_t)c * a * R;
    if (X0 >= N) return;  // the larger stride of the pair needs fewer blocks
    const uint32_t len = (uint32_t)(N - X0 < (uint64_t)a * R ? N - X0 : (uint64_t)a * R);

    const float *src = P.X + (size_t)k * N + X0;
    for (uint32_t i = threadIdx.x * 4u; i < len; i += kThreads * 4u)
        *reinterpret_cast<v4f *>(run + i) =
            __builtin_nontemporal_load(reinterpret_cast<const v4f *>(src + i));
    for (uint32_t w = threadIdx.x; w <= a; w += kThreads) {
        // ceil(num / a) through one correctly rounded FP64 division: |num| <
        // 2^32, and a non-integral quotient lies at least 1/a from an
        // integer, far above its rounding error
        const int64_t num = (int64_t)w * (int64_t)N - (int64_t)b;
        const int64_t q = (int64_t)__builtin_ceil((double)num / (double)a);
        s_tab[w] = (int32_t)q;
        r_tab[w] = (int32_t)(q * (int64_t)a - num);
    }
    __syncthreads();

    // Strand w covers j in [js, js + R), js = c R + s_w, read from the run at
    // r_w + a (j - js). Threads take aligned quads of j: interior quads are
    // one 16-byte store; the quads at the ends of a strand (and of the pool)
    // store their valid values one by one.
    float *g = P.G + (size_t)k * N;
    const int64_t jc = (int64_t)c * R;
    const uint32_t Q = (R >> 2) + 1u;  // aligned quads that cover R values
    const float rq = 1.0f / (float)Q;
    const uint32_t pairs = (a + 1u) * Q;
#pragma unroll 2
    for (uint32_t pr = threadIdx.x; pr < pairs; pr += kThreads) {
        uint32_t w = (uint32_t)((float)pr * rq);
        w = w * Q > pr ? w - 1u : ((w + 1u) * Q <= pr ? w + 1u : w);
        const uint32_t u = pr - w * Q;
        const int64_t js = jc + s_tab[w];
        const int64_t q0 = (js & ~(int64_t)3) + 4 * (int64_t)u;
        const int32_t t0 = (int32_t)(q0 - js);  // in [-3, R + 3)
        const uint32_t r = (uint32_t)r_tab[w];
        if (t0 >= 0 && t0 + 3 < (int32_t)R && q0 >= 0 && q0 + 3 < (int64_t)N &&
            r + a * (uint32_t)(t0 + 3) < len) {
            const uint32_t x0 = r + a * (uint32_t)t0;
            const v4f v = {run[x0], run[x0 + a], run[x0 + 2u * a], run[x0 + 3u * a]};
            *reinterpret_cast<v4f *>(g + q0) = v;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int32_t t = t0 + e;
                const int64_t j = q0 + e;
                if (t >= 0 && t < (int32_t)R && j >= 0 && j < (int64_t)N) {
                    const uint32_t xo = r + a * (uint32_t)t;
                    if (xo < len) g[j] = run[xo];
                }
            }
        }
    }
}

// n = 16 transform on the matrix cores (accuracy variant, not bit-exact):
// y = (h H16 D) v for 16 tuples per MFMA group. A wave's 64 tuples go
// through LDS: lane l of group g feeds component 4s + l/16 of tuple
// 16g + l%16 at step s (B operand, 4 x 16) against the 16 x 4 slice
// h H16[m][4s + kk] d_(4s + kk) (A operand), and receives components
// 4(l/16) .. 4(l/16)+3 of tuple 16g + l%16.
__device__ __forceinline__ void xform16_mfma(float (&v)[16], uint32_t signs, float h,
                                             float (*tile)[kThreads + 16])
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int base = tid & ~63;  // this wave's first tuple in the block
#pragma unroll
    for (int k = 0; k < 16; ++k) tile[k][tid] = v[k];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // wave-local LDS, in order
    const int m = lane & 15, q = lane >> 4;
    float a[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int kk = 4 * st + q;
        const int odd = (__builtin_popcount((unsigned)(m & kk)) + (int)((signs >> kk) & 1u)) & 1;
        a[st] = odd ? -h : h;
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int col = base + 16 * g + m;
        v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int st = 0; st < 4; ++st)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st], tile[4 * st + q][col], acc, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) tile[4 * q + i][col] = acc[i];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = tile[k][tid];
}

template <class Nd, int NC, int T, bool PERM, bool MF>
__global__ __launch_bounds__(kThreads) void k_stream_pass(Pass P)
{
    static_assert(!MF || (NC == 16 && T == 1), "matrix-core transform: n = 16, one tuple per thread");
    __shared__ double2 red[4 * NC];
    __shared__ float tile[MF ? 16 : 1][kThreads + 16];
    const GenState st = *P.state;
    if (st.flags & WALLACE_FLAG_CORRUPT) return;
    const uint32_t N = P.N;
    const uint32_t mask = N - 1u;
    const uint32_t nu = NC * N;

    uint64_t rng = P.rng;
    uint32_t a[NC], b[NC], signs = 0;
    // strides distinct and above one (sections 3, 9): streamed pools are
    // larger than every table prime, so only any-odd strides can clash
    static_for_k<0, NC>([&](auto k_c) {
        constexpr int k = decltype(k_c)::value;
        const uint64_t w = sm64_next(rng);
        const uint32_t ak = P.a_mode ? ((uint32_t)(w >> 32) | 1u)
                                     : stride_pick(k, (uint32_t)(w >> 63));
        a[k] = ak & mask;
        if (P.a_mode) a[k] = distinct_stride<k>(a[k], a, N);
        b[k] = (uint32_t)w & mask;
        if (NC == 16) signs |= (uint32_t)((w >> 62) & 1u) << k;
    });
    double rcs = 0.0, rsn = 0.0;  // n = 2: the pass's rotation (draw n + 1)
    if constexpr (NC == 2) rotation(sm64_next(rng), rcs, rsn);
    const int mat = (NC == 4) ? (int)P.mat : 0;

    // the tuples' values first, so that the loads are in flight while the
    // scale below is computed
    const uint32_t j0 = (blockIdx.x * kThreads + threadIdx.x) * (uint32_t)T;
    float X[NC][T];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if constexpr (PERM) {
            // plain loads: its new pool overwrites G in place, and
            // nontemporal loads here cost 4-5 us per pass at n = 16, N = 2^20
            load_run<T, false>(X[k], P.G + (size_t)k * N + j0);
        } else {
            const float *src = P.X + (size_t)k * N;
#pragma unroll
            for (int i = 0; i < T; ++i) X[k][i] = src[(a[k] * (j0 + i) + b[k]) & mask];
        }
    }

    // chi-squared scale from the old pool (section 4, eq. 3)
    const double xstar = (double)P.X[nu - 1];
    const double S = chi2_target(xstar, P.r_nu);
    double sigma_old = st.sigma;
    if (P.comp) {  // the previous pass of this call, from its component nodes
        Nd t[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) t[k] = Nd::unpack(P.comp[k]);
#pragma unroll
        for (int w = NC; w > 1; w >>= 1) {
#pragma unroll
            for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
        }
        sigma_old = t[0].value();
    }
    const double c64 = chi2_scale_from_S(S, sigma_old);
    const float c32 = (float)c64;
    const float h = c32 * (NC == 4 ? 0.5f : 0.25f);
    // n = 2: c folds into the rotation entries, each rounded once (section 4)
    const float rp = NC == 2 ? (float)(c64 * rcs) : 0.0f;
    const float rq = NC == 2 ? (float)(c64 * rsn) : 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0 && !__builtin_isfinite(c32))
        atomicOr(&P.state->flags, (uint32_t)WALLACE_FLAG_NONFINITE);

#pragma unroll
    for (int i = 0; i < T; ++i) {
        float v[NC];
        if constexpr (MF) {
#pragma unroll
            for (int k = 0; k < NC; ++k) v[k] = X[k][i];
            xform16_mfma(v, signs, h, tile);
#pragma unroll
            for (int k = 0; k < NC; ++k) X[k][i] = v[k];
            continue;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = ((signs >> k) & 1u) ? -X[k][i] : X[k][i];
        if constexpr (NC == 2) {
            const float px = rp * v[0], qy = rq * v[1], py = rp * v[1], qx = rq * v[0];
            v[0] = px + qy;
            v[1] = py - qx;
        } else if constexpr (NC == 4) {
            const float v0 = mat ? -v[0] : v[0];
            const float s0 = v0 + v[1], s1 = v0 - v[1];
            const float s2 = v[2] + v[3], s3 = v[2] - v[3];
            const float u0 = s0 + s2, u1 = s1 + s3, u2 = s0 - s2, u3 = s1 - s3;
            if (mat) {
                v[0] = u0 * h; v[1] = (-u2) * h; v[2] = (-u1) * h; v[3] = (-u3) * h;
            } else {
                v[0] = u0 * h; v[1] = u1 * h; v[2] = u2 * h; v[3] = u3 * h;
            }
        } else {
#pragma unroll
            for (int s = 1; s < NC; s <<= 1) {
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    if (q & s) continue;
                    const float lo = v[q], hi = v[q + s];
                    v[q] = lo + hi;
                    v[q + s] = lo - hi;
                }
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) v[k] = v[k] * h;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) X[k][i] = v[k];
    }

    // write back the new pool; return it if requested (flat order)
#pragma unroll
    for (int k = 0; k < NC; ++k) store_run<T, false>(P.Y + (size_t)k * N + j0, X[k]);
    if (P.out) {
        const bool vec = P.emit_cnt == nu && !P.affine &&
                         ((uintptr_t)P.out & (uintptr_t)(4 * (T < 4 ? T : 4) - 1)) == 0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            float *dst = P.out + (size_t)k * N + j0;
            if (vec) {
                store_run<T, true>(dst, X[k]);
            } else {
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const uint32_t fl = (uint32_t)k * N + j0 + i;
                    if (fl < P.emit_cnt) {
                        float y = X[k][i];
                        if (P.affine) y = P.mu + P.sig * y;
                        __builtin_nontemporal_store(y, dst + i);
                    }
                }
            }
        }
    }

    block_partials<Nd, NC, T>(X, P.partials, P.nblocks, red, blockIdx.x);
}

// Finish of a call's last pass (one block, after the pass kernel), and of
// every pass of the gather form. A launch of its own: no block of the pass
// kernel needs a device-wide fence (each would write back the whole L2).
template <class Nd, int NC>
__global__ __launch_bounds__(kThreads) void k_stream_finish(Pass P)
{
    finish_pass<Nd, NC, kThreads>(P.state, P.partials, P.nblocks, P.passes,
                                  P.rng + (uint64_t)draws_per_pass(NC) * 0x9E3779B97F4A7C15ull);
}

// Fused streamed pass (prime-pair strides, n = 2 and 4): the combine of
// pass p and the permutation of pass p + 1 in one launch. Block c owns
// tuples [c S, c S + S) with S = 1024 T. It reads their permuted values G_k
// (written by the previous launch), applies the scaled transform, writes
// the returned pool and its partial sums of squares (section 4), then
// keeps the new values in LDS and writes the strands of the next pass's
// permuted components G'_k[j] = X'_k[(a'_k j + b'_k) mod N] (eq. 1) whose
// sources lie in its run: strand w holds the j with a' j + b' - w N in
// [c S, c S + S), from s_w = ceil((c S + w N - b') / a') up to
// e_w = ceil((c S + S + w N - b') / a'). Every j of every component is
// written by exactly one block and strand. A value then costs 12 bytes of
// traffic per pass (read G, write the output, write G') instead of 16 with a
// separate permute and combine. The old pool's sum of squares comes from the
// previous pass's component nodes (k_stream_comp) and its last flat value
// from a slot that the previous launch wrote.
constexpr int kFuseThreads = 1024;
constexpr int kFuseStrands = 24;  // a + 1 for the largest stride of n <= 4

struct Fuse {
    const float *G;       // this pass's permuted components
    float *Y;             // the new pool in the workspace (NULL: not kept)
    float *out;           // returned copy (NULL: not returned); may be G
    float *Gn;            // next pass's permuted components (NULL: none)
    uint32_t emit_cnt;
    uint32_t affine;
    float mu, sig;
    GenState *state;
    double2 *partials;    // [n][nblocks]
    const double2 *comp;  // previous pass's component nodes (NULL: state.sigma)
    const float *xs_in;   // the old pool's last flat value
    float *xs_out;        // receives the new pool's last flat value (or NULL)
    double r_nu;
    uint64_t rng;         // splitmix64 state this pass draws from
    uint64_t rng_next;    // and the next pass
    uint32_t mat;         // n = 4: 1 for A1
    uint32_t N;
    uint32_t nblocks;
};

template <class Nd, int NC, int T>
__global__ __launch_bounds__(kFuseThreads) void k_stream_fuse(Fuse P)
{
    static_assert(NC == 2 || NC == 4, "strides up to 23");
    constexpr uint32_t S = (uint32_t)kFuseThreads * T;  // tuples per block
    constexpr int NW = kFuseThreads / 64;
    extern __shared__ __attribute__((aligned(16))) float run[];  // NC * S floats
    __shared__ double2 red[NW * NC];
    __shared__ int32_t s_tab[NC][kFuseStrands];
    __shared__ int32_t e_tab[NC][kFuseStrands];
    __shared__ int32_t r_tab[NC][kFuseStrands];
    const GenState st = *P.state;
    if (st.flags & WALLACE_FLAG_CORRUPT) return;
    const uint32_t N = P.N;
    const uint32_t mask = N - 1u;
    const uint32_t nu = NC * N;

    // Workgroups go round-robin to the 8 XCDs; block b takes tuple range
    // cb = (b mod 8) G/8 + b/8 instead, so each XCD covers one contiguous
    // eighth of the pool and the strand ends that adjacent ranges write to
    // the same lines of G' meet in one L2 (n = 2: 3.5% per pass). The
    // block's values are loaded first, so that the loads are in flight
    // while the scale below is computed (0.7 us of 40.6 per pass at n = 4,
    // N = 2^22). Nontemporal for n = 4 only: at n = 2, N = 2^23 they cost
    // 1.3 us per pass (43.6 against 42.3).
    const uint32_t cb = (gridDim.x % 8u) ? blockIdx.x
                                          : (blockIdx.x % 8u) * (gridDim.x / 8u) + blockIdx.x / 8u;
    const uint32_t j0 = cb * S + threadIdx.x * (uint32_t)T;
    float X[NC][T];
#pragma unroll
    for (int k = 0; k < NC; ++k) load_run<T, NC == 4>(X[k], P.G + (size_t)k * N + j0);

    double rcs = 0.0, rsn = 0.0;  // n = 2: the pass's rotation (draw n + 1)
    if constexpr (NC == 2) {
        uint64_t rng = P.rng + (uint64_t)NC * 0x9E3779B97F4A7C15ull;
        rotation(sm64_next(rng), rcs, rsn);
    }
    const int mat = (NC == 4) ? (int)P.mat : 0;

    // chi-squared scale from the old pool (section 4, eq. 3)
    const double xstar = (double)*P.xs_in;
    const double Sq = chi2_target(xstar, P.r_nu);
    double sigma_old = st.sigma;
    if (P.comp) {
        Nd tc[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) tc[k] = Nd::unpack(P.comp[k]);
#pragma unroll
        for (int w = NC; w > 1; w >>= 1) {
#pragma unroll
            for (int i = 0; i < w / 2; ++i) tc[i] = Nd::join(tc[2 * i], tc[2 * i + 1]);
        }
        sigma_old = tc[0].value();
    }
    const double c64 = chi2_scale_from_S(Sq, sigma_old);
    const float c32 = (float)c64;
    const float h = c32 * (NC == 4 ? 0.5f : 0.25f);
    const float rp = NC == 2 ? (float)(c64 * rcs) : 0.0f;
    const float rq = NC == 2 ? (float)(c64 * rsn) : 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0 && !__builtin_isfinite(c32))
        atomicOr(&P.state->flags, (uint32_t)WALLACE_FLAG_NONFINITE);

#pragma unroll
    for (int i = 0; i < T; ++i) {
        float v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = X[k][i];
        if constexpr (NC == 2) {
            const float px = rp * v[0], qy = rq * v[1], py = rp * v[1], qx = rq * v[0];
            v[0] = px + qy;
            v[1] = py - qx;
        } else {
            const float v0 = mat ? -v[0] : v[0];
            const float s0 = v0 + v[1], s1 = v0 - v[1];
            const float s2 = v[2] + v[3], s3 = v[2] - v[3];
            const float u0 = s0 + s2, u1 = s1 + s3, u2 = s0 - s2, u3 = s1 - s3;
            if (mat) {
                v[0] = u0 * h; v[1] = (-u2) * h; v[2] = (-u1) * h; v[3] = (-u3) * h;
            } else {
                v[0] = u0 * h; v[1] = u1 * h; v[2] = u2 * h; v[3] = u3 * h;
            }
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) X[k][i] = v[k];
    }

    // the new pool: workspace copy, returned copy (flat order)
    if (P.Y) {
#pragma unroll
        for (int k = 0; k < NC; ++k) store_run<T, false>(P.Y + (size_t)k * N + j0, X[k]);
    }
    if (P.out) {
        const bool vec = P.emit_cnt == nu && !P.affine && ((uintptr_t)P.out & 15u) == 0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            float *dst = P.out + (size_t)k * N + j0;
            if (vec) {
                store_run<T, true>(dst, X[k]);
            } else {
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const uint32_t fl = (uint32_t)k * N + j0 + i;
                    if (fl < P.emit_cnt) {
                        float y = X[k][i];
                        if (P.affine) y = P.mu + P.sig * y;
                        __builtin_nontemporal_store(y, dst + i);
                    }
                }
            }
        }
    }
    if (P.xs_out && j0 + (uint32_t)T == N) *P.xs_out = X[NC - 1][T - 1];
    block_partials<Nd, NC, T, NW>(X, P.partials, P.nblocks, red, cb);
    if (!P.Gn) return;

    // next pass's strides and offsets (its draws 1 .. n, section 8)
    uint32_t an[NC], bn[NC];
    {
        uint64_t r2 = P.rng_next;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const uint64_t w = sm64_next(r2);
            an[k] = stride_pick(k, (uint32_t)(w >> 63)) & mask;
            bn[k] = (uint32_t)w & mask;
        }
    }
    // the new values in LDS, tuple order, one component after another
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if constexpr (T % 4 == 0) {
#pragma unroll
            for (int i = 0; i < T; i += 4)
                *reinterpret_cast<v4f *>(run + k * S + threadIdx.x * T + i) =
                    v4f{X[k][i], X[k][i + 1], X[k][i + 2], X[k][i + 3]};
        } else {
#pragma unroll
            for (int i = 0; i < T; ++i) run[k * S + threadIdx.x * T + i] = X[k][i];
        }
    }
    const int64_t x0 = (int64_t)cb * S;
    for (uint32_t idx = threadIdx.x; idx < (uint32_t)(NC * kFuseStrands); idx += kFuseThreads) {
        const int k = (int)(idx / kFuseStrands);
        const uint32_t w = idx % kFuseStrands;
        uint32_t a = 0, b = 0;
#pragma unroll
        for (int q = 0; q < NC; ++q)
            if (q == k) { a = an[q]; b = bn[q]; }
        if (w <= a) {
            // ceil through one correctly rounded FP64 division (|num| < 2^32;
            // a non-integral quotient lies at least 1/a from an integer)
            const int64_t num = x0 + (int64_t)w * (int64_t)N - (int64_t)b;
            const int64_t q = (int64_t)__builtin_ceil((double)num / (double)a);
            const int64_t qe = (int64_t)__builtin_ceil((double)(num + (int64_t)S) / (double)a);
            s_tab[k][w] = (int32_t)q;
            e_tab[k][w] = (int32_t)qe;
            r_tab[k][w] = (int32_t)(q * (int64_t)a - num);
        }
    }
    __syncthreads();

    // strand w of component k: j in [s_w, e_w) (clipped to [0, N)), value
    // run[r_w + a (j - s_w)]. Threads take aligned quads of j: quads inside a
    // strand are one 16-byte store, the ones at its ends store their valid
    // values one by one.
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const uint32_t a = an[k];
        const uint32_t lmax = (S + a - 1u) / a;  // longest strand
        const uint32_t Q = (lmax + 3u) / 4u + 1u;
        const float rqq = 1.0f / (float)Q;
        const uint32_t pairs = (a + 1u) * Q;
        float *g = P.Gn + (size_t)k * N;
        const float *rk = run + k * S;
        for (uint32_t pr = threadIdx.x; pr < pairs; pr += kFuseThreads) {
            uint32_t w = (uint32_t)((float)pr * rqq);
            w = w * Q > pr ? w - 1u : ((w + 1u) * Q <= pr ? w + 1u : w);
            const uint32_t u = pr - w * Q;
            const int64_t js = s_tab[k][w];
            const int64_t je = e_tab[k][w];
            const uint32_t r = (uint32_t)r_tab[k][w];
            const int64_t q0 = (js & ~(int64_t)3) + 4 * (int64_t)u;
            if (q0 >= js && q0 + 3 < je && q0 >= 0 && q0 + 3 < (int64_t)N) {
                const uint32_t xo = r + a * (uint32_t)(q0 - js);
                const v4f v = {rk[xo], rk[xo + a], rk[xo + 2u * a], rk[xo + 3u * a]};
                *reinterpret_cast<v4f *>(g + q0) = v;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t j = q0 + e;
                    if (j >= js && j < je && j >= 0 && j < (int64_t)N)
                        g[j] = rk[r + a * (uint32_t)(j - js)];
                }
            }
        }
    }
}

// Per-component nodes of a fused pass's sum of squares (one block each),
// read by the next fused pass.
template <class Nd>
__global__ __launch_bounds__(kThreads) void k_stream_comp(const double2 *partials,
                                                          uint32_t nblocks, double2 *comp)
{
    const uint32_t k = blockIdx.x;
    const Nd r = comp_sum<Nd, kThreads>(partials + (size_t)k * nblocks, nblocks);
    if (threadIdx.x == 0) comp[k] = r.pack();
}

template <int NC>
const void *fuse_fn(uint32_t rmode)
{
    constexpr int T = 16 / NC;
    if (rmode == 1) return reinterpret_cast<const void *>(&k_stream_fuse<F32, NC, T>);
    if (rmode == 2) return reinterpret_cast<const void *>(&k_stream_fuse<F32C, NC, T>);
    return reinterpret_cast<const void *>(&k_stream_fuse<F64, NC, T>);
}

const void *comp_fn(uint32_t rmode)
{
    if (rmode == 1) return reinterpret_cast<const void *>(&k_stream_comp<F32>);
    if (rmode == 2) return reinterpret_cast<const void *>(&k_stream_comp<F32C>);
    return reinterpret_cast<const void *>(&k_stream_comp<F64>);
}

template <int NC>
const void *permute_fn(uint32_t rmode)
{
    if (rmode == 1) return reinterpret_cast<const void *>(&k_stream_permute<F32, NC>);
    if (rmode == 2) return reinterpret_cast<const void *>(&k_stream_permute<F32C, NC>);
    return reinterpret_cast<const void *>(&k_stream_permute<F64, NC>);
}

template <int NC>
const void *finish_fn(uint32_t rmode)
{
    if (rmode == 1) return reinterpret_cast<const void *>(&k_stream_finish<F32, NC>);
    if (rmode == 2) return reinterpret_cast<const void *>(&k_stream_finish<F32C, NC>);
    return reinterpret_cast<const void *>(&k_stream_finish<F64, NC>);
}

template <class Nd, int NC, int T, bool MF>
const void *pass_fn(bool perm)
{
    return perm ? reinterpret_cast<const void *>(&k_stream_pass<Nd, NC, T, true, MF>)
                : reinterpret_cast<const void *>(&k_stream_pass<Nd, NC, T, false, MF>);
}

template <int NC, int T, bool MF = false>
const void *pass_fn_mode(uint32_t rmode, bool perm)
{
    if (rmode == 1) return pass_fn<F32, NC, T, MF>(perm);
    if (rmode == 2) return pass_fn<F32C, NC, T, MF>(perm);
    return pass_fn<F64, NC, T, MF>(perm);
}

// Tuples per thread: 4 for n = 4 (16-byte accesses), 1 for n = 16 (16
// values per thread either way, which keeps 8 waves per SIMD), doubled
// until a pass needs at most 4096 blocks (the finish block reduces at most
// 4 partials per thread).
int stream_T(int n, uint32_t N)
{
    uint32_t T = n == 16 ? 1u : 16u / (uint32_t)n;
    while ((uint64_t)N / ((uint64_t)kThreads * T) > 4096) T *= 2;
    return (int)T;
}

const void *pass_kernel(int n, uint32_t N, uint32_t rmode, bool perm, bool mf)
{
    const int T = stream_T(n, N);
    if (mf) return (n == 16 && T == 1) ? pass_fn_mode<16, 1, true>(rmode, perm) : nullptr;
    if (n == 2) {
        if (T == 8) return pass_fn_mode<2, 8>(rmode, perm);
        if (T == 16) return pass_fn_mode<2, 16>(rmode, perm);
    } else if (n == 4) {
        if (T == 4) return pass_fn_mode<4, 4>(rmode, perm);
        if (T == 8) return pass_fn_mode<4, 8>(rmode, perm);
        if (T == 16) return pass_fn_mode<4, 16>(rmode, perm);
    } else if (n == 16) {
        if (T == 1) return pass_fn_mode<16, 1>(rmode, perm);
        if (T == 2) return pass_fn_mode<16, 2>(rmode, perm);
        if (T == 4) return pass_fn_mode<16, 4>(rmode, perm);
    }
    return nullptr;
}

// Larger prime of component k's pair (bounds the LDS run a * R).
uint32_t stride_hi(int k)
{
    constexpr uint32_t hi[16] = {5, 11, 17, 23, 31, 41, 47, 59,
                                 67, 73, 83, 97, 103, 109, 127, 137};
    return hi[k];
}

uint32_t stride_lo(int k)
{
    constexpr uint32_t lo[16] = {3, 7, 13, 19, 29, 37, 43, 53,
                                 61, 71, 79, 89, 101, 107, 113, 131};
    return lo[k];
}

// Launch shape of the permute kernel: R_k the largest power of two with
// hi_k R_k <= run_floats(n); enough blocks for the smaller stride of the pair.
Perm perm_shape(int n, uint32_t N)
{
    Perm p{};
    p.N = N;
    uint32_t blocks = 0;
    for (int k = 0; k < n; ++k) {
        uint32_t logR = 2;
        while ((stride_hi(k) << (logR + 1)) <= run_floats(n)) ++logR;
        p.logR[k] = logR;
        p.first[k] = blocks;
        const uint64_t run = (uint64_t)stride_lo(k) << logR;
        blocks += (uint32_t)((N + run - 1) / run);
    }
    p.first[n] = blocks;
    return p;
}

size_t perm_lds_bytes(const Perm &p, int n)
{
    size_t m = 0;
    for (int k = 0; k < n; ++k) m = std::max<size_t>(m, (size_t)stride_hi(k) << p.logR[k]);
    return m * sizeof(float);
}

}  // namespace

bool stream_shape_ok(int n, uint32_t N, int transform_mode)
{
    if (N < (uint32_t)kThreads * 4) return false;
    const int T = stream_T(n, N);
    if (transform_mode == 1) return n == 16 && T == 1;
    return (n == 2 && T <= 16) || (n == 4 && T <= 16) || (n == 16 && T <= 4);
}

size_t stream_partials_bytes(int n, uint32_t N)
{
    if (!stream_shape_ok(n, N, 0)) return 0;
    const uint32_t nb = N / (kThreads * (uint32_t)stream_T(n, N));
    // partials, component nodes, two last-value slots of the fused pass
    return ((size_t)n * nb + (size_t)n + 1) * sizeof(double2);
}

const float *stream_current_pool(wallace_gen *g)
{
    const size_t off = (g->passes_host & 1) ? g->lay.pool2 : g->lay.pool;
    return reinterpret_cast<const float *>(g->ws + off);
}

hipError_t stream_check(wallace_gen *g, hipStream_t s, const Scratch &sc)
{
    return launch_sumsq(stream_current_pool(g), g->nu, (uint32_t)g->opts.reduce_mode, sc.tree,
                        g->state, 1, s);
}

namespace {

// Passes of a call with the fused kernel (prime-pair strides, n = 2 or 4,
// butterflies). A chain starts with a plain permute of the workspace pool
// (at the call's start and after a refill); each fused launch then combines
// its pass and permutes for the next, and a one-block-per-component launch
// prepares the next pass's old sum of squares. The permuted components of a
// pass whose pool is returned whole, unscaled and 16-byte aligned are built
// in place of that output, which the pass then overwrites tuple by tuple;
// otherwise they alternate between the two workspace buffers. A chain's
// last pass writes the workspace pool (the call's last pass) and the finish
// launch advances the state.
hipError_t stream_run_fused(wallace_gen *g, float *out, uint32_t passes, uint32_t last_emit,
                            uint32_t affine, float mu, float sig, hipStream_t s,
                            const Scratch &sc)
{
    const int n = g->n;
    const uint32_t N = g->N;
    const uint32_t rm = (uint32_t)g->opts.reduce_mode;
    const void *ffn = n == 2 ? fuse_fn<2>(rm) : fuse_fn<4>(rm);
    const void *cfn = comp_fn(rm);
    const void *fin = n == 2 ? finish_fn<2>(rm) : finish_fn<4>(rm);
    const void *pfn = n == 2 ? permute_fn<2>(rm) : permute_fn<4>(rm);
    const uint32_t T = 16u / (uint32_t)n;
    const uint32_t S = (uint32_t)kFuseThreads * T;
    if (N % S) return hipErrorInvalidValue;
    const uint32_t nb = N / S;
    const size_t lds = (size_t)n * S * sizeof(float);
    {
        // 64 KiB of dynamic LDS plus the kernel's static arrays: allowed once
        // per device and kernel (not repeated, so that fills can be captured).
        // A fixed table of the six fused kernels per device, so that a fill
        // allocates no memory.
        constexpr int kMaxDevices = 64, kFusedKernels = 6;
        static std::mutex mu;
        static const void *allowed[kMaxDevices][kFusedKernels];
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
        std::lock_guard<std::mutex> lk(mu);
        int slot = -1;
        for (int i = 0; i < kFusedKernels && slot < 0; ++i)
            if (allowed[dev][i] == ffn || allowed[dev][i] == nullptr) slot = i;
        if (slot < 0) return hipErrorInvalidValue;
        if (allowed[dev][slot] != ffn) {
            e = hipFuncSetAttribute(ffn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            allowed[dev][slot] = ffn;
        }
    }
    Perm pm = perm_shape(n, N);
    const size_t pm_lds = perm_lds_bytes(pm, n);
    pm.state = g->state;
    double2 *partials = reinterpret_cast<double2 *>(sc.partials);
    const uint32_t nb_layout = N / (kThreads * (uint32_t)stream_T(n, N));
    double2 *comp = partials + (size_t)n * nb_layout;
    float *slot = reinterpret_cast<float *>(comp + n);  // [2], by pass parity
    float *pa = reinterpret_cast<float *>(g->ws + g->lay.pool);
    float *pb = reinterpret_cast<float *>(g->ws + g->lay.pool2);
    auto other = [&](const float *p) { return p == pa ? pb : pa; };
    const uint64_t nu = g->nu;
    const uint32_t f = (uint32_t)g->opts.f;
    const uint64_t R = (uint64_t)g->opts.restart_passes;
    // output of pass ps of this call, and whether it can hold its G
    auto emit_of = [&](uint32_t ps, float **o, uint32_t *cnt) {
        *o = nullptr;
        *cnt = 0;
        if ((ps + 1) % f != 0) return false;
        const uint32_t e = (ps + 1) / f - 1;
        *o = out + (uint64_t)e * g->emit_len;
        *cnt = (ps + 1 == passes) ? last_emit : (uint32_t)g->emit_len;
        return *cnt == nu && !affine && ((uintptr_t)*o & 15) == 0;
    };
    const float *cur = ((g->passes_host & 1) != 0) ? pb : pa;
    float *gcur = nullptr;
    const double2 *comp_in = nullptr;
    bool chain = false;
    for (uint32_t ps = 0; ps < passes; ++ps) {
        const uint64_t q = g->passes_host + ps;  // passes since init
        if (R && q > 0 && q % R == 0) {  // restart (section 5)
            float *w = (q & 1) != 0 ? pb : pa;
            hipError_t e = refill_pool(g, w, q, s, sc);
            if (e != hipSuccess) return e;
            cur = w;
            chain = false;
        }
        float *o = nullptr;
        uint32_t cnt = 0;
        const bool fast = emit_of(ps, &o, &cnt);
        if (!chain) {
            // this pass's permuted components from the workspace pool
            gcur = fast ? o : other(cur);
            pm.X = cur;
            pm.G = gcur;
            pm.rng = pass_rng(g, q);
            pm.fin = 0;
            pm.xs = slot + (q & 1);
            void *pargs[] = {&pm};
            hipError_t e = hipLaunchKernel(pfn, dim3(pm.first[n]), dim3(kThreads), pargs, pm_lds, s);
            if (e != hipSuccess) return e;
            comp_in = nullptr;  // the old sum of squares is the state's
        }
        const bool last = ps + 1 == passes;
        const bool cont = !last && !(R && (q + 1) % R == 0);
        float *gnext = nullptr;
        if (cont) {
            float *o2 = nullptr;
            uint32_t cnt2 = 0;
            gnext = emit_of(ps + 1, &o2, &cnt2) ? o2 : other(gcur);
        }
        Fuse F{};
        F.G = gcur;
        F.Y = last ? (((q + 1) & 1) != 0 ? pb : pa) : nullptr;
        F.out = o;
        F.Gn = gnext;
        F.emit_cnt = cnt;
        F.affine = affine;
        F.mu = mu;
        F.sig = sig;
        F.state = g->state;
        F.partials = partials;
        F.comp = comp_in;
        F.xs_in = slot + (q & 1);
        F.xs_out = cont ? slot + ((q + 1) & 1) : nullptr;
        F.r_nu = g->r_nu;
        F.rng = pass_rng(g, q);
        F.rng_next = pass_rng(g, q + 1);
        F.mat = (uint32_t)(q & 1u);
        F.N = N;
        F.nblocks = nb;
        void *fargs[] = {&F};
        hipError_t e = hipLaunchKernel(ffn, dim3(nb), dim3(kFuseThreads), fargs, lds, s);
        if (e != hipSuccess) return e;
        if (cont) {
            const double2 *cpart = partials;
            uint32_t cnb = nb;
            double2 *cdst = comp;
            void *cargs[] = {&cpart, &cnb, &cdst};
            e = hipLaunchKernel(cfn, dim3((uint32_t)n), dim3(kThreads), cargs, 0, s);
            if (e != hipSuccess) return e;
            comp_in = comp;
            gcur = gnext;
            chain = true;
        } else {
            Pass P{};
            P.state = g->state;
            P.partials = partials;
            P.nblocks = nb;
            P.passes = q + 1;
            P.rng = pass_rng(g, q);
            void *args[] = {&P};
            e = hipLaunchKernel(fin, dim3(1), dim3(kThreads), args, 0, s);
            if (e != hipSuccess) return e;
            chain = false;
        }
    }
    return hipSuccess;
}

}  // namespace

hipError_t stream_run(wallace_gen *g, float *out, uint32_t passes, uint32_t last_emit,
                      uint32_t affine, float mu, float sig, hipStream_t s, const Scratch &sc)
{
    if (g->opts.a_mode == 0 && g->N >= kRunFloatsMax && (g->n == 2 || g->n == 4) &&
        g->opts.transform_mode == 0)
        return stream_run_fused(g, out, passes, last_emit, affine, mu, sig, s, sc);
    // prime-pair strides keep a * R small enough for the LDS runs
    const bool perm = g->opts.a_mode == 0 && g->N >= kRunFloatsMax;
    const void *fn = pass_kernel(g->n, g->N, (uint32_t)g->opts.reduce_mode, perm,
                                 g->opts.transform_mode == 1);
    if (!fn) return hipErrorInvalidValue;
    const void *ffn = g->n == 2   ? finish_fn<2>((uint32_t)g->opts.reduce_mode)
                      : g->n == 4 ? finish_fn<4>((uint32_t)g->opts.reduce_mode)
                                : finish_fn<16>((uint32_t)g->opts.reduce_mode);
    Perm pm{};
    size_t pm_lds = 0;
    const void *pfn = nullptr;
    if (perm) {
        pm = perm_shape(g->n, g->N);
        pm_lds = perm_lds_bytes(pm, g->n);
        pfn = g->n == 2   ? permute_fn<2>((uint32_t)g->opts.reduce_mode)
              : g->n == 4 ? permute_fn<4>((uint32_t)g->opts.reduce_mode)
                        : permute_fn<16>((uint32_t)g->opts.reduce_mode);
        pm.state = g->state;
        pm.partials = reinterpret_cast<const double2 *>(sc.partials);
    }
    const int T = stream_T(g->n, g->N);
    const uint32_t nblocks = g->N / (kThreads * (uint32_t)T);
    float *pa = reinterpret_cast<float *>(g->ws + g->lay.pool);
    float *pb = reinterpret_cast<float *>(g->ws + g->lay.pool2);
    const uint32_t f = (uint32_t)g->opts.f;
    // A returned pool that is emitted whole, unscaled and 16-byte aligned is
    // the next pass's old pool: the pass then writes only the caller's
    // output (one 4 nu-byte stream less). The call's last pass always writes
    // the workspace pool that the next call starts from.
    const float *src = ((g->passes_host & 1) != 0) ? pb : pa;
    const uint64_t R = (uint64_t)g->opts.restart_passes;
    for (uint32_t ps = 0; ps < passes; ++ps) {
        float *ws_dst = ((g->passes_host + ps + 1) & 1) != 0 ? pb : pa;
        // restart (section 5): refill into the workspace buffer of this
        // pass's parity; the pass then starts from the state's new sum
        bool refilled = false;
        {
            const uint64_t q = g->passes_host + ps;
            if (R && q > 0 && q % R == 0) {
                float *w = (q & 1) != 0 ? pb : pa;
                hipError_t e = refill_pool(g, w, q, s, sc);
                if (e != hipSuccess) return e;
                src = w;
                refilled = true;
            }
        }
        Pass P{};
        P.X = src;
        P.Y = ws_dst;
        P.out = nullptr;
        P.emit_cnt = 0;
        if ((ps + 1) % f == 0) {
            const uint32_t e = (ps + 1) / f - 1;
            P.out = out + (uint64_t)e * g->emit_len;
            P.emit_cnt = (ps + 1 == passes) ? last_emit : (uint32_t)g->emit_len;
        }
        if (P.out && ps + 1 < passes && P.emit_cnt == g->nu && !affine &&
            ((uintptr_t)P.out & 15) == 0) {
            P.Y = P.out;
            P.out = nullptr;
        }
        P.G = P.Y;  // permuted in place of the new pool
        src = P.Y;
        P.affine = affine;
        P.mu = mu;
        P.sig = sig;
        P.state = g->state;
        P.partials = reinterpret_cast<double2 *>(sc.partials);
        P.r_nu = g->r_nu;
        P.N = g->N;
        P.a_mode = (uint32_t)g->opts.a_mode;
        P.nblocks = nblocks;
        const uint64_t q = g->passes_host + ps;  // passes since init
        P.rng = pass_rng(g, q);
        P.mat = (uint32_t)(q & 1u);
        P.passes = q + 1;
        double2 *comp = reinterpret_cast<double2 *>(sc.partials) +
                        (size_t)g->n * nblocks;
        P.comp = nullptr;
        if (perm) {
            pm.X = P.X;
            pm.G = P.Y;
            pm.rng = P.rng;
            pm.fin = (ps > 0 && !refilled) ? 1u : 0u;  // this call's previous pass
            pm.fin_nblocks = nblocks;
            pm.comp = comp;
            if (pm.fin) P.comp = comp;
            void *pargs[] = {&pm};
            hipError_t e = hipLaunchKernel(pfn, dim3(pm.first[g->n] + pm.fin * (uint32_t)g->n),
                                           dim3(kThreads), pargs, pm_lds, s);
            if (e != hipSuccess) return e;
        }
        void *args[] = {&P};
        hipError_t e = hipLaunchKernel(fn, dim3(nblocks), dim3(kThreads), args, 0, s);
        if (e == hipSuccess && (!perm || ps + 1 == passes))
            e = hipLaunchKernel(ffn, dim3(1), dim3(kThreads), args, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace wallace
