// HIP kernels (gfx950) of the Wallace generator library.
//
// One pass (Brent 1997, section 2, eq. 1) regenerates a pool of nu = n*N
// normals held as n component arrays of N values:
//   draw per-component odd strides a_k and offsets b_k (eq. 2, sections 3, 8),
//   gather v_k[j] = X_k[(a_k j + b_k) mod N],
//   y[j] = c * A v[j] with A orthogonal (section 3) and c the chi-squared
//   scale computed from the old pool's sum of squares (section 4, eq. 3),
//   write y back as the new pool (double buffering, section 2),
//   emit it in flat order f = k*N + j (section 3),
//   sum its squares for the next pass's scale (section 4).
//
// Arithmetic order is fixed so that results are bit-exact: FP32 butterflies
// in the order s = (v0 +- v1, v2 +- v3), u = (s0 +- s2, s1 +- s3) (n = 4) or
// the radix-2 Walsh-Hadamard stages 1, 2, 4, 8 (n = 16), no contraction
// (-ffp-contract=off), and the sum of squares as a perfect binary tree over
// the flat index with every node rounded once.
#include "wallace_internal.h"

#include "wallace.h"

namespace wallace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

// splitmix64 (Steele, Lea and Flood 2014): Weyl step then two xor-shift-
// multiply rounds and a final xor-shift.
__device__ __forceinline__ uint64_t sm64_next(uint64_t &s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Stride pair of component k: RANN4's alpha in {3,5} and beta in {7,11}
// (section 8) continued with the following pairs of odd primes, so that the
// strides of different components are distinct and greater than one
// (sections 3 and 7).
__device__ __forceinline__ uint32_t stride_pick(int k, uint32_t top)
{
    constexpr uint32_t lo[16] = {3, 7, 13, 19, 29, 37, 43, 53,
                                 61, 71, 79, 89, 101, 107, 113, 131};
    constexpr uint32_t hi[16] = {5, 11, 17, 23, 31, 41, 47, 59,
                                 67, 73, 83, 97, 103, 109, 127, 137};
    return top ? hi[k] : lo[k];
}

// Chi-squared scale (section 4, eq. 3): S = (x* + sqrt(2 nu - 1))^2 / 2 is a
// chi2_nu sample; the new pool gets sum of squares S via c = sqrt(S / sigma).
// Every step is one IEEE operation; FP64 divide and square root are
// correctly rounded on gfx950.
__device__ __forceinline__ float chi2_scale(double xstar, double sigma,
                                            double r_nu)
{
    double t = xstar + r_nu;
    double S = (t * t) * 0.5;
    double q = S / sigma;
    double c64 = __builtin_sqrt(q);
    return (float)c64;
}

// Ordering of LDS traffic between the lanes of a pool group. A group inside
// one wavefront relies on in-order LDS execution of a wave and only needs a
// compiler barrier; a multi-wave group uses s_barrier. Neither waits for
// outstanding global stores.
__device__ __forceinline__ void group_sync(bool multiwave)
{
    if (multiwave) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// ---------------------------------------------------------------------------
// Sum-of-squares tree nodes for the three reduction modes
// ---------------------------------------------------------------------------

struct NodeF64 {  // FP64 nodes; leaves (double)y*(double)y are exact
    double v;
    __device__ static NodeF64 leaf(float y) { return {(double)y * (double)y}; }
    __device__ static NodeF64 zero() { return {0.0}; }
    __device__ static NodeF64 join(NodeF64 a, NodeF64 b) { return {a.v + b.v}; }
    __device__ static NodeF64 shfl_xor(NodeF64 a, int m, int w)
    {
        return {__shfl_xor(a.v, m, w)};
    }
    __device__ static NodeF64 shfl(NodeF64 a, int src, int w)
    {
        return {__shfl(a.v, src, w)};
    }
    __device__ static NodeF64 sel(bool c, NodeF64 a, NodeF64 b) { return c ? a : b; }
    __device__ double value() const { return v; }
    __device__ double2 pack() const { return make_double2(v, 0.0); }
    __device__ static NodeF64 unpack(double2 d) { return {d.x}; }
};

struct NodeF32 {  // FP32 nodes (the "naive" FP32 reduction)
    float v;
    __device__ static NodeF32 leaf(float y) { return {y * y}; }
    __device__ static NodeF32 zero() { return {0.0f}; }
    __device__ static NodeF32 join(NodeF32 a, NodeF32 b) { return {a.v + b.v}; }
    __device__ static NodeF32 shfl_xor(NodeF32 a, int m, int w)
    {
        return {__shfl_xor(a.v, m, w)};
    }
    __device__ static NodeF32 shfl(NodeF32 a, int src, int w)
    {
        return {__shfl(a.v, src, w)};
    }
    __device__ static NodeF32 sel(bool c, NodeF32 a, NodeF32 b) { return c ? a : b; }
    __device__ double value() const { return (double)v; }
    __device__ double2 pack() const { return make_double2((double)v, 0.0); }
    __device__ static NodeF32 unpack(double2 d) { return {(float)d.x}; }
};

struct NodeComp {  // FP32 value plus FP32 error term (TwoProd / TwoSum)
    float s, e;
    __device__ static NodeComp leaf(float y)
    {
        float p = y * y;
        return {p, __builtin_fmaf(y, y, -p)};
    }
    __device__ static NodeComp zero() { return {0.0f, 0.0f}; }
    __device__ static NodeComp join(NodeComp a, NodeComp b)
    {
        float sum = a.s + b.s;
        float bb = sum - a.s;
        float err = (a.s - (sum - bb)) + (b.s - bb);
        return {sum, (a.e + b.e) + err};
    }
    __device__ static NodeComp shfl_xor(NodeComp a, int m, int w)
    {
        return {__shfl_xor(a.s, m, w), __shfl_xor(a.e, m, w)};
    }
    __device__ static NodeComp shfl(NodeComp a, int src, int w)
    {
        return {__shfl(a.s, src, w), __shfl(a.e, src, w)};
    }
    __device__ static NodeComp sel(bool c, NodeComp a, NodeComp b) { return c ? a : b; }
    __device__ double value() const { return (double)s + (double)e; }
    __device__ double2 pack() const { return make_double2((double)s, (double)e); }
    __device__ static NodeComp unpack(double2 d) { return {(float)d.x, (float)d.y}; }
};

template <int V>
struct Log2 {
    static constexpr int value = 1 + Log2<V / 2>::value;
};
template <>
struct Log2<1> {
    static constexpr int value = 0;
};

// Canonical tree over the T consecutive values a lane holds for one
// component: pairs (2i, 2i+1), then pairs of pairs.
template <class Nd, int T>
__device__ __forceinline__ Nd lane_tree(const float (&x)[T])
{
    Nd t[T];
#pragma unroll
    for (int i = 0; i < T; ++i) t[i] = Nd::leaf(x[i]);
#pragma unroll
    for (int w = T; w > 1; w >>= 1) {
#pragma unroll
        for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
    }
    return t[0];
}

// Sum of squares of a pool spread over a group of L lanes (lane `lane` holds
// tuples [T*lane, T*lane + T) of every component). Tree levels, bottom up:
// the T values inside a lane; the lanes (a value for every component per
// lane: the first log2(n) lane levels halve the values each lane carries,
// the rest are butterflies); the waves of a multi-wave group (through LDS);
// finally the n components. Every level pairs the same nodes as the
// canonical tree over the flat index, so the result does not depend on L, T
// or the wave count.
template <class Nd, int NC, int T, bool MW>
__device__ double pool_sumsq(const float (&X)[NC][T], int lane, int L,
                             int logL, double2 *red)
{
    constexpr int LOG_NC = Log2<NC>::value;
    constexpr bool multiwave = MW;
    const int width = multiwave ? 64 : L;
    const int logw = multiwave ? 6 : logL;
    const int wl = lane & (width - 1);
    Nd v[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) v[k] = lane_tree<Nd, T>(X[k]);
    // halving levels: lane bit m decides which half of the remaining
    // components this lane keeps; both partners pair the same component.
#pragma unroll
    for (int m = 0; m < LOG_NC; ++m) {
        const int V = NC >> m;
        const bool hi = (wl >> m) & 1;
#pragma unroll
        for (int t = 0; t < V / 2; ++t) {
            Nd keep = Nd::sel(hi, v[t + V / 2], v[t]);
            Nd send = Nd::sel(hi, v[t], v[t + V / 2]);
            v[t] = Nd::join(keep, Nd::shfl_xor(send, 1 << m, width));
        }
    }
    Nd acc = v[0];  // component kappa(lane) = bit-reverse of the low bits
    for (int m = LOG_NC; m < logw; ++m)
        acc = Nd::join(acc, Nd::shfl_xor(acc, 1 << m, width));
    if constexpr (multiwave) {
        const int wave = lane >> 6;
        const int W = L >> 6;
        int kappa = 0;
#pragma unroll
        for (int m = 0; m < LOG_NC; ++m) kappa |= ((wl >> m) & 1) << (LOG_NC - 1 - m);
        if (wl < NC) red[wave * NC + kappa] = acc.pack();
        group_sync(true);
        Nd t[16];
        const int kk = kappa;
#pragma unroll
        for (int w = 0; w < 16; ++w)
            t[w] = (w < W) ? Nd::unpack(red[w * NC + kk]) : Nd::zero();
#pragma unroll
        for (int s = 1; s < 16; s <<= 1) {
            if (s < W) {
#pragma unroll
                for (int w = 0; w < 16; w += 2 * s) t[w] = Nd::join(t[w], t[w + s]);
            }
        }
        acc = t[0];
    }
    // component levels: kappa and kappa ^ 2^q differ in lane bit LOG_NC-1-q
#pragma unroll
    for (int m = LOG_NC - 1; m >= 0; --m)
        acc = Nd::join(acc, Nd::shfl_xor(acc, 1 << m, width));
    if constexpr (multiwave) acc = Nd::shfl(acc, 0, 64);
    return acc.value();
}

template <int RM>
struct NodeOf {
    using type = NodeF64;
};
template <>
struct NodeOf<1> {
    using type = NodeF32;
};
template <>
struct NodeOf<2> {
    using type = NodeComp;
};

// ---------------------------------------------------------------------------
// The orthogonal transforms (section 3), unscaled butterflies then * h
// ---------------------------------------------------------------------------

// n = 4: A0 = H4/2 (mat 0) and A1 = J/2 - I (mat 1). A1 = D_r P (H4/2) D_c
// with D_c = diag(-1,1,1,1), P swapping rows 1 and 2, D_r = diag(1,-1,-1,-1).
__device__ __forceinline__ void xform4(float (&v)[4], int mat, float h)
{
    float v0 = mat ? -v[0] : v[0];
    float s0 = v0 + v[1], s1 = v0 - v[1];
    float s2 = v[2] + v[3], s3 = v[2] - v[3];
    float u0 = s0 + s2, u1 = s1 + s3, u2 = s0 - s2, u3 = s1 - s3;
    if (mat) {
        v[0] = u0 * h;
        v[1] = (-u2) * h;
        v[2] = (-u1) * h;
        v[3] = (-u3) * h;
    } else {
        v[0] = u0 * h;
        v[1] = u1 * h;
        v[2] = u2 * h;
        v[3] = u3 * h;
    }
}

// n = 16: H16 D / 4 with D = diag((-1)^(bit k of signs)), radix-2 stages.
__device__ __forceinline__ void xform16(float (&v)[16], uint32_t signs, float h)
{
#pragma unroll
    for (int k = 0; k < 16; ++k)
        v[k] = ((signs >> k) & 1u) ? -v[k] : v[k];
#pragma unroll
    for (int s = 1; s < 16; s <<= 1) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i & s) continue;
            float lo = v[i], hi = v[i + s];
            v[i] = lo + hi;
            v[i + s] = lo - hi;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = v[k] * h;
}

// ---------------------------------------------------------------------------
// Vector loads and stores of a lane's T consecutive values
// ---------------------------------------------------------------------------

template <int T>
__device__ __forceinline__ void load_run(float (&x)[T], const float *p)
{
    if constexpr (T % 4 == 0) {
#pragma unroll
        for (int i = 0; i < T; i += 4) {
            float4 q = *reinterpret_cast<const float4 *>(p + i);
            x[i] = q.x; x[i + 1] = q.y; x[i + 2] = q.z; x[i + 3] = q.w;
        }
    } else if constexpr (T == 2) {
        float2 q = *reinterpret_cast<const float2 *>(p);
        x[0] = q.x; x[1] = q.y;
    } else {
        x[0] = p[0];
    }
}

template <int T>
__device__ __forceinline__ void store_run(float *p, const float (&x)[T], bool nt)
{
    if constexpr (T % 4 == 0) {
#pragma unroll
        for (int i = 0; i < T; i += 4) {
            const v4f q = {x[i], x[i + 1], x[i + 2], x[i + 3]};
            if (nt)
                __builtin_nontemporal_store(q, reinterpret_cast<v4f *>(p + i));
            else
                *reinterpret_cast<v4f *>(p + i) = q;
        }
    } else if constexpr (T == 2) {
        const v2f q = {x[0], x[1]};
        if (nt)
            __builtin_nontemporal_store(q, reinterpret_cast<v2f *>(p));
        else
            *reinterpret_cast<v2f *>(p) = q;
    } else {
        if (nt)
            __builtin_nontemporal_store(x[0], p);
        else
            p[0] = x[0];
    }
}

// Element-wise emission for partial pools, unaligned outputs or the
// N(mu, sigma^2) map (one multiply then one add).
template <int NC, int T>
__device__ __forceinline__ void emit_slow(const float (&X)[NC][T], float *base,
                                                    uint32_t cnt, int N, int lane,
                                                    uint32_t affine, float mu, float sig)
{
#pragma unroll
    for (int k = 0; k < NC; ++k) {
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const uint32_t fl = (uint32_t)k * N + (uint32_t)(T * lane + i);
            if (fl < cnt) {
                float y = X[k][i];
                if (affine) y = mu + sig * y;
                __builtin_nontemporal_store(y, base + fl);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pool-resident pass loop
// ---------------------------------------------------------------------------
//
// A group of L lanes owns one pool for the whole job; lane l holds tuples
// j = T*l .. T*l + T - 1 of every component in registers across passes. The
// per-pass permutation goes through LDS, C components at a time. In LDS a
// component's element x sits at (x mod T) * L + (x div T): the writes of
// consecutive lanes and the gathers with odd stride a (addresses a*T*l + c
// across lanes) then fall in distinct banks.

template <int NC, int T, bool MW, int RM, int NST>
__device__ void run_job(const PoolArgs &P, const Job &job, float *lds,
                        double2 *red, int lane)
{
    using Nd = typename NodeOf<RM>::type;
    constexpr int C = NC / NST;  // components per on-chip stage
    constexpr int LOG_T = Log2<T>::value;
    const int L = P.L;
    const int logL = P.logL;
    const int N = P.N;
    const uint32_t mask = (uint32_t)N - 1u;
    const uint32_t nu = (uint32_t)(NC * N);

    float X[NC][T];
    const float *pool = P.pools + job.pool_off;
#pragma unroll
    for (int k = 0; k < NC; ++k) load_run<T>(X[k], pool + (size_t)k * N + (size_t)T * lane);

    GenState *stp = P.states + job.gen;
    uint64_t rng = stp->rng;
    double sigma = stp->sigma;
    const uint64_t done = stp->passes;
    uint32_t flags = stp->flags;

    if (P.sigma_mode) {
        group_sync(MW);  // the previous job's last reduction has been read
        double s = pool_sumsq<Nd, NC, T, MW>(X, lane, L, logL, red);
        if (P.sigma_mode == 2)
            sigma = s;
        else if (!(s == sigma))
            flags |= WALLACE_FLAG_CORRUPT;
    }
    const bool skip = (flags & WALLACE_FLAG_CORRUPT) != 0;
    const uint32_t passes = skip ? 0u : job.passes;

    for (uint32_t ps = 0; ps < passes; ++ps) {
        const int mat = (NC == 4) ? (int)((done + ps) & 1u) : 0;
        uint32_t signs = 0;
        double xstar = 0.0;
#pragma unroll
        for (int st = 0; st < NST; ++st) {
            // per-pass parameters of this stage's components: one draw per
            // component, in component order (eq. 1, section 8)
            uint32_t a[C], b[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int k = st * C + c;
                const uint64_t w = sm64_next(rng);
                const uint32_t ak = P.a_mode ? ((uint32_t)(w >> 32) | 1u)
                                             : stride_pick(k, (uint32_t)(w >> 63));
                a[c] = ak & mask;
                b[c] = (uint32_t)w & mask;
                if (NC == 16) signs |= (uint32_t)((w >> 62) & 1u) << k;
            }
            group_sync(MW);  // previous gathers done before overwrite
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float *dst = lds + (size_t)c * N + lane;
#pragma unroll
                for (int i = 0; i < T; ++i) dst[i * L] = X[st * C + c][i];
            }
            group_sync(MW);
            if (st == NST - 1)  // the old pool's last flat value (section 4)
                xstar = (double)lds[(size_t)(C - 1) * N + (N - 1)];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float *src = lds + (size_t)c * N;
                const uint32_t q = a[c] * (uint32_t)lane;
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const uint32_t cc = a[c] * (uint32_t)i + b[c];
                    const uint32_t hiTL = (cc & (uint32_t)(T - 1)) << logL;
                    const uint32_t idx = (q + (cc >> LOG_T)) & (uint32_t)(L - 1);
                    X[st * C + c][i] = src[hiTL | idx];
                }
            }
        }

        // scale folded into the matrix (section 4)
        const float c32 = chi2_scale(xstar, sigma, P.r_nu);
        if (!__builtin_isfinite(c32)) flags |= WALLACE_FLAG_NONFINITE;
        const float h = c32 * (NC == 4 ? 0.5f : 0.25f);
#pragma unroll
        for (int i = 0; i < T; ++i) {
            float v[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) v[k] = X[k][i];
            if constexpr (NC == 4)
                xform4(v, mat, h);
            else
                xform16(v, signs, h);
#pragma unroll
            for (int k = 0; k < NC; ++k) X[k][i] = v[k];
        }

        // emit the new pool when it is a returned one (section 6)
        if ((ps + 1) % P.f == 0) {
            const uint32_t e = (ps + 1) / P.f - 1;
            const bool last = (ps + 1 == passes);
            const uint32_t cnt = last ? job.last_emit : P.emit_len;
            float *base = P.out + job.out_off + (uint64_t)e * P.emit_len;
            const bool aligned =
                (((uintptr_t)base) & (uintptr_t)(4 * (T >= 4 ? 4 : T) - 1)) == 0;
            if (cnt == nu && aligned && !P.affine) {
#pragma unroll
                for (int k = 0; k < NC; ++k)
                    store_run<T>(base + (size_t)k * N + (size_t)T * lane, X[k], true);
            } else {
                emit_slow<NC, T>(X, base, cnt, N, lane, P.affine, P.mu, P.sigma_out);
            }
        }

        // sum of squares of the new pool (section 4)
        sigma = pool_sumsq<Nd, NC, T, MW>(X, lane, L, logL, red);
    }

    float *wpool = P.pools + job.pool_off;
#pragma unroll
    for (int k = 0; k < NC; ++k)
        store_run<T>(wpool + (size_t)k * N + (size_t)T * lane, X[k], false);
    if (lane == 0) {
        stp->rng = rng;
        stp->sigma = sigma;
        stp->passes = done + passes;
        stp->flags = flags;
    }
}

template <int NC, int T, bool MW, int RM, int NST>
__global__ __launch_bounds__(MW ? 1024 : 256) void k_pool(PoolArgs P)
{
    extern __shared__ float lds_all[];
    const int L = P.L;
    const int gpb = P.groups_per_block;
    const int grp = (int)threadIdx.x / L;
    const int lane = (int)threadIdx.x % L;
    const size_t grp_floats = (size_t)P.C * P.N;
    float *lds = lds_all + grp_floats * grp;
    double2 *red = reinterpret_cast<double2 *>(lds_all + grp_floats * gpb);

    const uint32_t total = gridDim.x * (uint32_t)gpb;
    for (uint32_t j = blockIdx.x * (uint32_t)gpb + (uint32_t)grp; j < P.njobs; j += total) {
        const Job job = P.jobs ? P.jobs[j] : P.one;
        run_job<NC, T, MW, RM, NST>(P, job, lds, red, lane);
    }
}

// ---------------------------------------------------------------------------
// Small kernels: emit leftover values of the current pool; canonical
// sum-of-squares tree over a pool in memory (initialisation and checks)
// ---------------------------------------------------------------------------

__global__ void k_copy_head(float *out, const float *pool, uint32_t count,
                            uint32_t affine, float mu, float sig)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += gridDim.x * blockDim.x) {
        float y = pool[i];
        if (affine) y = mu + sig * y;
        out[i] = y;
    }
}

// Copies one generator's state and pool into `copies` slots (tuning runs).
__global__ void k_replicate(GenState *states, float *pools, uint64_t stride,
                            uint32_t copies, const GenState *src_state,
                            const float *src_pool, uint64_t nu)
{
    const uint64_t total = (uint64_t)copies * nu;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t c = i / nu, f = i - c * nu;
        pools[c * stride + f] = src_pool[f];
        if (f == 0) states[c] = *src_state;
    }
}

// One block reduces 1024 consecutive leaves (or nodes) to one node with the
// canonical tree; missing inputs beyond `count` are zero, which leaves every
// node of the real subtree unchanged.
template <class Nd, bool LEAVES>
__device__ void block_tree(const void *in, size_t count, double2 *out)
{
    __shared__ double2 part[4];
    const size_t base = (size_t)blockIdx.x * 1024 + (size_t)threadIdx.x * 4;
    Nd t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const size_t f = base + i;
        if (f < count) {
            if (LEAVES)
                t[i] = Nd::leaf(static_cast<const float *>(in)[f]);
            else
                t[i] = Nd::unpack(static_cast<const double2 *>(in)[f]);
        } else {
            t[i] = Nd::zero();
        }
    }
    Nd acc = Nd::join(Nd::join(t[0], t[1]), Nd::join(t[2], t[3]));
    for (int m = 0; m < 6; ++m) acc = Nd::join(acc, Nd::shfl_xor(acc, 1 << m, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc.pack();
    __syncthreads();
    if (threadIdx.x == 0) {
        Nd r = Nd::join(Nd::join(Nd::unpack(part[0]), Nd::unpack(part[1])),
                        Nd::join(Nd::unpack(part[2]), Nd::unpack(part[3])));
        out[blockIdx.x] = r.pack();
    }
}

template <class Nd, bool LEAVES>
__global__ __launch_bounds__(256) void k_tree(const void *in, size_t count,
                                              double2 *out)
{
    block_tree<Nd, LEAVES>(in, count, out);
}

// mode 0: store the root as the state's sigma; mode 1: compare and flag.
template <class Nd>
__global__ void k_tree_finish(const double2 *root, GenState *state, uint32_t mode)
{
    const double s = Nd::unpack(root[0]).value();
    if (mode == 0)
        state->sigma = s;
    else if (!(s == state->sigma))
        state->flags |= WALLACE_FLAG_CORRUPT;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

int pool_block_threads(const Sched &s) { return s.L > 64 ? s.L : 256; }

size_t pool_lds_bytes(const Sched &s, int N)
{
    const int gpb = s.L > 64 ? 1 : 256 / s.L;
    return (size_t)gpb * s.C * N * sizeof(float) + 16 * 16 * sizeof(double2);
}

bool pool_sched_supported(const Sched &s, int N)
{
    if (s.C < 1 || s.n % s.C) return false;
    if (s.L <= 64 && s.C != s.n) return false;
    if (s.n / s.C > 2) return false;
    if (s.n != 4 && s.n != 16) return false;
    if (s.T * s.L != N) return false;
    if (s.L < s.n || s.L > 1024 || (s.L & (s.L - 1))) return false;
    if (s.C < 1 || s.n % s.C) return false;
    if (s.n == 4 && !(s.T == 1 || s.T == 2 || s.T == 4 || s.T == 8 || s.T == 16)) return false;
    if (s.n == 16 && !(s.T == 1 || s.T == 2 || s.T == 4)) return false;
    return pool_lds_bytes(s, N) <= 160 * 1024;
}

template <int NC, int T, bool MW, int NST>
static const void *pool_kernel_rm(uint32_t rm)
{
    if (rm == 1) return reinterpret_cast<const void *>(&k_pool<NC, T, MW, 1, NST>);
    if (rm == 2) return reinterpret_cast<const void *>(&k_pool<NC, T, MW, 2, NST>);
    return reinterpret_cast<const void *>(&k_pool<NC, T, MW, 0, NST>);
}

// Instantiated shapes: single-wave groups keep all components on chip;
// multi-wave groups (large pools) use one stage, or two when n*N floats
// exceed the LDS budget.
template <int NC, int T>
static const void *pool_kernel_ptr(bool mw, int nst, uint32_t rm)
{
    if (!mw) return nst == 1 ? pool_kernel_rm<NC, T, false, 1>(rm) : nullptr;
    if (nst == 1) return pool_kernel_rm<NC, T, true, 1>(rm);
    if (nst == 2) return pool_kernel_rm<NC, T, true, 2>(rm);
    return nullptr;
}

static const void *pool_kernel(const Sched &s, uint32_t rm)
{
    const bool mw = s.L > 64;
    if (s.C < 1 || s.n % s.C) return nullptr;
    const int nst = s.n / s.C;
    if (s.n == 4) {
        switch (s.T) {
        case 1: return pool_kernel_ptr<4, 1>(mw, nst, rm);
        case 2: return pool_kernel_ptr<4, 2>(mw, nst, rm);
        case 4: return pool_kernel_ptr<4, 4>(mw, nst, rm);
        case 8: return pool_kernel_ptr<4, 8>(mw, nst, rm);
        case 16: return pool_kernel_ptr<4, 16>(mw, nst, rm);
        }
    } else if (s.n == 16) {
        switch (s.T) {
        case 1: return pool_kernel_ptr<16, 1>(mw, nst, rm);
        case 2: return pool_kernel_ptr<16, 2>(mw, nst, rm);
        case 4: return pool_kernel_ptr<16, 4>(mw, nst, rm);
        }
    }
    return nullptr;
}

// Kernels that need more than 64 KiB of LDS declare it once per process.
static hipError_t allow_lds(const void *fn, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t pool_max_blocks_per_cu(const Sched &s, int N, uint32_t rmode, int *blocks)
{
    const void *fn = pool_kernel(s, rmode);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = allow_lds(fn, pool_lds_bytes(s, N));
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, fn, pool_block_threads(s), pool_lds_bytes(s, N));
}

hipError_t launch_pool(const Sched &s, const PoolArgs &a, int grid,
                       hipStream_t stream)
{
    const void *fn = pool_kernel(s, a.rmode);
    if (!fn) return hipErrorInvalidValue;
    if (!pool_sched_supported(s, a.N) || a.L != s.L || a.C != s.C) return hipErrorInvalidValue;
    hipError_t e = allow_lds(fn, pool_lds_bytes(s, a.N));
    if (e != hipSuccess) return e;
    PoolArgs args = a;
    void *kargs[] = {&args};
    return hipLaunchKernel(fn, dim3(grid), dim3(pool_block_threads(s)), kargs,
                           pool_lds_bytes(s, a.N), stream);
}

hipError_t launch_copy_head(float *out, const float *pool, uint32_t count,
                            uint32_t affine, float mu, float sig,
                            hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    int grid = (int)((count + 255) / 256);
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_copy_head, dim3(grid), dim3(256), 0, stream, out, pool,
                       count, affine, mu, sig);
    return hipGetLastError();
}

hipError_t launch_replicate(GenState *states, float *pools, uint64_t stride,
                            uint32_t copies, const GenState *src_state,
                            const float *src_pool, uint64_t nu, hipStream_t stream)
{
    hipLaunchKernelGGL(k_replicate, dim3(2048), dim3(256), 0, stream, states, pools,
                       stride, copies, src_state, src_pool, nu);
    return hipGetLastError();
}

template <class Nd>
static hipError_t sumsq_chain(const float *pool, size_t nu, double2 *scratch,
                              GenState *state, uint32_t mode, hipStream_t stream)
{
    // level 0: leaves -> ceil(nu / 1024) nodes; then nodes -> nodes / 1024
    size_t count = nu;
    size_t blocks = (count + 1023) / 1024;
    double2 *bufA = scratch;
    double2 *bufB = scratch + blocks;
    hipLaunchKernelGGL((k_tree<Nd, true>), dim3((unsigned)blocks), dim3(256), 0,
                       stream, (const void *)pool, count, bufA);
    count = blocks;
    while (count > 1) {
        blocks = (count + 1023) / 1024;
        hipLaunchKernelGGL((k_tree<Nd, false>), dim3((unsigned)blocks), dim3(256), 0,
                           stream, (const void *)bufA, count, bufB);
        double2 *t = bufA;
        bufA = bufB;
        bufB = t;
        count = blocks;
    }
    hipLaunchKernelGGL(k_tree_finish<Nd>, dim3(1), dim3(1), 0, stream,
                       (const double2 *)bufA, state, mode);
    return hipGetLastError();
}

// scratch must hold ceil(nu/1024) + ceil(nu/1024^2) + 2 double2 values.
hipError_t launch_sumsq(const float *pool, size_t nu, uint32_t rmode,
                        double *scratch, double *unused, GenState *state,
                        uint32_t mode, hipStream_t stream)
{
    (void)unused;
    double2 *s = reinterpret_cast<double2 *>(scratch);
    if (rmode == 1) return sumsq_chain<NodeF32>(pool, nu, s, state, mode, stream);
    if (rmode == 2) return sumsq_chain<NodeComp>(pool, nu, s, state, mode, stream);
    return sumsq_chain<NodeF64>(pool, nu, s, state, mode, stream);
}

}  // namespace wallace
