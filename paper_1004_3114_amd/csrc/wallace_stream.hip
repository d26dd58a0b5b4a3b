// Streaming pass for pools too large to stay on chip (tens of MB): the old
// pool is gathered from HBM (it mostly stays in the 256 MB last-level
// cache), the new pool is written to a second buffer and, when it is a
// returned pool, to the caller's output. One launch per pass (section 2,
// eq. 1); the pass's sum of squares (section 4) is reduced by the last
// block to arrive, which also advances the generator state for the next
// launch.
#include "wallace_runtime.h"

namespace wallace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

namespace {

__device__ __forceinline__ uint64_t sm64(uint64_t &s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Component k's stride pair (section 8: {3,5}, {7,11}, then further odd
// primes so that the strides of different components differ).
__device__ __forceinline__ uint32_t stride_of(int k, uint32_t top)
{
    constexpr uint32_t lo[16] = {3, 7, 13, 19, 29, 37, 43, 53,
                                 61, 71, 79, 89, 101, 107, 113, 131};
    constexpr uint32_t hi[16] = {5, 11, 17, 23, 31, 41, 47, 59,
                                 67, 73, 83, 97, 103, 109, 127, 137};
    return top ? hi[k] : lo[k];
}

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

template <int V>
struct Lg {
    static constexpr int value = 1 + Lg<V / 2>::value;
};
template <>
struct Lg<1> {
    static constexpr int value = 0;
};

constexpr int kThreads = 256;

struct Pass {
    const float *X;   // old pool
    float *Y;         // new pool
    float *out;       // returned copy of the new pool (NULL: not returned)
    uint32_t emit_cnt;
    uint32_t affine;
    float mu, sig;
    GenState *state;
    double2 *partials;  // [n][nblocks]
    uint32_t *counter;
    double r_nu;
    uint32_t N;
    uint32_t a_mode;
    uint32_t nblocks;
};

// Per-block partial sums for every component: the block's tuples
// [j0, j0 + 256 T) form an aligned subtree of each component's part of the
// canonical tree over the flat index.
template <class Nd, int NC, int T>
__device__ void block_partials(const float (&X)[NC][T], double2 *dst,
                               uint32_t nblocks, double2 *red)
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
        const int k = threadIdx.x;
        Nd r = Nd::join(Nd::join(Nd::unpack(red[k]), Nd::unpack(red[NC + k])),
                        Nd::join(Nd::unpack(red[2 * NC + k]), Nd::unpack(red[3 * NC + k])));
        dst[(size_t)k * nblocks + blockIdx.x] = r.pack();
        __threadfence();
    }
}

// Canonical tree over the n*nblocks partial nodes (nblocks <= 1024): per
// component over its blocks, then over the components.
template <class Nd, int NC>
__device__ double final_tree(const double2 *partials, uint32_t nblocks, double2 *red)
{
    __shared__ double2 comp[NC];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int k = 0; k < NC; ++k) {
        Nd t[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t b = threadIdx.x * 4 + i;
            t[i] = b < nblocks ? Nd::unpack(partials[(size_t)k * nblocks + b]) : Nd::zero();
        }
        Nd acc = Nd::join(Nd::join(t[0], t[1]), Nd::join(t[2], t[3]));
#pragma unroll
        for (int m = 0; m < 6; ++m) acc = Nd::join(acc, Nd::xr(acc, 1 << m));
        if (lane == 0) red[wave] = acc.pack();
        __syncthreads();
        if (threadIdx.x == 0)
            comp[k] = Nd::join(Nd::join(Nd::unpack(red[0]), Nd::unpack(red[1])),
                               Nd::join(Nd::unpack(red[2]), Nd::unpack(red[3])))
                          .pack();
        __syncthreads();
    }
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

template <class Nd, int NC, int T>
__global__ __launch_bounds__(kThreads) void k_stream_pass(Pass P)
{
    __shared__ double2 red[4 * NC];
    __shared__ uint32_t last;
    const GenState st = *P.state;
    if (st.flags & WALLACE_FLAG_CORRUPT) return;
    const uint32_t N = P.N;
    const uint32_t mask = N - 1u;
    const uint32_t nu = NC * N;

    uint64_t rng = st.rng;
    uint32_t a[NC], b[NC], signs = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const uint64_t w = sm64(rng);
        const uint32_t ak = P.a_mode ? ((uint32_t)(w >> 32) | 1u)
                                     : stride_of(k, (uint32_t)(w >> 63));
        a[k] = ak & mask;
        b[k] = (uint32_t)w & mask;
        if (NC == 16) signs |= (uint32_t)((w >> 62) & 1u) << k;
    }
    const int mat = (NC == 4) ? (int)(st.passes & 1u) : 0;

    // chi-squared scale from the old pool (section 4, eq. 3)
    const double xstar = (double)P.X[nu - 1];
    const double t = xstar + P.r_nu;
    const double S = (t * t) * 0.5;
    const float c32 = (float)__builtin_sqrt(S / st.sigma);
    const float h = c32 * (NC == 4 ? 0.5f : 0.25f);

    const uint32_t j0 = (blockIdx.x * kThreads + threadIdx.x) * (uint32_t)T;
    float X[NC][T];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const float *src = P.X + (size_t)k * N;
#pragma unroll
        for (int i = 0; i < T; ++i) X[k][i] = src[(a[k] * (j0 + i) + b[k]) & mask];
    }
#pragma unroll
    for (int i = 0; i < T; ++i) {
        float v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = ((signs >> k) & 1u) ? -X[k][i] : X[k][i];
        if constexpr (NC == 4) {
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
    for (int k = 0; k < NC; ++k) {
        float *dst = P.Y + (size_t)k * N + j0;
#pragma unroll
        for (int i = 0; i < T; i += 4)
            *reinterpret_cast<v4f *>(dst + i) =
                v4f{X[k][i], X[k][i + 1], X[k][i + 2], X[k][i + 3]};
    }
    if (P.out) {
        const bool vec = P.emit_cnt == nu && !P.affine && ((uintptr_t)P.out & 15) == 0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            float *dst = P.out + (size_t)k * N + j0;
            if (vec) {
#pragma unroll
                for (int i = 0; i < T; i += 4)
                    __builtin_nontemporal_store(
                        v4f{X[k][i], X[k][i + 1], X[k][i + 2], X[k][i + 3]},
                        reinterpret_cast<v4f *>(dst + i));
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

    block_partials<Nd, NC, T>(X, P.partials, P.nblocks, red);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = (atomicAdd(P.counter, 1u) == P.nblocks - 1u) ? 1u : 0u;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const double sigma = final_tree<Nd, NC>(P.partials, P.nblocks, red);
    if (threadIdx.x == 0) {
        GenState ns = st;
        ns.rng = rng;
        ns.sigma = sigma;
        ns.passes = st.passes + 1;
        if (!__builtin_isfinite(c32)) ns.flags |= WALLACE_FLAG_NONFINITE;
        *P.state = ns;
        *P.counter = 0u;
        __threadfence();
    }
}

template <class Nd, int NC, int T>
const void *pass_fn()
{
    return reinterpret_cast<const void *>(&k_stream_pass<Nd, NC, T>);
}

template <int NC, int T>
const void *pass_fn_mode(uint32_t rmode)
{
    if (rmode == 1) return pass_fn<F32, NC, T>();
    if (rmode == 2) return pass_fn<F32C, NC, T>();
    return pass_fn<F64, NC, T>();
}

// Tuples per thread: at least 4 (16-byte stores) and enough that a pass
// needs at most 1024 blocks (the last block reduces 4 partials per thread).
int stream_T(int n, uint32_t N)
{
    uint32_t T = 4;
    while ((uint64_t)N / ((uint64_t)kThreads * T) > 1024) T *= 2;
    (void)n;
    return (int)T;
}

const void *pass_kernel(int n, uint32_t N, uint32_t rmode)
{
    const int T = stream_T(n, N);
    if (n == 4) {
        if (T == 4) return pass_fn_mode<4, 4>(rmode);
        if (T == 8) return pass_fn_mode<4, 8>(rmode);
        if (T == 16) return pass_fn_mode<4, 16>(rmode);
    } else if (n == 16) {
        if (T == 4) return pass_fn_mode<16, 4>(rmode);
    }
    return nullptr;
}

}  // namespace

bool stream_shape_ok(int n, uint32_t N)
{
    if (N < (uint32_t)kThreads * 4) return false;
    const int T = stream_T(n, N);
    return (n == 4 && T <= 16) || (n == 16 && T <= 4);
}

size_t stream_partials_bytes(int n, uint32_t N)
{
    if (N < (uint32_t)kThreads * 4) return 0;
    const uint32_t nb = N / (kThreads * (uint32_t)stream_T(n, N));
    return (size_t)n * nb * sizeof(double2);
}

const float *stream_current_pool(wallace_gen *g)
{
    const size_t off = (g->passes_host & 1) ? g->lay.pool2 : g->lay.pool;
    return reinterpret_cast<const float *>(g->ws + off);
}

hipError_t stream_check(wallace_gen *g, hipStream_t s)
{
    return launch_sumsq(stream_current_pool(g), g->nu, (uint32_t)g->opts.reduce_mode,
                        reinterpret_cast<double *>(g->ws + g->lay.scratch), nullptr,
                        g->state, 1, s);
}

hipError_t stream_run(wallace_gen *g, float *out, uint32_t passes, uint32_t last_emit,
                      uint32_t affine, float mu, float sig, hipStream_t s)
{
    const void *fn = pass_kernel(g->n, g->N, (uint32_t)g->opts.reduce_mode);
    if (!fn) return hipErrorInvalidValue;
    const int T = stream_T(g->n, g->N);
    const uint32_t nblocks = g->N / (kThreads * (uint32_t)T);
    float *pa = reinterpret_cast<float *>(g->ws + g->lay.pool);
    float *pb = reinterpret_cast<float *>(g->ws + g->lay.pool2);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(g->ws);
    const uint32_t f = (uint32_t)g->opts.f;
    for (uint32_t ps = 0; ps < passes; ++ps) {
        const bool odd = ((g->passes_host + ps) & 1) != 0;
        Pass P{};
        P.X = odd ? pb : pa;
        P.Y = odd ? pa : pb;
        P.out = nullptr;
        P.emit_cnt = 0;
        if ((ps + 1) % f == 0) {
            const uint32_t e = (ps + 1) / f - 1;
            P.out = out + (uint64_t)e * g->emit_len;
            P.emit_cnt = (ps + 1 == passes) ? last_emit : (uint32_t)g->emit_len;
        }
        P.affine = affine;
        P.mu = mu;
        P.sig = sig;
        P.state = g->state;
        P.partials = reinterpret_cast<double2 *>(g->ws + g->lay.partials);
        P.counter = &hdr->stream_ctr;
        P.r_nu = g->r_nu;
        P.N = g->N;
        P.a_mode = (uint32_t)g->opts.a_mode;
        P.nblocks = nblocks;
        void *args[] = {&P};
        hipError_t e = hipLaunchKernel(fn, dim3(nblocks), dim3(kThreads), args, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace wallace
