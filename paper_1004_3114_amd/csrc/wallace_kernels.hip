// Small HIP kernels of the Wallace generator library and the dispatch of the
// pool-resident pass kernels (wallace_pool.hpp, instantiated in
// wallace_pool_inst.hip): emission of leftover values of a partly returned
// pool, replication of a generator for tuning runs, and the canonical
// sum-of-squares tree over a pool in memory (initialisation and the
// corruption check of section 8's drift monitor).
#include "wallace_internal.h"
#include "wallace_pool.hpp"

#include "wallace.h"

namespace wallace {

// ---------------------------------------------------------------------------
// Sum-of-squares tree nodes (same three reduction modes as the pass kernels)
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

// Restart (section 5): refills a pool of nu values by Box-Muller from the
// splitmix64 stream at state r0, as the initial pool is made: pair m takes
// draws 2m+1 and 2m+2, u1 = ((w >> 11) + 1) 2^-53 in (0, 1], u2 = (w >> 11)
// 2^-53, cos to flat index 2m and sin to 2m+1, in FP64 rounded to FP32.
// The device's FP64 log, cos and sin are not the host's libm, so a value
// can differ from the host's in its last bit. Writes the state after the nu
// draws; the sum of squares is recomputed by the tree kernels afterwards.
__global__ void k_refill(float *pool, uint64_t nu, uint64_t r0, GenState *state)
{
    constexpr uint64_t gam = 0x9E3779B97F4A7C15ull;
    const uint64_t pairs = nu / 2;
    for (uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m < pairs;
         m += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t z1 = sm64_mix(r0 + (2 * m + 1) * gam);
        const uint64_t z2 = sm64_mix(r0 + (2 * m + 2) * gam);
        const double u1 = (double)((z1 >> 11) + 1) * 0x1.0p-53;
        const double u2 = (double)(z2 >> 11) * 0x1.0p-53;
        const double rho = __builtin_sqrt(-2.0 * log(u1));
        const double theta = (2.0 * 3.14159265358979323846) * u2;
        pool[2 * m] = (float)(rho * cos(theta));
        pool[2 * m + 1] = (float)(rho * sin(theta));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) state->rng = r0 + nu * gam;
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

namespace pool {
extern const PoolEntry pool_table_2_0[], pool_table_2_1[], pool_table_2_2[];
extern const int pool_table_len_2_0, pool_table_len_2_1, pool_table_len_2_2;
extern const PoolEntry pool_table_4_0[], pool_table_4_1[], pool_table_4_2[];
extern const PoolEntry pool_table_16_0[], pool_table_16_1[], pool_table_16_2[];
extern const int pool_table_len_4_0, pool_table_len_4_1, pool_table_len_4_2;
extern const int pool_table_len_16_0, pool_table_len_16_1, pool_table_len_16_2;
}  // namespace pool

static const pool::PoolEntry *pool_entry(const Sched &s, uint32_t rm)
{
    if (s.C < 1 || s.n % s.C) return nullptr;
    const int nst = s.n / s.C;
    const pool::PoolEntry *tab = nullptr;
    int len = 0;
    if (s.n == 2) {
        tab = rm == 1 ? pool::pool_table_2_1 : rm == 2 ? pool::pool_table_2_2 : pool::pool_table_2_0;
        len = rm == 1 ? pool::pool_table_len_2_1 : rm == 2 ? pool::pool_table_len_2_2 : pool::pool_table_len_2_0;
    } else if (s.n == 4) {
        tab = rm == 1 ? pool::pool_table_4_1 : rm == 2 ? pool::pool_table_4_2 : pool::pool_table_4_0;
        len = rm == 1 ? pool::pool_table_len_4_1 : rm == 2 ? pool::pool_table_len_4_2 : pool::pool_table_len_4_0;
    } else if (s.n == 16) {
        tab = rm == 1 ? pool::pool_table_16_1 : rm == 2 ? pool::pool_table_16_2 : pool::pool_table_16_0;
        len = rm == 1 ? pool::pool_table_len_16_1 : rm == 2 ? pool::pool_table_len_16_2 : pool::pool_table_len_16_0;
    }
    for (int i = 0; i < len; ++i)
        if (tab[i].T == s.T && tab[i].L == s.L && tab[i].nst == nst) return &tab[i];
    return nullptr;
}

int pool_block_threads(const Sched &s)
{
    const pool::PoolEntry *e = pool_entry(s, 0);
    return e ? e->block : 0;
}

size_t pool_lds_bytes(const Sched &s, int N)
{
    (void)N;
    const pool::PoolEntry *e = pool_entry(s, 0);
    return e ? (size_t)e->lds_bytes : 0;
}

bool pool_sched_supported(const Sched &s, int N)
{
    if (s.T * s.L != N) return false;
    const pool::PoolEntry *e = pool_entry(s, 0);
    return e && e->lds_bytes <= 160 * 1024;
}

// Kernels that need more than 64 KiB of LDS declare it once per process.
static hipError_t allow_lds(const void *fn, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t pool_max_blocks_per_cu(const Sched &s, int N, uint32_t rmode, int *blocks)
{
    const pool::PoolEntry *e = pool_entry(s, rmode);
    if (!e || e->T * e->L != N) return hipErrorInvalidValue;
    hipError_t err = allow_lds(e->fn, (size_t)e->lds_bytes);
    if (err != hipSuccess) return err;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, e->fn, e->block,
                                                        (size_t)e->lds_bytes);
}

hipError_t launch_pool(const Sched &s, const PoolArgs &a, int grid, hipStream_t stream)
{
    const pool::PoolEntry *e = pool_entry(s, a.rmode);
    if (!e || e->T * e->L != a.N || a.L != s.L || a.C != s.C) return hipErrorInvalidValue;
    hipError_t err = allow_lds(e->fn, (size_t)e->lds_bytes);
    if (err != hipSuccess) return err;
    PoolArgs args = a;
    void *kargs[] = {&args};
    return hipLaunchKernel(e->fn, dim3(grid), dim3(e->block), kargs, (size_t)e->lds_bytes, stream);
}

hipError_t launch_refill(float *pool, uint64_t nu, uint64_t r0, GenState *state,
                         hipStream_t stream)
{
    uint64_t grid = (nu / 2 + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_refill, dim3((unsigned)grid), dim3(256), 0, stream, pool, nu, r0,
                       state);
    return hipGetLastError();
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
hipError_t launch_sumsq(const float *pool, size_t nu, uint32_t rmode, double *scratch,
                        GenState *state, uint32_t mode, hipStream_t stream)
{
    double2 *s = reinterpret_cast<double2 *>(scratch);
    if (rmode == 1) return sumsq_chain<NodeF32>(pool, nu, s, state, mode, stream);
    if (rmode == 2) return sumsq_chain<NodeComp>(pool, nu, s, state, mode, stream);
    return sumsq_chain<NodeF64>(pool, nu, s, state, mode, stream);
}

}  // namespace wallace
