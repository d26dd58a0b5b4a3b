// Pool-resident pass kernels of the Wallace generator library (gfx950).
//
// One pass (Brent 1997, section 2, eq. 1) regenerates a pool of nu = n*N
// normals held as n component arrays of N values:
//   per-pass parameters: one splitmix64 draw per component k gives an odd
//   stride a_k and an offset b_k (eq. 2, sections 3 and 8) and, for n = 16,
//   a column sign;
//   gather v_k[j] = X_k[(a_k j + b_k) mod N];
//   y[j] = h * (butterflies of v[j]) with h = RN32(c) times the matrix's
//   power-of-two factor; c is the chi-squared scale computed from the old
//   pool (section 4, eq. 3), folded into the matrix as section 4 notes;
//   the new pool replaces the old (double buffering, section 2), is returned
//   in flat order f = k*N + j (section 3), and its sum of squares is formed
//   for the next pass (section 4).
//
// A group of L lanes owns one pool for a whole job. When the pool fits in
// the group's LDS share (every shape with one stage) it lives there between
// passes: lane l gathers tuples j = l + L*i (i < T), so the lanes of a wave
// read L consecutive multiples of the stride, which fall in distinct banks;
// the new values overwrite the image in place, and the lane then reads back
// tuples T*l .. T*l+T-1 for the sum of squares and 16-byte chunks
// l + L*q for the store to HBM, so that every store instruction of a wave
// covers consecutive output (run_job_lds). Larger pools (multi-wave groups
// only) live in registers, lane l holding tuples T*l .. T*l+T-1 of every
// component, and LDS is the per-pass permutation network, C = n/NST
// components at a time, in a swizzled layout (run_job). The per-pass draws
// are counter-based (splitmix64 draw m is a
// function of state + m * gamma), so each lane computes one pass's
// parameters for a chunk of up to 64 passes at once and every pass reads its
// parameters with one lane read per component. T and L are compile-time, so
// every LDS and store offset is an immediate.
//
// Bit-exactness: no FMA contraction (-ffp-contract=off), butterflies in a
// fixed order, and the sum of squares as the canonical pairwise tree over
// the flat index. FP64 leaves y*y are exact, so fma(y1, y1, y0*y0) equals
// the tree node y0^2 + y1^2 rounded once.
#pragma once

#include <type_traits>

#include "wallace_devmath.hpp"
#include "wallace_internal.h"
#include "wallace.h"

namespace wallace {
namespace pool {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

template <int V>
struct Log2 {
    static constexpr int value = 1 + Log2<V / 2>::value;
};
template <>
struct Log2<1> {
    static constexpr int value = 0;
};

// Splitmix64 draws per pass: one per component, and for n = 2 one more for
// the rotation (section 8).
template <int NC>
struct Draws {
    static constexpr int value = NC == 2 ? 3 : NC;
};

// n = 2: x' = p x + q y, y' = p y - q x, each product and the sum rounded
// once (two multiplies and one add per number, section 7).
__device__ __forceinline__ void xform2(float (&v)[2], float p, float q)
{
    const float px = p * v[0], qy = q * v[1], py = p * v[1], qx = q * v[0];
    v[0] = px + qy;
    v[1] = py - qx;
}

template <bool MW>
__device__ __forceinline__ void group_sync()
{
    if constexpr (MW) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
        // one wave: LDS executes its instructions in order; only the
        // compiler must not move LDS accesses across this point
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// Exchange of a 32-bit value with lane (lane ^ M), M = 1..32. Every partner
// is the exact xor partner, so the same helper serves reductions whose lanes
// hold different values.
template <int M>
__device__ __forceinline__ int xchg(int v)
{
    if constexpr (M == 1)
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
    else if constexpr (M == 2)
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm 2,3,0,1
    else if constexpr (M == 4 || M == 8 || M == 16)
        return __builtin_amdgcn_ds_swizzle(v, 0x1F | (M << 10));  // bit mode, xor M
    else
        return __builtin_amdgcn_ds_bpermute((int)((__lane_id() ^ 32u) << 2), v);
}

template <int M>
__device__ __forceinline__ float xchg(float v)
{
    return __int_as_float(xchg<M>(__float_as_int(v)));
}

template <int M>
__device__ __forceinline__ double xchg(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(xchg<M>(hi), xchg<M>(lo));
}

// Sum-of-squares tree nodes of the three reduction modes.
struct NodeF64 {  // FP64 nodes; leaves (double)y * (double)y are exact
    double v;
    __device__ static NodeF64 leaf(float y) { return {(double)y * (double)y}; }
    // node of the pair (y0, y1): one rounding of y0^2 + y1^2
    __device__ static NodeF64 leaf2(float y0, float y1)
    {
        const double d0 = (double)y0, d1 = (double)y1;
        return {__builtin_fma(d1, d1, d0 * d0)};
    }
    __device__ static NodeF64 zero() { return {0.0}; }
    __device__ static NodeF64 join(NodeF64 a, NodeF64 b) { return {a.v + b.v}; }
    template <int M>
    __device__ static NodeF64 xch(NodeF64 a) { return {xchg<M>(a.v)}; }
    __device__ static NodeF64 sel(bool c, NodeF64 a, NodeF64 b) { return c ? a : b; }
    __device__ double value() const { return v; }
    __device__ void put(char *p) const { *reinterpret_cast<double *>(p) = v; }
    __device__ static NodeF64 get(const char *p) { return {*reinterpret_cast<const double *>(p)}; }
    __device__ NodeF64 uniform() const
    {
        return {__hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                                 __builtin_amdgcn_readfirstlane(__double2loint(v)))};
    }
    static constexpr int kBytes = 8;
};

struct NodeF32 {  // FP32 nodes (the plain FP32 reduction)
    float v;
    __device__ static NodeF32 leaf(float y) { return {y * y}; }
    __device__ static NodeF32 leaf2(float y0, float y1) { return join(leaf(y0), leaf(y1)); }
    __device__ static NodeF32 zero() { return {0.0f}; }
    __device__ static NodeF32 join(NodeF32 a, NodeF32 b) { return {a.v + b.v}; }
    template <int M>
    __device__ static NodeF32 xch(NodeF32 a) { return {xchg<M>(a.v)}; }
    __device__ static NodeF32 sel(bool c, NodeF32 a, NodeF32 b) { return c ? a : b; }
    __device__ double value() const { return (double)v; }
    __device__ void put(char *p) const { *reinterpret_cast<float *>(p) = v; }
    __device__ static NodeF32 get(const char *p) { return {*reinterpret_cast<const float *>(p)}; }
    __device__ NodeF32 uniform() const
    {
        return {__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)))};
    }
    static constexpr int kBytes = 4;
};

struct NodeComp {  // FP32 value and FP32 error term (TwoProd leaves, TwoSum joins)
    float s, e;
    __device__ static NodeComp leaf(float y)
    {
        const float p = y * y;
        return {p, __builtin_fmaf(y, y, -p)};
    }
    __device__ static NodeComp leaf2(float y0, float y1) { return join(leaf(y0), leaf(y1)); }
    __device__ static NodeComp zero() { return {0.0f, 0.0f}; }
    __device__ static NodeComp join(NodeComp a, NodeComp b)
    {
        const float sum = a.s + b.s;
        const float bb = sum - a.s;
        const float err = (a.s - (sum - bb)) + (b.s - bb);
        return {sum, (a.e + b.e) + err};
    }
    template <int M>
    __device__ static NodeComp xch(NodeComp a) { return {xchg<M>(a.s), xchg<M>(a.e)}; }
    __device__ static NodeComp sel(bool c, NodeComp a, NodeComp b) { return c ? a : b; }
    __device__ double value() const { return (double)s + (double)e; }
    __device__ void put(char *p) const { *reinterpret_cast<v2f *>(p) = v2f{s, e}; }
    __device__ static NodeComp get(const char *p)
    {
        const v2f q = *reinterpret_cast<const v2f *>(p);
        return {q.x, q.y};
    }
    __device__ NodeComp uniform() const
    {
        return {__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s))),
                __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(e)))};
    }
    static constexpr int kBytes = 8;
};

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

// Canonical tree over the T consecutive values of one component in a lane.
template <class Nd, int T>
__device__ __forceinline__ Nd lane_tree(const float (&x)[T])
{
    if constexpr (T == 1) {
        return Nd::leaf(x[0]);
    } else {
        Nd t[T / 2];
#pragma unroll
        for (int i = 0; i < T / 2; ++i) t[i] = Nd::leaf2(x[2 * i], x[2 * i + 1]);
#pragma unroll
        for (int w = T / 2; w > 1; w >>= 1) {
#pragma unroll
            for (int i = 0; i < w / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
        }
        return t[0];
    }
}

// Butterfly over lane bits [M0, log2 W): afterwards every lane of each
// aligned group of W lanes holds the group's node.
template <class Nd, int M, int W>
__device__ __forceinline__ Nd butterfly(Nd a)
{
    if constexpr (M >= W) {
        return a;
    } else {
        a = Nd::join(a, Nd::template xch<M>(a));
        return butterfly<Nd, 2 * M, W>(a);
    }
}

// One halving level at lane bit m (mask M = 2^m): a lane keeps half of the
// V components it carries and adds the partner's node of the same
// components (the partner keeps the other half).
template <class Nd, int M, int V>
__device__ __forceinline__ void halve(Nd (&v)[16], bool hi)
{
#pragma unroll
    for (int t = 0; t < V / 2; ++t) {
        const Nd keep = Nd::sel(hi, v[t + V / 2], v[t]);
        const Nd send = Nd::sel(hi, v[t], v[t + V / 2]);
        v[t] = Nd::join(keep, Nd::template xch<M>(send));
    }
}

template <class Nd, int M, int V>
__device__ __forceinline__ void halve_all(Nd (&v)[16], int wl)
{
    if constexpr (V > 1) {
        halve<Nd, M, V>(v, (wl & M) != 0);
        halve_all<Nd, 2 * M, V / 2>(v, wl);
    }
}

// Component levels after halving: kappa and kappa ^ 2^q sit in lanes that
// differ in bit log2(n) - 1 - q.
template <class Nd, int M>
__device__ __forceinline__ Nd comp_levels(Nd a)
{
    if constexpr (M == 0) {
        return a;
    } else {
        a = Nd::join(a, Nd::template xch<M>(a));
        return comp_levels<Nd, M / 2>(a);
    }
}

template <int NC, int T, int L, int RM, int NST>
struct Cfg {
    static constexpr int N = T * L;
    static constexpr int C = NC / NST;
    static constexpr bool MW = L > 64;
    static constexpr bool UNIFORM = L >= 64;   // a group is one or more whole waves
    static constexpr int GPB = MW ? 1 : 256 / L;   // groups per block
    static constexpr int BLOCK = MW ? L : 256;
    static constexpr int W = MW ? L / 64 : 1;      // waves per group
    using Nd = typename NodeOf<RM>::type;
    // One stage (the whole pool fits): the pool lives in LDS between passes
    // (run_job_lds). Several stages (only multi-wave groups with pools over
    // 128 KiB): it lives in registers and LDS holds C components at a time
    // (run_job).
    static constexpr bool LDSRES = NST == 1;
    static_assert(LDSRES || MW, "several stages only for multi-wave groups");
    // swizzled stage images (register-resident form; see swz4)
    static constexpr bool SWZ = !LDSRES && T >= 2;
    // register-resident with more than 4 tuples per lane: the output goes
    // through wave-private LDS slices (emit_transposed); L/64 waves times C
    // slices of 64*T floats fill the C*N floats of the stage area exactly
    static constexpr bool EMIT_LDS = !LDSRES && T > 4;
    static constexpr int POOL_BYTES = C * N * 4;
    // groups sharing a wave start L words apart in bank terms, so their
    // lanes use different banks
    static constexpr int GROUP_BYTES = POOL_BYTES + (L < 64 ? 4 * L : 0);
    static constexpr int CH = L >= 64 ? 64 : L;  // passes per parameter chunk
    static constexpr int XW_BYTES = MW ? 16 * W * NC : 0;  // cross-wave nodes
    static constexpr int LDS_BYTES = GPB * GROUP_BYTES + XW_BYTES;
};

// Sum of squares of a pool held by a multi-wave group, in two halves so that
// a pass can overlap the first with other work. First half: per lane a tree
// over its T consecutive values of each component; within each wave the
// halving levels (each joins lane pairs in tree order while the lanes split
// the components) and the remaining lane levels; lane kappa of each wave
// leaves its node of component kappa in the cross-wave area. GUARD: wait
// first until every wave has read that area in the previous call.
// The node is computed in registers only (pool_sumsq_node) and stored by
// pool_sumsq_put, so a pass can keep it in registers past other LDS work.
template <int NC, int T, int L, int RM, int NST>
__device__ __forceinline__ typename Cfg<NC, T, L, RM, NST>::Nd pool_sumsq_node(
    const float (&X)[NC][T], int lane)
{
    using C = Cfg<NC, T, L, RM, NST>;
    using Nd = typename C::Nd;
    static_assert(C::MW, "multi-wave groups; pool_sumsq_regs serves one wave or less");
    Nd v[16];
#pragma unroll
    for (int k = 0; k < NC; ++k) v[k] = lane_tree<Nd, T>(X[k]);
    halve_all<Nd, 1, NC>(v, lane & 63);
    return butterfly<Nd, NC, 64>(v[0]);
}

template <int NC, class Nd>
__device__ __forceinline__ void pool_sumsq_put(const Nd &acc, int lane, char *xw_lds)
{
    constexpr int LOG_NC = Log2<NC>::value;
    const int wl = lane & 63;
    const int wave = lane >> 6;
    int kappa = 0;
#pragma unroll
    for (int m = 0; m < LOG_NC; ++m) kappa |= ((wl >> m) & 1) << (LOG_NC - 1 - m);
    if (wl < NC) acc.put(xw_lds + (wave * NC + kappa) * 16);
}

template <int NC, int T, int L, int RM, int NST, bool GUARD>
__device__ __forceinline__ void pool_sumsq_wave(const float (&X)[NC][T], int lane, char *xw_lds)
{
    const auto acc = pool_sumsq_node<NC, T, L, RM, NST>(X, lane);
    if constexpr (GUARD) group_sync<true>();  // earlier readers of the cross-wave area are done
    pool_sumsq_put<NC>(acc, lane, xw_lds);
}

// Second half, after a group barrier that follows every wave's first half:
// the waves' nodes in order, then the component levels. Every lane returns
// the total.
template <int NC, int T, int L, int RM, int NST>
__device__ __forceinline__ double pool_sumsq_join(int lane, const char *xw_lds)
{
    using C = Cfg<NC, T, L, RM, NST>;
    using Nd = typename C::Nd;
    constexpr int LOG_NC = Log2<NC>::value;
    const int wl = lane & 63;
    int kappa = 0;
#pragma unroll
    for (int m = 0; m < LOG_NC; ++m) kappa |= ((wl >> m) & 1) << (LOG_NC - 1 - m);
    Nd t[C::W];
#pragma unroll
    for (int w = 0; w < C::W; ++w) t[w] = Nd::get(xw_lds + (w * NC + kappa) * 16);
#pragma unroll
    for (int s = C::W; s > 1; s >>= 1) {
#pragma unroll
        for (int i = 0; i < s / 2; ++i) t[i] = Nd::join(t[2 * i], t[2 * i + 1]);
    }
    const Nd acc = comp_levels<Nd, NC / 2>(t[0]);
    // lanes 0..NC-1 of every wave now hold the total; lane 0 is uniform
    return acc.uniform().value();
}

// Both halves with the barrier between them.
template <int NC, int T, int L, int RM, int NST, bool GUARD = true>
__device__ __forceinline__ double pool_sumsq(const float (&X)[NC][T], int lane, char *xw_lds)
{
    pool_sumsq_wave<NC, T, L, RM, NST, GUARD>(X, lane, xw_lds);
    group_sync<true>();
    return pool_sumsq_join<NC, T, L, RM, NST>(lane, xw_lds);
}

// Sum of squares of a pool held by a group of at most one wave, in registers
// only: the same halving as the multi-wave path (each exchange level joins
// lane pairs in tree order while the lanes split the components), then the
// remaining lane levels and the component levels. Every lane of the group
// ends with the total.
template <int NC, int T, int L, int RM>
__device__ __forceinline__ double pool_sumsq_regs(const float (&X)[NC][T], int lane)
{
    using Nd = typename NodeOf<RM>::type;
    static_assert(L <= 64 && L >= NC, "one wave or less, at least n lanes");
    Nd v[16];
#pragma unroll
    for (int k = 0; k < NC; ++k) v[k] = lane_tree<Nd, T>(X[k]);
    const int wl = lane & 63;
    halve_all<Nd, 1, NC>(v, wl);
    Nd acc = butterfly<Nd, NC, L>(v[0]);
    acc = comp_levels<Nd, NC / 2>(acc);
    return (L >= 64 ? acc.uniform() : acc).value();
}

// n = 4: A0 = H4/2 (mat 0) and A1 = J/2 - I (mat 1) with
// A1 = D_r P (H4/2) D_c, D_c = diag(-1,1,1,1), P swapping rows 1 and 2,
// D_r = diag(1,-1,-1,-1).
__device__ __forceinline__ void xform4(float (&v)[4], int mat, float h)
{
    const float v0 = mat ? -v[0] : v[0];
    const float s0 = v0 + v[1], s1 = v0 - v[1];
    const float s2 = v[2] + v[3], s3 = v[2] - v[3];
    const float u0 = s0 + s2, u1 = s1 + s3, u2 = s0 - s2, u3 = s1 - s3;
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

// n = 16: H16 D / 4, D = diag((-1)^(bit k of signs)), radix-2 stages 1,2,4,8.
__device__ __forceinline__ void xform16(float (&v)[16], uint32_t signs, float h)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = ((signs >> k) & 1u) ? -v[k] : v[k];
#pragma unroll
    for (int s = 1; s < 16; s <<= 1) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i & s) continue;
            const float lo = v[i], hi = v[i + s];
            v[i] = lo + hi;
            v[i + s] = lo - hi;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = v[k] * h;
}

template <int T>
__device__ __forceinline__ void load_run(float (&x)[T], const float *p)
{
    if constexpr (T % 4 == 0) {
#pragma unroll
        for (int i = 0; i < T; i += 4) {
            const v4f q = *reinterpret_cast<const v4f *>(p + i);
            x[i] = q.x;
            x[i + 1] = q.y;
            x[i + 2] = q.z;
            x[i + 3] = q.w;
        }
    } else if constexpr (T == 2) {
        const v2f q = *reinterpret_cast<const v2f *>(p);
        x[0] = q.x;
        x[1] = q.y;
    } else {
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

// A lane's T consecutive values into LDS with vector stores.
template <int T>
__device__ __forceinline__ void store_lds(float *p, const float (&x)[T])
{
    if constexpr (T % 4 == 0) {
#pragma unroll
        for (int i = 0; i < T; i += 4)
            *reinterpret_cast<v4f *>(p + i) = v4f{x[i], x[i + 1], x[i + 2], x[i + 3]};
    } else if constexpr (T == 2) {
        *reinterpret_cast<v2f *>(p) = v2f{x[0], x[1]};
    } else {
        p[0] = x[0];
    }
}

// Stage images of the register-resident form keep word x of a component at
// x ^ ((x >> 6) & (T - 1)). A wave's gather reads words a*T apart (a odd):
// without the swizzle only 64/T banks would serve the 64 lanes; with it
// every lane of a 64-word row group lands in its own bank. The swizzle stays
// inside T-word blocks, so a lane's T values remain in its own block.
// Byte-address form: x4 = 4x.
template <int T>
__device__ __forceinline__ uint32_t swz4(uint32_t x4)
{
    return x4 ^ ((x4 >> 6) & (uint32_t)(4 * (T - 1)));
}

// A lane's T consecutive values into a swizzled stage image; blk4 is the
// byte offset of the lane's block with the swizzle applied to its first
// word (the swizzle of word B + t is (B + sw) ^ t for the block base B).
template <int T>
__device__ __forceinline__ void store_lds_swz(char *comp, uint32_t blk4, const float (&x)[T])
{
#pragma unroll
    for (int t = 0; t < T; ++t) *reinterpret_cast<float *>(comp + (blk4 ^ (uint32_t)(4 * t))) = x[t];
}

// Output of the new pool of a multi-wave group whose lanes hold T > 4
// consecutive values per component. Stored straight from registers, each
// store instruction of a wave would be lane-strided (T*4 bytes between
// lanes), a pattern that streams several times slower than consecutive
// chunks. Instead each wave passes its values through a private slice of
// the stage area (64*T floats per component, free once every gather of the
// pass is done) and reads them back transposed: store instruction s of a
// wave covers its 16-byte chunks 64*s .. 64*s + 63, 1 KB of consecutive
// output. Chunk c of a slice sits in slot c ^ ((c >> 4) & (Q - 1)), which
// keeps the 16 lanes of each quarter-wave in distinct slots mod 16 both
// when writing (c = Q*lane + q) and when reading (c = 64*s + lane). Slices
// are wave-private and LDS operations of a wave complete in order, so the C
// components of one round and the rounds after it need no barrier.
template <int NC, int T, int C, int N>
__device__ __forceinline__ void emit_transposed(const float (&X)[NC][T], float *out, char *lds,
                                                uint32_t ln)
{
    static_assert(T % 4 == 0 && T > 4, "whole chunks, more than one per lane");
    constexpr int Q = T / 4;                  // 16-byte chunks per lane and component
    constexpr uint32_t SL = 64u * T * 4u;      // bytes of one slice
    const uint32_t w = ln >> 6, wl = ln & 63u;
    auto slot = [](uint32_t c) { return c ^ ((c >> 4) & (uint32_t)(Q - 1)); };
#pragma unroll
    for (int r = 0; r < NC / C; ++r) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            char *sl = lds + (w * (uint32_t)C + (uint32_t)c) * SL;
            const float(&x)[T] = X[r * C + c];
#pragma unroll
            for (int q = 0; q < Q; ++q)
                *reinterpret_cast<v4f *>(sl + 16u * slot((uint32_t)Q * wl + (uint32_t)q)) =
                    v4f{x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]};
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const char *sl = lds + (w * (uint32_t)C + (uint32_t)c) * SL;
            // the wave's tuples start at 64*T*w
            v4f *o = reinterpret_cast<v4f *>(out + (r * C + c) * N + 64u * T * w);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint32_t k = 64u * (uint32_t)q + wl;
                __builtin_nontemporal_store(*reinterpret_cast<const v4f *>(sl + 16u * slot(k)), o + k);
            }
        }
    }
}

// Compile-time loop: f(integral_constant<int, I>) for I in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        static_for<B + 1, E>(f);
    }
}

// Element-wise emission: partial pools, unaligned outputs, N(mu, sigma^2).
// One base address per component; the T values of a lane are immediate
// offsets from it, and value i is inside the emitted prefix iff i < lim.
template <int NC, int T, int N>
__device__ __forceinline__ void emit_slow(const float (&X)[NC][T], float *base, uint32_t cnt,
                                          int lane, uint32_t affine, float mu, float sig)
{
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int32_t lim = (int32_t)cnt - (int32_t)(k * N) - (int32_t)(T * lane);
        if (lim <= 0) continue;
        float *bk = base + (k * N + T * lane);
#pragma unroll
        for (int i = 0; i < T; ++i) {
            if (i < lim) {
                float y = X[k][i];
                if (affine) y = mu + sig * y;
                __builtin_nontemporal_store(y, bk + i);
            }
        }
    }
}

// Lane-broadcast of a per-lane word within the group: lane `src` (< CH) of
// the wave (groups of >= 64 lanes) or of the group (smaller groups).
template <int L>
__device__ __forceinline__ uint32_t bcast(uint32_t v, uint32_t src)
{
    if constexpr (L >= 64)
        return __builtin_amdgcn_readlane(v, src);
    else
        return (uint32_t)__shfl((int)v, (int)src, L);
}

// Parameters of pass `pass` (0-based within the job) from the job's starting
// splitmix64 state: component k uses draw number Draws*pass + k + 1 (section
// 8 draws). Per component a packed word 4a | 4b << 16 (N <= 2^14): stride a
// (eq. 2; a table prime, or any odd value in a_mode 1, reduced mod N and
// made distinct and above one, sections 3 and 9) and offset b; for n = 16
// also the column sign bits.
template <int NC, int N>
__device__ __forceinline__ void pass_words(uint64_t rng0, uint32_t pass, uint32_t a_mode,
                                           uint32_t (&words)[NC], uint32_t *signs)
{
    constexpr uint32_t mask = (uint32_t)N - 1u;
    // with N above the largest table prime, table strides never clash
    constexpr bool table_may_clash = (uint32_t)N <= max_table_stride(NC);
    uint32_t a[NC];
    *signs = 0;
    static_for<0, NC>([&](auto k_c) {
        constexpr int k = decltype(k_c)::value;
        const uint64_t m = (uint64_t)Draws<NC>::value * pass + (uint64_t)(k + 1);
        const uint64_t w = sm64_mix(rng0 + m * kGamma);
        const uint32_t ak = a_mode ? ((uint32_t)(w >> 32) | 1u) : stride_pick(k, (uint32_t)(w >> 63));
        uint32_t ar = ak & mask;
        if (table_may_clash || a_mode) ar = distinct_stride<k>(ar, a, (uint32_t)N);
        a[k] = ar;
        const uint32_t b = (uint32_t)w & mask;
        if (NC == 16) *signs |= (uint32_t)((w >> 62) & 1u) << k;
        words[k] = (ar << 2) | ((b << 2) << 16);
    });
}

template <int NC, int T, int L, int RM, int NST>
__device__ void run_job(const PoolArgs &P, const Job &job, float *lds, char *xw, int lane)
{
    using Cf = Cfg<NC, T, L, RM, NST>;
    constexpr int N = Cf::N;
    constexpr int C = Cf::C;
    constexpr int CH = Cf::CH;
    constexpr bool MW = Cf::MW;
    constexpr uint32_t nu = (uint32_t)(NC * N);
    constexpr uint32_t amask = 4u * (uint32_t)N - 4u;
    static_assert(N <= (1 << 14), "packed parameters need N <= 2^14");

    float X[NC][T];
    const float *pool = P.pools + job.pool_off;
#pragma unroll
    for (int k = 0; k < NC; ++k) load_run<T>(X[k], pool + k * N + T * lane);

    GenState *stp = P.states + job.gen;
    const uint64_t rng0 = stp->rng;
    double sigma = stp->sigma;
    const uint64_t done = stp->passes;
    uint32_t flags = stp->flags;

    if (P.sigma_mode) {
        const double s = pool_sumsq<NC, T, L, RM, NST>(X, lane, xw);
        if (P.sigma_mode == 2)
            sigma = s;
        else if (!(s == sigma))
            flags |= WALLACE_FLAG_CORRUPT;
    }
    const uint32_t passes = (flags & WALLACE_FLAG_CORRUPT) ? 0u : job.passes;
    const uint32_t qlane = (uint32_t)lane % (uint32_t)CH;  // pass slot this lane computes

    uint32_t words[NC];  // packed (4a, 4b) of pass chunk + qlane, per component
    uint32_t swords = 0; // column signs of that pass (n = 16)
    double rcs = 0.0, rsn = 0.0;  // rotation of that pass (n = 2)
    uint32_t slot = 0;   // pass index within the chunk
    auto draw_chunk = [&](uint32_t ps0) {
        // this lane's pass of the chunk starting at ps0 (eq. 1, section 8 draws)
        pass_words<NC, N>(rng0, ps0 + qlane, P.a_mode, words, &swords);
        if constexpr (NC == 2) {
            const uint64_t m = 3ull * (ps0 + qlane) + 3ull;
            rotation(sm64_mix(rng0 + m * kGamma), rcs, rsn);
        }
        slot = 0;
    };
    uint32_t fcount = 0; // passes since the last returned pool
    uint32_t emitted = 0;

    // One pass with the matrix fixed at compile time (n = 4 alternates A0
    // and A1; a uniform branch picks the body, so no per-value selects).
    auto one_pass = [&](uint32_t ps, auto mat_c) {
        // The lane index is made opaque once per pass, so the compiler
        // recomputes the per-value LDS and output offsets derived from it
        // instead of keeping them in registers across the pass loop (which
        // made the largest shapes spill inside the loop).
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const uint32_t pj0 = (uint32_t)(T * ln);  // first tuple of this lane
        const uint32_t pblk = swz4<T>(4u * pj0);  // its block in a stage image
        constexpr int MAT = decltype(mat_c)::value;
        const uint32_t signs = NC == 16 ? bcast<L>(swords, slot) : 0u;
        double cs = 0.0, sn = 0.0;
        if constexpr (NC == 2) {
            cs = __hiloint2double((int)bcast<L>((uint32_t)__double2hiint(rcs), slot),
                                  (int)bcast<L>((uint32_t)__double2loint(rcs), slot));
            sn = __hiloint2double((int)bcast<L>((uint32_t)__double2hiint(rsn), slot),
                                  (int)bcast<L>((uint32_t)__double2loint(rsn), slot));
        }
        // stage st of the current pool into the LDS stage image (swizzled)
        auto store_stage = [&](auto st_c) {
            constexpr int st = decltype(st_c)::value;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (Cf::SWZ)
                    store_lds_swz<T>(reinterpret_cast<char *>(lds + c * N), pblk, X[st * C + c]);
                else
                    store_lds<T>(lds + c * N + pj0, X[st * C + c]);
            }
        };
        // gather of eq. (1) for the components of stage st from its image
        auto gather_stage = [&](auto st_c) {
            constexpr int st = decltype(st_c)::value;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const uint32_t wd = bcast<L>(words[st * C + c], slot);
                const uint32_t a4 = wd & 0xFFFFu, b4 = wd >> 16;
                const char *src = reinterpret_cast<const char *>(lds + c * N);
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    // 4 * ((a j + b) mod N) for tuple j = T*lane + i
                    const uint32_t x4 = (__umul24(a4, pj0 + i) + b4) & amask;
                    X[st * C + c][i] =
                        *reinterpret_cast<const float *>(src + (Cf::SWZ ? swz4<T>(x4) : x4));
                }
            }
        };
        // the old pool's last flat value (section 4): last word of the last
        // component of the last stage
        auto read_xstar = [&]() {
            return (double)*reinterpret_cast<const float *>(
                reinterpret_cast<const char *>(lds + (C - 1) * N) +
                (Cf::SWZ ? swz4<T>(4u * (N - 1)) : 4u * (N - 1)));
        };
        double xstar = 0.0;
        static_for<0, NST>([&](auto st_c) {
            group_sync<MW>();  // previous readers of this LDS space are done
            store_stage(st_c);
            group_sync<MW>();
            if (decltype(st_c)::value == NST - 1) xstar = read_xstar();
            gather_stage(st_c);
        });
        ++slot;

        const double c64 = chi2_scale64(xstar, sigma, P.r_nu);
        const float c32 = (float)c64;
        if (!__builtin_isfinite(c32)) flags |= WALLACE_FLAG_NONFINITE;
        // n = 4, 16: the matrix's power-of-two factor; n = 2: c folds into
        // the rotation entries, each rounded once (section 4)
        const float h = c32 * (NC == 4 ? 0.5f : 0.25f);
        const float rp = NC == 2 ? (float)(c64 * cs) : 0.0f;
        const float rq = NC == 2 ? (float)(c64 * sn) : 0.0f;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            float v[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) v[k] = X[k][i];
            if constexpr (NC == 4)
                xform4(v, MAT, h);
            else if constexpr (NC == 2)
                xform2(v, rp, rq);
            else
                xform16(v, signs, h);
#pragma unroll
            for (int k = 0; k < NC; ++k) X[k][i] = v[k];
        }

        // return the new pool when it is a returned one (section 6)
        float *base = nullptr;
        uint32_t cnt = 0;
        bool fast = false;
        if (++fcount == P.f) {
            fcount = 0;
            const bool last = (ps + 1 == passes);
            cnt = last ? job.last_emit : P.emit_len;
            base = P.out + job.out_off + (uint64_t)emitted * P.emit_len;
            ++emitted;
            constexpr uintptr_t vmask = (uintptr_t)(4 * (T >= 4 ? 4 : T) - 1);
            fast = cnt == nu && ((uintptr_t)base & vmask) == 0 && !P.affine;
        }
        if (base) {
            if (!fast) {
                emit_slow<NC, T, N>(X, base, cnt, ln, P.affine, P.mu, P.sigma_out);
            } else if constexpr (Cf::EMIT_LDS) {
                group_sync<MW>();  // every gather of the stage area is done
                emit_transposed<NC, T, C, N>(X, base, reinterpret_cast<char *>(lds), (uint32_t)ln);
            } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) store_run<T, true>(base + k * N + T * ln, X[k]);
            }
        }

        // the next call comes after the next pass's stage barriers
        sigma = pool_sumsq<NC, T, L, RM, NST, false>(X, ln, xw);
    };

    // Chunks of CH passes (CH is even, so every chunk starts on the same
    // matrix); two passes per iteration (n = 4: A0 then A1), so the sum of
    // squares of one pass and the permutation of the next share a block
    // (measured faster for every shape, multi-wave groups included).
    using M0 = std::integral_constant<int, 0>;
    using M1 = std::integral_constant<int, NC == 4 ? 1 : 0>;
    const bool odd = NC == 4 && (done & 1u);
    for (uint32_t c0 = 0; c0 < passes; c0 += (uint32_t)CH) {
        const uint32_t end = passes - c0 < (uint32_t)CH ? passes : c0 + (uint32_t)CH;
        draw_chunk(c0);
        uint32_t ps = c0;
        if (odd) one_pass(ps++, M1());
        for (; ps + 2 <= end; ps += 2) {
            one_pass(ps, M0());
            one_pass(ps + 1, M1());
        }
        if (ps < end) one_pass(ps, M0());
    }

    float *wpool = P.pools + job.pool_off;
#pragma unroll
    for (int k = 0; k < NC; ++k) store_run<T, false>(wpool + k * N + T * lane, X[k]);
    if (lane == 0) {
        stp->rng = rng0 + (uint64_t)Draws<NC>::value * passes * kGamma;
        stp->sigma = sigma;
        stp->passes = done + passes;
        stp->flags = flags;
    }
}

// One job with the pool resident in LDS between passes (one stage). Each
// pass: lane l gathers tuples j = l + L*i (i < T) from the old pool's LDS
// image; consecutive lanes then read addresses a apart (a odd), which hits
// distinct banks. The new pool overwrites the image in the same tuple
// order; the lanes read it back as T consecutive tuples each (the order of
// the output and of the sum-of-squares tree) for emission and the sum of
// squares.
template <int NC, int T, int L, int RM>
__device__ void run_job_lds(const PoolArgs &P, const Job &job, float *lds, char *xw, int lane)
{
    using Cf = Cfg<NC, T, L, RM, 1>;
    constexpr int N = Cf::N;
    constexpr int CH = Cf::CH;
    constexpr bool MW = Cf::MW;
    constexpr uint32_t nu = (uint32_t)(NC * N);
    constexpr uint32_t amask = 4u * (uint32_t)N - 4u;
    static_assert(N <= (1 << 14), "packed parameters need N <= 2^14");

    GenState *stp = P.states + job.gen;
    const uint64_t rng0 = stp->rng;
    double sigma = stp->sigma;
    const uint64_t done = stp->passes;
    uint32_t flags = stp->flags;

    // in_pass: the call follows the pass's image barriers, which every wave
    // reaches only after reading the previous call's cross-wave area
    auto sumsq = [&](const float (&Z)[NC][T], auto in_pass) -> double {
        if constexpr (MW)
            return pool_sumsq<NC, T, L, RM, 1, !decltype(in_pass)::value>(Z, lane, xw);
        else
            return pool_sumsq_regs<NC, T, L, RM>(Z, lane);
    };

    {
        float Z[NC][T];
        const float *pool = P.pools + job.pool_off;
#pragma unroll
        for (int k = 0; k < NC; ++k) load_run<T>(Z[k], pool + k * N + T * lane);
        if (P.sigma_mode) {
            const double s = sumsq(Z, std::false_type());
            if (P.sigma_mode == 2)
                sigma = s;
            else if (!(s == sigma))
                flags |= WALLACE_FLAG_CORRUPT;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) store_lds<T>(lds + k * N + T * lane, Z[k]);
    }
    group_sync<MW>();
    const uint32_t passes = (flags & WALLACE_FLAG_CORRUPT) ? 0u : job.passes;
    const uint32_t qlane = (uint32_t)lane % (uint32_t)CH;

    uint32_t words[NC];
    uint32_t swords = 0;
    double rcs = 0.0, rsn = 0.0;
    uint32_t slot = 0;
    auto draw_chunk = [&](uint32_t ps0) {
        pass_words<NC, N>(rng0, ps0 + qlane, P.a_mode, words, &swords);
        if constexpr (NC == 2) {
            const uint64_t m = 3ull * (ps0 + qlane) + 3ull;
            rotation(sm64_mix(rng0 + m * kGamma), rcs, rsn);
        }
        slot = 0;
    };
    uint32_t fcount = 0;
    uint32_t emitted = 0;
    // Multi-wave groups pipeline the sum of squares: a pass leaves each
    // wave's node of its new pool in the cross-wave area, and the next pass
    // joins them after the barrier that also ends its gathers. The per-wave
    // work overlaps the next gathers, the butterflies (n = 4, 16) run before
    // the scale is known (the scale is their last multiply; times 1 is
    // exact), and a pass needs two barriers instead of three.
    bool pending = false;  // the previous pass's wave node awaits its join
    typename Cf::Nd pend{};  // that node, kept in registers until the barrier

    auto one_pass = [&](uint32_t ps, auto mat_c) {
        constexpr int MAT = decltype(mat_c)::value;
        constexpr bool SPLIT = MW && NC != 2;  // n = 2: the scale is inside the rotation
        const uint32_t signs = NC == 16 ? bcast<L>(swords, slot) : 0u;
        double cs = 0.0, sn = 0.0;
        if constexpr (NC == 2) {
            cs = __hiloint2double((int)bcast<L>((uint32_t)__double2hiint(rcs), slot),
                                  (int)bcast<L>((uint32_t)__double2loint(rcs), slot));
            sn = __hiloint2double((int)bcast<L>((uint32_t)__double2hiint(rsn), slot),
                                  (int)bcast<L>((uint32_t)__double2loint(rsn), slot));
        }
        // the old pool's last flat value (section 4)
        const double xstar = (double)lds[(NC - 1) * N + (N - 1)];
        float V[NC][T];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const uint32_t wd = bcast<L>(words[k], slot);
            const uint32_t a4 = wd & 0xFFFFu, b4 = wd >> 16;
            const char *src = reinterpret_cast<const char *>(lds + k * N);
            // 4 ((a j + b) mod N) for j = l + L i: x0 + 4 (a L i mod N)
            const uint32_t x0 = (__umul24(a4, (uint32_t)lane) + b4) & amask;
#pragma unroll
            for (int i = 0; i < T; ++i) {
                const uint32_t d4 = (a4 * (uint32_t)(L * i)) & amask;  // wave-uniform
                V[k][i] = *reinterpret_cast<const float *>(src + ((x0 + d4) & amask));
            }
        }
        ++slot;

        if constexpr (SPLIT) {
#pragma unroll
            for (int i = 0; i < T; ++i) {
                float v[NC];
#pragma unroll
                for (int k = 0; k < NC; ++k) v[k] = V[k][i];
                if constexpr (NC == 4)
                    xform4(v, MAT, 1.0f);
                else
                    xform16(v, signs, 1.0f);
#pragma unroll
                for (int k = 0; k < NC; ++k) V[k][i] = v[k];
            }
        }
        if constexpr (MW) {
            // every gather of the old image is done, and every wave's node of
            // the old pool's sum of squares is in the cross-wave area
            if (pending) pool_sumsq_put<NC>(pend, lane, xw);
            group_sync<MW>();
            if (pending) sigma = pool_sumsq_join<NC, T, L, RM, 1>(lane, xw);
        }

        const double c64 = chi2_scale64(xstar, sigma, P.r_nu);
        const float c32 = (float)c64;
        if (!__builtin_isfinite(c32)) flags |= WALLACE_FLAG_NONFINITE;
        const float h = c32 * (NC == 4 ? 0.5f : 0.25f);
        const float rp = NC == 2 ? (float)(c64 * cs) : 0.0f;
        const float rq = NC == 2 ? (float)(c64 * sn) : 0.0f;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            float v[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) v[k] = V[k][i];
            if constexpr (SPLIT) {
#pragma unroll
                for (int k = 0; k < NC; ++k) v[k] = v[k] * h;
            } else if constexpr (NC == 4) {
                xform4(v, MAT, h);
            } else if constexpr (NC == 2) {
                xform2(v, rp, rq);
            } else {
                xform16(v, signs, h);
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) V[k][i] = v[k];
        }

        if constexpr (!MW) group_sync<MW>();  // every gather of the old image is done
#pragma unroll
        for (int k = 0; k < NC; ++k) {
#pragma unroll
            for (int i = 0; i < T; ++i) lds[k * N + lane + L * i] = V[k][i];
        }
        group_sync<MW>();
        bool slow = false;  // the returned pool needs element-wise emission
        float *base = nullptr;
        uint32_t cnt = 0;
        if (++fcount == P.f) {  // a returned pool (section 6)
            fcount = 0;
            const bool last = (ps + 1 == passes);
            cnt = last ? job.last_emit : P.emit_len;
            base = P.out + job.out_off + (uint64_t)emitted * P.emit_len;
            ++emitted;
            constexpr uintptr_t vmask = (uintptr_t)(4 * (T >= 4 ? 4 : T) - 1);
            if (cnt == nu && ((uintptr_t)base & vmask) == 0 && !P.affine) {
                if constexpr (T > 4) {
                    // 16-byte chunks c = lane + L*s straight from the image:
                    // one store instruction of a wave covers 1 KB of
                    // consecutive output (T consecutive values per lane
                    // would leave each store instruction lane-strided)
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
#pragma unroll
                        for (int q = 0; q < T / 4; ++q) {
                            const int c = k * (N / 4) + lane + L * q;
                            __builtin_nontemporal_store(reinterpret_cast<const v4f *>(lds)[c],
                                                        reinterpret_cast<v4f *>(base) + c);
                        }
                    }
                }
            } else {
                slow = true;
            }
        }
        float Z[NC][T];  // the new pool, T consecutive tuples per lane
#pragma unroll
        for (int k = 0; k < NC; ++k) load_run<T>(Z[k], lds + k * N + T * lane);
        if (base) {
            if (slow)
                emit_slow<NC, T, N>(Z, base, cnt, lane, P.affine, P.mu, P.sigma_out);
            else if constexpr (T <= 4) {
#pragma unroll
                for (int k = 0; k < NC; ++k) store_run<T, true>(base + k * N + T * lane, Z[k]);
            }
        }
        if constexpr (MW) {
            pend = pool_sumsq_node<NC, T, L, RM, 1>(Z, lane);
            pending = true;
        } else {
            sigma = sumsq(Z, std::true_type());
        }
    };

    using M0 = std::integral_constant<int, 0>;
    using M1 = std::integral_constant<int, NC == 4 ? 1 : 0>;
    const bool odd = NC == 4 && (done & 1u);
    for (uint32_t c0 = 0; c0 < passes; c0 += (uint32_t)CH) {
        const uint32_t end = passes - c0 < (uint32_t)CH ? passes : c0 + (uint32_t)CH;
        draw_chunk(c0);
        uint32_t ps = c0;
        if (odd) one_pass(ps++, M1());
        for (; ps + 2 <= end; ps += 2) {
            one_pass(ps, M0());
            one_pass(ps + 1, M1());
        }
        if (ps < end) one_pass(ps, M0());
    }

    if constexpr (MW) {
        if (pending) {  // the last pass's sum of squares
            pool_sumsq_put<NC>(pend, lane, xw);
            group_sync<MW>();
            sigma = pool_sumsq_join<NC, T, L, RM, 1>(lane, xw);
        }
    }

    // the final pool from its LDS image
    float *wpool = P.pools + job.pool_off;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        float Z[T];
        load_run<T>(Z, lds + k * N + T * lane);
        store_run<T, false>(wpool + k * N + T * lane, Z);
    }
    group_sync<MW>();  // the next job of this group reuses the LDS image
    if (lane == 0) {
        stp->rng = rng0 + (uint64_t)Draws<NC>::value * passes * kGamma;
        stp->sigma = sigma;
        stp->passes = done + passes;
        stp->flags = flags;
    }
}

// n = 16 shapes hold 16 components per tuple in registers; left alone the
// compiler gives the larger ones up to 230 VGPRs (two waves per SIMD).
// Asking for three waves per SIMD caps them at 168 without spilling the
// one-stage shapes, which measured 4% faster on the uneven batch.
template <int NC, int T, int L, int RM, int NST>
__global__ __launch_bounds__((L > 64 ? L : 256))
__attribute__((amdgpu_waves_per_eu(NC == 16 ? 3 : 1))) void k_pool(PoolArgs P)
{
    using Cf = Cfg<NC, T, L, RM, NST>;
    extern __shared__ __attribute__((aligned(16))) char lds_all[];
    const int grp = (int)threadIdx.x / L;
    const int lane = (int)threadIdx.x % L;
    float *lds = reinterpret_cast<float *>(lds_all + grp * Cf::GROUP_BYTES);
    char *xw = lds_all + Cf::GPB * Cf::GROUP_BYTES;
    const uint32_t total = gridDim.x * (uint32_t)Cf::GPB;
    uint32_t j = blockIdx.x * (uint32_t)Cf::GPB + (uint32_t)grp;
    if constexpr (Cf::UNIFORM) j = __builtin_amdgcn_readfirstlane(j);
    for (; j < P.njobs; j += total) {
        const Job job = P.jobs ? P.jobs[j] : P.one;
        if constexpr (Cf::LDSRES)
            run_job_lds<NC, T, L, RM>(P, job, lds, xw, lane);
        else
            run_job<NC, T, L, RM, NST>(P, job, lds, xw, lane);
    }
}

// Shapes instantiated for each (n, reduction mode): single-wave groups
// (L <= 64) keep all components on chip; multi-wave groups use one stage,
// or two when the n*N floats exceed 128 KiB.
#define WALLACE_POOL_SHAPES_4(X)                                                         \
    X(4, 1, 4, 1) X(4, 1, 8, 1) X(4, 1, 16, 1) X(4, 1, 32, 1) X(4, 1, 64, 1)             \
    X(4, 2, 4, 1) X(4, 2, 8, 1) X(4, 2, 16, 1) X(4, 2, 32, 1) X(4, 2, 64, 1)             \
    X(4, 4, 4, 1) X(4, 4, 8, 1) X(4, 4, 16, 1) X(4, 4, 32, 1) X(4, 4, 64, 1)             \
    X(4, 8, 4, 1) X(4, 8, 8, 1) X(4, 8, 16, 1) X(4, 8, 32, 1) X(4, 8, 64, 1)             \
    X(4, 16, 4, 1) X(4, 16, 8, 1) X(4, 16, 16, 1) X(4, 16, 32, 1) X(4, 16, 64, 1)        \
    X(4, 1, 128, 1) X(4, 1, 256, 1) X(4, 1, 512, 1) X(4, 1, 1024, 1)                     \
    X(4, 2, 128, 1) X(4, 2, 256, 1) X(4, 2, 512, 1) X(4, 2, 1024, 1)                     \
    X(4, 4, 128, 1) X(4, 4, 256, 1) X(4, 4, 512, 1) X(4, 4, 1024, 1)                     \
    X(4, 8, 128, 1) X(4, 8, 256, 1) X(4, 8, 512, 1) X(4, 8, 1024, 1)                     \
    X(4, 16, 128, 1) X(4, 16, 256, 1) X(4, 16, 512, 1) X(4, 16, 1024, 2)

#define WALLACE_POOL_SHAPES_2(X)                                                         \
    X(2, 1, 4, 1) X(2, 1, 8, 1) X(2, 1, 16, 1) X(2, 1, 32, 1) X(2, 1, 64, 1)             \
    X(2, 2, 4, 1) X(2, 2, 8, 1) X(2, 2, 16, 1) X(2, 2, 32, 1) X(2, 2, 64, 1)             \
    X(2, 4, 4, 1) X(2, 4, 8, 1) X(2, 4, 16, 1) X(2, 4, 32, 1) X(2, 4, 64, 1)             \
    X(2, 8, 4, 1) X(2, 8, 8, 1) X(2, 8, 16, 1) X(2, 8, 32, 1) X(2, 8, 64, 1)             \
    X(2, 16, 4, 1) X(2, 16, 8, 1) X(2, 16, 16, 1) X(2, 16, 32, 1) X(2, 16, 64, 1)        \
    X(2, 1, 128, 1) X(2, 1, 256, 1) X(2, 1, 512, 1) X(2, 1, 1024, 1)                     \
    X(2, 2, 128, 1) X(2, 2, 256, 1) X(2, 2, 512, 1) X(2, 2, 1024, 1)                     \
    X(2, 4, 128, 1) X(2, 4, 256, 1) X(2, 4, 512, 1) X(2, 4, 1024, 1)                     \
    X(2, 8, 128, 1) X(2, 8, 256, 1) X(2, 8, 512, 1) X(2, 8, 1024, 1)                     \
    X(2, 16, 128, 1) X(2, 16, 256, 1) X(2, 16, 512, 1) X(2, 16, 1024, 1)

#define WALLACE_POOL_SHAPES_16(X)                                                        \
    X(16, 1, 16, 1) X(16, 1, 32, 1) X(16, 1, 64, 1)                                      \
    X(16, 2, 16, 1) X(16, 2, 32, 1) X(16, 2, 64, 1)                                      \
    X(16, 4, 16, 1) X(16, 4, 32, 1) X(16, 4, 64, 1)                                      \
    X(16, 1, 128, 1) X(16, 1, 256, 1) X(16, 1, 512, 1) X(16, 1, 1024, 1)                 \
    X(16, 2, 128, 1) X(16, 2, 256, 1) X(16, 2, 512, 1) X(16, 2, 1024, 1)                 \
    X(16, 4, 128, 1) X(16, 4, 256, 1) X(16, 4, 512, 1) X(16, 4, 1024, 2)

// Entry of the kernel table: shape and kernel address.
struct PoolEntry {
    int n, T, L, nst;
    const void *fn;
    int lds_bytes, block;
};

}  // namespace pool
}  // namespace wallace
