// Internal layout shared by the host runtime and the HIP kernels of the
// Wallace generator library. Not part of the public C ABI (include/wallace.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace wallace {

constexpr uint32_t kWsMagic = 0x574c4c43u;  // "WLLC"
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Per-generator device state (32 bytes). Together with the pool this is all
// the mutable state of a generator (section 8: the work area preserved
// between calls).
struct GenState {
    uint64_t rng;     // splitmix64 state
    double sigma;     // sum of squares of the current pool (reduce mode's value)
    uint64_t passes;  // passes done since initialisation
    uint32_t flags;   // WALLACE_FLAG_* bits
    uint32_t pad;
};
static_assert(sizeof(GenState) == 32, "GenState layout");

// Workspace header at offset 0 (256 bytes).
struct WsHeader {
    uint32_t magic;
    uint32_t G;          // generators in this workspace
    uint32_t queue;      // dynamic work-queue cursor (self-resetting)
    uint32_t done;       // groups that found the queue empty (self-resetting)
    uint32_t stream_ctr; // arrival counter of the streaming pass (self-resetting)
    uint32_t pad[59];
};
static_assert(sizeof(WsHeader) == 256, "WsHeader layout");

// One unit of pool-resident work: run `passes` passes of one generator.
struct Job {
    uint64_t out_off;    // element offset in d_out of the first emitted value
    uint64_t pool_off;   // element offset of the pool in the pool region
    uint32_t gen;        // state slot
    uint32_t passes;     // passes to run (a multiple of f)
    uint32_t last_emit;  // values to emit from the last emitted pool
    uint32_t cls;        // schedule class index (uneven batches)
};
static_assert(sizeof(Job) == 32, "Job layout");

// Shape of one pool-resident schedule: pools of n components and N = T*L
// tuples handled by groups of L lanes, each lane owning T consecutive tuples;
// C components pass through the on-chip permutation network at a time.
struct Sched {
    int n;
    int T;
    int L;
    int C;
};

// Arguments of the pool-resident kernels.
struct PoolArgs {
    const Job *jobs;     // job list (device); NULL -> use `one`
    Job one;             // the single job of a one-generator call
    uint32_t njobs;
    uint32_t f;          // throw-away factor (section 6)
    uint32_t emit_len;   // values emitted per returned pool (nu or nu - 1)
    uint32_t a_mode;     // 0 prime pairs, 1 any odd stride
    uint32_t rmode;      // 0 FP64 tree, 1 FP32 tree, 2 compensated FP32 tree
    uint32_t sigma_mode; // 0: none; 1: recompute at job start and compare
                         // (flag on mismatch); 2: compute and store (init)
    uint32_t affine;     // apply mu + sigma_out * x on store
    float mu;
    float sigma_out;
    float *out;
    float *pools;
    GenState *states;
    double r_nu;         // RN64(sqrt(2 nu - 1)) for the chi-squared draw
    uint32_t *queue;     // dynamic queue counters (NULL: static assignment)
    int N;
    int L;
    int logL;
    int C;
    int groups_per_block;
};

// Launchers (wallace_kernels.hip).
hipError_t launch_pool(const Sched &s, const PoolArgs &a, int grid,
                       hipStream_t stream);
int pool_block_threads(const Sched &s);
size_t pool_lds_bytes(const Sched &s, int N);
bool pool_sched_supported(const Sched &s, int N);
hipError_t pool_max_blocks_per_cu(const Sched &s, int N, uint32_t rmode, int *blocks);

// Restart refill of a pool (section 5) from the stream at r0; sets state->rng.
hipError_t launch_refill(float *pool, uint64_t nu, uint64_t r0, GenState *state,
                         hipStream_t stream);
hipError_t launch_copy_head(float *out, const float *pool, uint32_t count,
                            uint32_t affine, float mu, float sig,
                            hipStream_t stream);
hipError_t launch_replicate(GenState *states, float *pools, uint64_t stride,
                            uint32_t copies, const GenState *src_state,
                            const float *src_pool, uint64_t nu, hipStream_t stream);
hipError_t launch_sumsq(const float *pool, size_t nu, uint32_t rmode, double *scratch,
                        GenState *state, uint32_t mode, hipStream_t stream);

}  // namespace wallace
