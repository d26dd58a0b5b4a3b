// Internal interfaces between the host runtime pieces of the Wallace
// generator library (single generators, streaming large pools, batches).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wallace.h"
#include "wallace_internal.h"

namespace wallace {

uint64_t host_splitmix_next(uint64_t &s);
void host_box_muller(uint64_t seed, size_t nu, float *pool, uint64_t *rng_after);
// Records the HIP error text for wallace_last_error and returns WALLACE_EHIP.
int32_t hip_fail(hipError_t e, const char *where);
// Records a non-HIP error text for wallace_last_error.
void record_error(const char *what);
bool pow2(uint64_t x);
int ilog2(uint64_t x);
bool shape_ok(int n, uint32_t N);
bool default_sched(int n, uint32_t N, Sched *out);
hipError_t num_cus(int *cus);
double chi2_root(uint64_t nu);

// Byte offsets of a single generator's workspace regions.
struct Layout {
    size_t state, pool, pool2, partials, scratch, total;
};

// Per-call scratch of a single generator's fill: the streamed passes'
// partial sums of squares, component nodes and last-value slots
// (`partials`, stream_partials_bytes), and the sum-of-squares tree of a
// pool in memory (`tree`, sumsq_tree_bytes; restarts and workspace checks).
// Nothing in it outlives a call: every word is written before it is read
// within the call. wallace_fill takes it from the workspace,
// wallace_fill_static from the library's static device array.
struct Scratch {
    char *partials;
    double *tree;
};

size_t sumsq_tree_bytes(uint64_t nu);

}  // namespace wallace

// Host handle of one generator. The device state lives in the workspace;
// the host keeps only what is decided on the host (shape, options, how much
// of the current pool has been returned, passes enqueued).
struct wallace_gen {
    int n;
    uint32_t N;
    uint64_t nu;
    wallace_opts opts;
    char *ws;
    wallace::Layout lay;
    wallace::GenState *state;
    float *pool;
    uint64_t emit_len;
    uint64_t cursor;       // values of the current returned pool already emitted
    uint64_t passes_host;  // passes enqueued since init (ping-pong parity)
    uint64_t rng0;         // splitmix64 state after the initial pool: pass q
                           // (0-based) draws from rng0 + n q gamma
    bool streaming;
    wallace::Sched sched;
    double r_nu;
};

namespace wallace {

// Splitmix64 state before pass q + 1 of a single generator (q passes done
// since init): the pass draws (n per pass, 3 for n = 2) plus nu per restart
// refill, which happens before pass q + 1 when q is a positive multiple of
// the restart interval (section 5).
uint64_t pass_rng(const wallace_gen *g, uint64_t q);

// Restart refill before pass q + 1 (q a positive multiple of the interval):
// Box-Muller into `pool`, new state rng and sum of squares.
hipError_t refill_pool(wallace_gen *g, float *pool, uint64_t q, hipStream_t s,
                       const Scratch &sc);

// The workspace's scratch regions of a generator.
Scratch workspace_scratch(const wallace_gen *g);

// Bytes of per-call scratch a fill of g can use (0 for on-chip pools without
// restarts or workspace checks).
size_t fill_scratch_bytes(const wallace_gen *g);

// wallace_fill / wallace_fill_normal with the given per-call scratch.
int32_t fill_with_scratch(wallace_gen *g, float *d_out, uint64_t count, uint32_t affine,
                          float mu, float sig, void *stream, const Scratch &sc);

// Streaming path for pools too large to stay on chip (wallace_stream.hip).
size_t stream_partials_bytes(int n, uint32_t N);
bool stream_shape_ok(int n, uint32_t N, int transform_mode);
const float *stream_current_pool(wallace_gen *g);
hipError_t stream_check(wallace_gen *g, hipStream_t s, const Scratch &sc);
hipError_t stream_run(wallace_gen *g, float *out, uint32_t passes, uint32_t last_emit,
                      uint32_t affine, float mu, float sig, hipStream_t s, const Scratch &sc);

}  // namespace wallace
