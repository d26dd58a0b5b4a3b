/*
 * wallace.h -- C ABI of an MI355X (gfx950) implementation of Wallace's
 * normal pseudo-random generator as described in R. P. Brent, "A fast
 * vectorised implementation of Wallace's normal random number generator"
 * (1997).
 *
 * The generator keeps a pool of nu = n*N normal variates, stored as n arrays
 * of length N. One "pass" (section 2, eq. 1) regenerates the whole pool:
 *
 *     x'_k[j] = c * sum_i A[k][i] x_i[(a_i j + b_i) mod N],   j = 0..N-1,
 *
 * with odd strides a_i and offsets b_i drawn once per pass (eq. 2, sections
 * 3 and 8), an orthogonal n x n matrix A (n = 2: RANN4's rotation by a
 * random angle theta with min(|sin|, |cos|) >= 1/2, section 8; n = 4:
 * alternately H4/2 and J/2 - I; n = 16: H16 D/4 with random column signs D),
 * and a scale c that gives the new pool a chi-squared sum of squares
 * (section 4, eq. 3).
 * The output stream is the sequence of pools, each in flat order
 * f = k*N + j (section 3).
 *
 * Every pass runs in HIP kernels on the GPU. Memory is owned by the caller:
 * the library never allocates device memory. A generator's entire mutable
 * device state lives in a caller-provided workspace that must be preserved
 * between calls (section 8: RANN4's work area). The library allocates only a
 * small host handle (freed by the matching destroy call).
 *
 * Conventions for every entry point:
 *   - returns WALLACE_OK (0) or a negative WALLACE_E* code;
 *   - argument errors are detected on the host BEFORE anything is enqueued,
 *     and leave the generator unchanged;
 *   - `stream` is a hipStream_t (NULL = the default stream); work is enqueued
 *     on it and the call returns without synchronising, unless the comment
 *     says otherwise;
 *   - device pointers must come from hipMalloc (or a caching allocator on top
 *     of it) on the current device; host pointers are plain host memory;
 *   - a handle is not re-entrant: calls on one handle must be ordered (same
 *     stream or external synchronisation). Two handles must not share a
 *     workspace.
 */
#ifndef WALLACE_H
#define WALLACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define WALLACE_OK 0
#define WALLACE_EINVAL (-1)   /* bad argument (shape, pointer, option)       */
#define WALLACE_ENOSPC (-2)   /* workspace smaller than required             */
#define WALLACE_EHIP (-3)     /* a HIP runtime call failed                   */
#define WALLACE_ECORRUPT (-4) /* workspace check failed (section 8 footnote) */
#define WALLACE_EUNSUP (-5)   /* valid but unsupported combination           */
#define WALLACE_ESTATE (-6)   /* call not valid in the handle's state        */

/* Device flag bits reported by wallace_status / wallace_batch_status. */
#define WALLACE_FLAG_CORRUPT 1u  /* sum of squares of the pool != stored value */
#define WALLACE_FLAG_NONFINITE 2u /* scale factor not finite (pool destroyed)  */

/* ---- options ----------------------------------------------------------------
 * Zero-initialise and call wallace_default_opts, then change fields. */
typedef struct wallace_opts {
    int32_t f;               /* throw-away factor f >= 1 (section 6): only the
                                pool after every f-th pass is returned          */
    int32_t a_mode;          /* 0: strides from fixed prime pairs per component
                                (section 8: alpha in {3,5}, beta in {7,11}, ...);
                                1: any odd stride (eq. 2). Either way a stride
                                reduced mod N that is 1, or equal to an earlier
                                component's while a free odd residue remains,
                                moves up by 2 mod N (distinct strides above
                                one, sections 3 and 9)                          */
    int32_t reduce_mode;     /* sum of squares (section 4): 0 = FP64 pairwise
                                tree (default), 1 = FP32 pairwise tree,
                                2 = FP32 pairwise tree with error terms        */
    int32_t transform_mode;  /* 0 = add/sub butterflies (bit-exact, default);
                                1 = matrix cores (n = 16 only, not bit-exact)   */
    int32_t withhold_driver; /* 1: do not return the pool value used to draw
                                the chi-squared sum (section 4)                 */
    int32_t check_workspace; /* 1: recompute the pool's sum of squares at the
                                start of every call and flag a mismatch (RANN4
                                uses this sum to detect a work area that the
                                caller damaged between calls, section 8)       */
    int32_t restart_passes;  /* R > 0: refill the pool by Box-Muller from the
                                generator's stream after every R passes
                                (section 5; R a multiple of f; single
                                generators only). The refill runs on the GPU
                                with its FP64 log/sin/cos, so it may differ
                                from the host's libm in the last bit of a rare
                                value; 0 = never (default)                     */
} wallace_opts;

/* Fills *opts with the defaults: f = 1, prime-pair strides, FP64 sum of
 * squares, butterflies, emit the whole pool, no workspace check. */
void wallace_default_opts(wallace_opts *opts);

/* Human-readable text for a status code (static storage). */
const char *wallace_strerror(int32_t code);

/* Text of the last HIP runtime error behind a WALLACE_EHIP return in the
 * calling thread, or of the limit behind wallace_fill_static's
 * WALLACE_ENOSPC (empty if none). Valid until the next call in the thread. */
const char *wallace_last_error(void);

/* ---- single generator ------------------------------------------------------ */

typedef struct wallace_gen wallace_gen;

/* Workspace bytes needed by one generator with n components (2, 4 or 16)
 * and N tuples (a power of two, N >= n; n = 2 needs N >= 4). opts may be
 * NULL.
 * Section 8: the pool occupies about half of the work area in RANN4; here
 * the pool needs 4*n*N bytes, plus a second pool buffer and reduction space
 * when the pool is too large to stay on chip. */
int32_t wallace_workspace_bytes(int32_t n, uint32_t N, const wallace_opts *opts,
                                size_t *bytes);

/* Creates a generator. Initial pool (section 5): n*N uniforms from splitmix64
 * seeded with `seed`, Box-Muller in FP64 on the host, rounded to FP32, copied
 * into d_workspace (256-byte aligned, >= wallace_workspace_bytes). The
 * initial pool itself is not part of the output. Synchronises `stream`
 * before returning. */
int32_t wallace_init(uint64_t seed, int32_t n, uint32_t N,
                     const wallace_opts *opts, void *d_workspace,
                     size_t workspace_bytes, void *stream, wallace_gen **out);

/* The initial pool that wallace_init uploads (section 5), computed on the
 * host into host_pool (n*N floats, flat order); *rng_after receives the
 * splitmix64 state after the n*N draws (may be NULL). Needs no GPU. */
int32_t wallace_initial_pool(uint64_t seed, int32_t n, uint32_t N,
                             float *host_pool, uint64_t *rng_after);

/* Writes the next `count` values of the generator's output stream to d_out
 * (device, 4-byte aligned, `count` floats). Any count >= 0 is allowed and
 * the output count may differ from call to call; the stream is the same
 * however it is split over calls (RANN4's interface, section 8). The position in the
 * stream (and, for pools too large for the chip, each pass's parameters)
 * advances on the host at every call, so a HIP graph that captured a call
 * does not continue the stream when replayed; wallace_fill_batched keeps
 * all state on the device and can be captured. */
int32_t wallace_fill(wallace_gen *g, float *d_out, uint64_t count, void *stream);

/* Same as wallace_fill, then the affine map out = mu + sigma*x (one FP32
 * multiply then one FP32 add) for N(mu, sigma^2) output (section 7). */
int32_t wallace_fill_normal(wallace_gen *g, float *d_out, uint64_t count,
                            float mu, float sigma, void *stream);

/* For callers that cannot allocate device memory or must not touch a
 * workspace's scratch regions (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same as wallace_fill, with
 * the call's scratch (a streamed pool's partial sums of squares, component
 * nodes and last-value slots; the sum-of-squares tree of restarts and
 * workspace checks) taken from a static device array of
 * WALLACE_STATIC_SCRATCH_BYTES bytes (4 MiB) that the library holds on
 * each GPU it runs on until the process ends, instead of from the
 * workspace. The generator's state and pools stay in its workspace. Output,
 * stream position and state are identical to wallace_fill's. Allocates
 * nothing. A generator whose scratch exceeds the array returns
 * WALLACE_ENOSPC (no supported shape needs more than about 2 MiB). Every
 * call on a GPU shares that GPU's array: calls that overlap in time on one
 * GPU (different streams, or different host threads) race and must be
 * ordered by the caller. */
#define WALLACE_STATIC_SCRATCH_BYTES (4u << 20)
int32_t wallace_fill_static(wallace_gen *g, float *d_out, uint64_t count, void *stream);

/* Reads the current pool's sum of squares (as used for the next pass's
 * scale) and the number of passes done. Synchronises `stream`. */
int32_t wallace_sumsq(wallace_gen *g, double *sigma, uint64_t *passes,
                      void *stream);

/* Copies the current pool (n*N floats, flat order) to host memory.
 * Synchronises `stream`. */
int32_t wallace_read_pool(wallace_gen *g, float *host_pool, void *stream);

/* Device flags (WALLACE_FLAG_*) accumulated since init; returns
 * WALLACE_ECORRUPT if the corruption flag is set. Synchronises `stream`. */
int32_t wallace_status(wallace_gen *g, uint32_t *flags, void *stream);

/* Frees the host handle (not the workspace). NULL is a no-op. */
int32_t wallace_destroy(wallace_gen *g);

/* ---- many independent generators --------------------------------------------
 * Section 9: independent streams need no communication after initialisation.
 * A batch holds G generators, each with its own seed, n_g and N_g, in one
 * workspace. Batched calls always run whole pools. */

typedef struct wallace_batch wallace_batch;

/* Workspace bytes for G generators with shapes n[g], N[g] (host arrays). */
int32_t wallace_batch_workspace_bytes(uint32_t G, const int32_t *n,
                                      const uint32_t *N, size_t *bytes);

/* Initialises G generators (host arrays seeds, n, N; opts may be NULL and
 * applies to all; f must be 1 and withhold_driver 0 in a batch). Box-Muller
 * runs on the host on all cores. Synchronises `stream`. */
int32_t wallace_batch_init(uint32_t G, const uint64_t *seeds, const int32_t *n,
                           const uint32_t *N, const wallace_opts *opts,
                           void *d_workspace, size_t workspace_bytes,
                           void *stream, wallace_batch **out);

/* Plans the next fills: generator g will run passes[g] passes and write
 * passes[g]*n[g]*N[g] floats starting at element offsets[g] of the d_out
 * given to wallace_fill_batched (pass-major, flat order within a pass).
 * Regions must not overlap. Host arrays. Builds the work list (largest jobs
 * first) with the schedule from the tuner (or defaults), copies it into the
 * workspace and synchronises `stream`. */
int32_t wallace_batch_plan(wallace_batch *b, const uint64_t *offsets,
                           const uint32_t *passes, void *stream);

/* Runs the planned passes for all generators. Each (n, N) class of the
 * batch is one launch of its pool-resident kernel, whose blocks take the
 * class's jobs largest first. The classes are spread over `stream` and up
 * to three side streams forked from it and joined back into it (parallel
 * branches under graph capture): classes of pools with at most 8192 values,
 * whose time is set by their longest chain of passes, run first on
 * `stream`; the others go largest first onto the least loaded side stream.
 * The side streams are the caller's (wallace_batch_set_streams) or else
 * created by the library at the first fill that needs them. Allocates no
 * memory, copies nothing from the host and never synchronises, so it can be
 * captured into a HIP graph; every call advances every generator. d_out must
 * be 16-byte aligned and hold out_len floats; out_len below the planned
 * extent (the largest offsets[g] + passes[g]*n[g]*N[g]) returns
 * WALLACE_EINVAL before anything is enqueued. */
int32_t wallace_fill_batched(wallace_batch *b, float *d_out, uint64_t out_len, void *stream);

/* Side streams for wallace_fill_batched (section 9: independent generators
 * can run side by side): count (<= 3) hipStream_t handles owned by the
 * caller, which must keep them alive while fills that use them are pending
 * and must not pass a fill's own `stream` among them. count = 0 returns to
 * streams the library creates itself (the default). With fewer side streams
 * than classes need, fills use the ones given. Host call; enqueues
 * nothing. */
int32_t wallace_batch_set_streams(wallace_batch *b, uint32_t count, void *const *streams);

/* Autotuner: for every (n, N) class in the batch, times each candidate
 * schedule (lanes per pool, components per on-chip stage) on copies of the
 * class's first generator in d_scratch (>= wallace_batch_tune_bytes), keeps
 * the fastest and records it in the tuning cache file named by the
 * environment variable WALLACE_TUNE_CACHE (if set). The generators' state is
 * not touched. All candidates give bit-identical output. Synchronises.
 * The environment variable WALLACE_SCHED="n:N:T:L:C,..." (read by every
 * wallace_batch_init and wallace_init, and by both autotuners) forces the
 * schedule of a class or of a single on-chip generator: L lanes per pool, T
 * tuples per lane (T*L = N), C components per on-chip stage. The first entry
 * naming a class must be a compiled shape, else wallace_batch_init or
 * wallace_init returns WALLACE_EINVAL; the autotuners keep a class forced
 * this way as it is. Without it a single generator spreads its pool over up
 * to 1024 lanes (its pass is a latency chain), while a batch uses one wave
 * or less per pool. */
int32_t wallace_batch_tune_bytes(wallace_batch *b, size_t *bytes);
int32_t wallace_batch_tune(wallace_batch *b, void *d_scratch,
                           size_t scratch_bytes, void *stream);

/* Autotuner on the planned fill itself (after wallace_batch_plan): for every
 * (n, N) class, runs the class's planned jobs (their pass counts and output
 * offsets) under each candidate schedule, on a copy of every generator's
 * state and pool in d_scratch (>= wallace_batch_tune_bytes), writing into
 * d_out (>= the planned extent, 16-byte aligned; its contents are
 * overwritten), and keeps the fastest for the class, as wallace_batch_tune
 * does. Each class is timed alone first. With more than one class, the
 * whole planned fill is then timed on the same copy: each class holding at
 * least 1/20 of the values tries its schedules that came within 25% of its
 * best alone, and one replaces the choice only if the whole fill gets at
 * least 0.5% faster (the classes share the GPU during a fill). The
 * generators' state is not touched, and every candidate gives the same
 * bits. Synchronises. WALLACE_ESTATE before a plan. */
int32_t wallace_batch_tune_planned(wallace_batch *b, float *d_out, uint64_t out_len,
                                   void *d_scratch, size_t scratch_bytes, void *stream);

/* Per-generator sum of squares and passes done; synchronises. */
int32_t wallace_batch_sumsq(wallace_batch *b, uint32_t g, double *sigma,
                            uint64_t *passes, void *stream);

/* The batch's (n, N) classes and their schedules (the tuner's choice, or
 * the default): *count receives the number of classes; for the first
 * min(max, count) classes, desc[7i .. 7i+6] = n, N, T (tuples per lane),
 * L (lanes per pool), C (components per on-chip stage), generators in the
 * class, blocks of its planned launch (0 before a plan). Host call. */
int32_t wallace_batch_classes(wallace_batch *b, uint32_t max, int64_t *desc, uint32_t *count);

/* OR of the device flags of all generators; synchronises. */
int32_t wallace_batch_status(wallace_batch *b, uint32_t *flags, void *stream);

/* Frees the host handle. NULL is a no-op. */
int32_t wallace_batch_destroy(wallace_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* WALLACE_H */
