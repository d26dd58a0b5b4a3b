// Host runtime of the Wallace generator library: argument checks, workspace
// layout, initial pools (Box-Muller on the host, section 5), planning of
// pool-resident jobs and launches. Every pass runs in the HIP kernels of
// wallace_kernels.hip / wallace_stream.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "wallace.h"
#include "wallace_internal.h"
#include "wallace_runtime.h"
#include "wallace_tune.h"

using namespace wallace;

// ---------------------------------------------------------------------------
// Shared helpers
// ---------------------------------------------------------------------------

namespace wallace {

uint64_t host_splitmix_next(uint64_t &s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Box-Muller on consecutive pairs of uniforms: u1 in (0, 1] (so log is
// finite), u2 in [0, 1); the cosine goes to the even flat index and the sine
// to the odd one; FP64 then rounded to FP32.
void host_box_muller(uint64_t seed, size_t nu, float *pool, uint64_t *rng_after)
{
    uint64_t s = seed;
    const double two_pi = 0x1.921fb54442d18p+2;
    for (size_t m = 0; m + 1 < nu; m += 2) {
        const uint64_t w1 = host_splitmix_next(s);
        const uint64_t w2 = host_splitmix_next(s);
        const double u1 = (double)((w1 >> 11) + 1) * 0x1p-53;
        const double u2 = (double)(w2 >> 11) * 0x1p-53;
        const double rho = std::sqrt(-2.0 * std::log(u1));
        const double theta = two_pi * u2;
        pool[m] = (float)(rho * std::cos(theta));
        pool[m + 1] = (float)(rho * std::sin(theta));
    }
    if (rng_after) *rng_after = s;
}

static thread_local char g_last_error[256];

int32_t hip_fail(hipError_t e, const char *where)
{
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where,
                  hipGetErrorString(e), (int)e);
    return WALLACE_EHIP;
}

void record_error(const char *what)
{
    std::snprintf(g_last_error, sizeof(g_last_error), "%s", what);
}

const char *last_error_text() { return g_last_error; }

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

int ilog2(uint64_t x)
{
    int l = 0;
    while ((1ull << l) < x) ++l;
    return l;
}

bool shape_ok(int n, uint32_t N)
{
    if (n != 2 && n != 4 && n != 16) return false;
    if (!pow2(N) || N < (uint32_t)n) return false;
    if ((uint64_t)n * N > (1ull << 31)) return false;
    return true;
}

// Default pool-resident schedule for (n, N): a wave (64 lanes) per pool when
// that gives a supported tuples-per-lane count, fewer lanes for small pools,
// more (up to 1024) for large ones; all components on chip at once when they
// fit in 128 KiB of LDS, else half of them per stage.
bool default_sched(int n, uint32_t N, Sched *out)
{
    const int tmax = n == 16 ? 4 : 16;
    Sched s{n, 1, 64, n};
    if (N <= 64) {
        s.L = (int)N;
        s.T = 1;
    } else if (N / 64 <= (uint32_t)tmax) {
        s.L = 64;
        s.T = (int)(N / 64);
    } else {
        s.T = tmax;
        s.L = (int)(N / (uint32_t)tmax);
    }
    if (s.L < n || s.L > 1024) return false;
    while (s.C > 1 && (size_t)s.C * N * sizeof(float) > 128 * 1024) s.C /= 2;
    if (!pool_sched_supported(s, (int)N)) return false;
    *out = s;
    return true;
}

// One generator alone on the GPU: the pass is a latency chain, so the pool
// is spread over more lanes than in a batch (where single-wave groups keep
// the chip busy with many pools): up to 512 lanes for n = 4 and 256 for
// n = 2 and 16, with at most 8 tuples per lane (4 for n = 16) and at most
// 1024 lanes. Measured per pass against every compiled shape for n = 2, 4,
// 16 and N = 64 .. 16384, this is the fastest or within 5% of it; for
// example n = 4, N = 1024: 1.02 us (16 tuples per lane on 64 lanes: 1.9 us);
// n = 16, N = 2048: 5.1 us (2 tuples on 1024 lanes: 5.8 us).
bool single_sched(int n, uint32_t N, Sched *out)
{
    const uint32_t tcap = n == 16 ? 4u : 8u;
    const uint32_t lmax = n == 4 ? 512u : 256u;
    Sched s{n, 1, 0, n};
    uint32_t T = N > lmax ? N / lmax : 1;
    if (T > tcap) T = tcap;
    while (N / T > 1024) T *= 2;
    if (T > 16 || (n == 16 && T > 4) || N % T) return false;
    s.T = (int)T;
    s.L = (int)(N / T);
    if (s.L < n) return false;
    while (s.C > 1 && (size_t)s.C * N * sizeof(float) > 128 * 1024) s.C /= 2;
    if (!pool_sched_supported(s, (int)N)) return false;
    *out = s;
    return true;
}

hipError_t num_cus(int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    return hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}

double chi2_root(uint64_t nu) { return std::sqrt((double)(2 * nu - 1)); }

uint64_t pass_rng(const wallace_gen *g, uint64_t q)
{
    const uint64_t draws = g->n == 2 ? 3u : (uint64_t)g->n;
    const uint64_t R = (uint64_t)g->opts.restart_passes;
    const uint64_t refills = R ? q / R : 0;
    return g->rng0 + (draws * q + g->nu * refills) * 0x9E3779B97F4A7C15ull;
}

hipError_t refill_pool(wallace_gen *g, float *pool, uint64_t q, hipStream_t s,
                       const Scratch &sc)
{
    const uint64_t r0 = pass_rng(g, q) - g->nu * 0x9E3779B97F4A7C15ull;
    hipError_t e = launch_refill(pool, g->nu, r0, g->state, s);
    if (e == hipSuccess)
        e = launch_sumsq(pool, g->nu, (uint32_t)g->opts.reduce_mode, sc.tree, g->state, 0, s);
    return e;
}

// ceil(nu/1024) + ceil(nu/1024^2) + 2 double2 nodes (launch_sumsq).
size_t sumsq_tree_bytes(uint64_t nu)
{
    const size_t blocks = (nu + 1023) / 1024;
    return (blocks + (blocks + 1023) / 1024 + 2) * 2 * sizeof(double);
}

Scratch workspace_scratch(const wallace_gen *g)
{
    Scratch sc;
    sc.partials = g->streaming ? g->ws + g->lay.partials : nullptr;
    sc.tree = reinterpret_cast<double *>(g->ws + g->lay.scratch);
    return sc;
}

size_t fill_scratch_bytes(const wallace_gen *g)
{
    size_t b = 0;
    if (g->streaming) b += align_up(stream_partials_bytes(g->n, g->N), kAlign);
    if (g->opts.restart_passes || (g->opts.check_workspace && g->streaming))
        b += align_up(sumsq_tree_bytes(g->nu), kAlign);
    return b;
}

}  // namespace wallace

// ---------------------------------------------------------------------------
// Single generator
// ---------------------------------------------------------------------------

namespace {

// Workspace of one generator: header | state | pool | (streaming: second
// pool, per-block partial sums) | reduction scratch.
Layout single_layout(int n, uint32_t N)
{
    const size_t nu = (size_t)n * N;
    Layout L{};
    size_t off = sizeof(WsHeader);
    L.state = off;
    off = align_up(off + sizeof(GenState), kAlign);
    L.pool = off;
    off = align_up(off + nu * sizeof(float), kAlign);
    Sched s;
    if (!default_sched(n, N, &s)) {  // streaming pool: ping-pong + partials
        L.pool2 = off;
        off = align_up(off + nu * sizeof(float), kAlign);
        L.partials = off;
        off = align_up(off + stream_partials_bytes(n, N), kAlign);
    }
    L.scratch = off;
    off = align_up(off + sumsq_tree_bytes(nu), kAlign);
    L.total = off;
    return L;
}

bool opts_ok(const wallace_opts &o)
{
    if (o.f < 1 || o.f > (1 << 20)) return false;
    if (o.a_mode < 0 || o.a_mode > 1) return false;
    if (o.reduce_mode < 0 || o.reduce_mode > 2) return false;
    if (o.transform_mode < 0 || o.transform_mode > 1) return false;
    if (o.withhold_driver < 0 || o.withhold_driver > 1) return false;
    if (o.check_workspace < 0 || o.check_workspace > 1) return false;
    if (o.restart_passes < 0 || (o.restart_passes % o.f) != 0) return false;
    return true;
}

}  // namespace

extern "C" {

void wallace_default_opts(wallace_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->f = 1;
}

const char *wallace_last_error(void) { return last_error_text(); }

const char *wallace_strerror(int32_t code)
{
    switch (code) {
    case WALLACE_OK: return "ok";
    case WALLACE_EINVAL: return "invalid argument";
    case WALLACE_ENOSPC: return "workspace too small";
    case WALLACE_EHIP: return "HIP runtime error";
    case WALLACE_ECORRUPT: return "workspace corrupted (sum of squares changed)";
    case WALLACE_EUNSUP: return "unsupported combination";
    case WALLACE_ESTATE: return "call not valid in this state";
    default: return "unknown error";
    }
}

int32_t wallace_workspace_bytes(int32_t n, uint32_t N, const wallace_opts *opts,
                                size_t *bytes)
{
    if (!bytes) return WALLACE_EINVAL;
    wallace_opts o;
    wallace_default_opts(&o);
    if (opts) o = *opts;
    if (!opts_ok(o) || !shape_ok(n, N)) return WALLACE_EINVAL;
    *bytes = single_layout(n, N).total;
    return WALLACE_OK;
}

int32_t wallace_initial_pool(uint64_t seed, int32_t n, uint32_t N,
                             float *host_pool, uint64_t *rng_after)
{
    if (!host_pool || !shape_ok(n, N)) return WALLACE_EINVAL;
    host_box_muller(seed, (size_t)n * N, host_pool, rng_after);
    return WALLACE_OK;
}

int32_t wallace_init(uint64_t seed, int32_t n, uint32_t N,
                     const wallace_opts *opts, void *d_workspace,
                     size_t workspace_bytes, void *stream, wallace_gen **out)
{
    if (!out || !d_workspace) return WALLACE_EINVAL;
    *out = nullptr;
    wallace_opts o;
    wallace_default_opts(&o);
    if (opts) o = *opts;
    if (!opts_ok(o) || !shape_ok(n, N)) return WALLACE_EINVAL;
    if (((uintptr_t)d_workspace) & (kAlign - 1)) return WALLACE_EINVAL;
    if (o.transform_mode == 1 && n != 16) return WALLACE_EUNSUP;
    const Layout lay = single_layout(n, N);
    if (workspace_bytes < lay.total) return WALLACE_ENOSPC;

    wallace_gen *g = new (std::nothrow) wallace_gen();
    if (!g) return WALLACE_EINVAL;
    g->n = n;
    g->N = N;
    g->nu = (uint64_t)n * N;
    g->opts = o;
    g->ws = static_cast<char *>(d_workspace);
    g->lay = lay;
    g->state = reinterpret_cast<GenState *>(g->ws + lay.state);
    g->pool = reinterpret_cast<float *>(g->ws + lay.pool);
    g->emit_len = o.withhold_driver ? g->nu - 1 : g->nu;
    g->cursor = g->emit_len;  // the initial pool is not returned
    g->streaming = !default_sched(n, N, &g->sched);
    if (!g->streaming) {
        Sched t{};
        const int forced = forced_sched(n, N, &t);  // WALLACE_SCHED
        if (forced < 0) {  // names a shape that is not compiled
            delete g;
            return WALLACE_EINVAL;
        }
        if (forced > 0 || single_sched(n, N, &t)) g->sched = t;
    }
    g->passes_host = 0;
    if ((o.transform_mode == 1 && !g->streaming) || (g->streaming && !stream_shape_ok(n, N, o.transform_mode))) {
        delete g;
        return WALLACE_EUNSUP;
    }
    g->r_nu = chi2_root(g->nu);

    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<float> host(g->nu);
    GenState st{};
    host_box_muller(seed, g->nu, host.data(), &st.rng);
    g->rng0 = st.rng;
    WsHeader hdr{};
    hdr.magic = kWsMagic;
    hdr.G = 1;
    hipError_t e = hipMemcpyAsync(g->ws, &hdr, sizeof(hdr), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->state, &st, sizeof(st), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->pool, host.data(), g->nu * sizeof(float),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_sumsq(g->pool, g->nu, (uint32_t)o.reduce_mode,
                         reinterpret_cast<double *>(g->ws + lay.scratch), g->state, 0, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "wallace_init");
    }
    *out = g;
    return WALLACE_OK;
}

}  // extern "C"

namespace wallace {

int32_t fill_with_scratch(wallace_gen *g, float *d_out, uint64_t count, uint32_t affine,
                          float mu, float sig, void *stream, const Scratch &sc)
{
    if (!g) return WALLACE_EINVAL;
    if (count == 0) return WALLACE_OK;
    if (!d_out || (((uintptr_t)d_out) & 3)) return WALLACE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t len = g->emit_len;
    const uint64_t k0 = std::min<uint64_t>(count, len - g->cursor);
    const uint64_t rem = count - k0;
    const uint64_t npools = (rem + len - 1) / len;
    const uint64_t passes = npools * (uint64_t)g->opts.f;
    if (passes > 0xFFFFFFFFull) return WALLACE_EINVAL;

    hipError_t e = hipSuccess;
    if (g->opts.check_workspace) {
        // pool-resident jobs check inside the pass kernel
        e = g->streaming ? stream_check(g, s, sc) : hipSuccess;
        if (e != hipSuccess) return hip_fail(e, "workspace check");
    }
    if (k0 > 0) {
        const float *cur = g->streaming ? stream_current_pool(g) : g->pool;
        e = launch_copy_head(d_out, cur + g->cursor, (uint32_t)k0, affine, mu, sig, s);
        if (e != hipSuccess) return hip_fail(e, "copy head");
    }
    if (rem > 0) {
        const uint64_t tail = rem - (npools - 1) * len;
        if (g->streaming) {
            e = stream_run(g, d_out + k0, (uint32_t)passes, (uint32_t)tail, affine, mu,
                           sig, s, sc);
        } else {
          // restarts split the passes into segments (multiples of f, since
          // the interval is); each segment is one launch
          const uint64_t R = (uint64_t)g->opts.restart_passes;
          const uint32_t f = (uint32_t)g->opts.f;
          for (uint64_t done = 0; done < passes && e == hipSuccess;) {
            const uint64_t q = g->passes_host + done;
            if (R && q > 0 && q % R == 0) {
                e = refill_pool(g, g->pool, q, s, sc);
                if (e != hipSuccess) break;
            }
            uint64_t seg = passes - done;
            if (R) seg = std::min<uint64_t>(seg, R - q % R);
            const bool last = done + seg == passes;
            PoolArgs a{};
            a.jobs = nullptr;
            a.one.out_off = k0 + (done / f) * len;
            a.one.pool_off = 0;
            a.one.gen = 0;
            a.one.passes = (uint32_t)seg;
            a.one.last_emit = last ? (uint32_t)tail : (uint32_t)len;
            a.one.cls = 0;
            a.njobs = 1;
            a.f = (uint32_t)g->opts.f;
            a.emit_len = (uint32_t)len;
            a.a_mode = (uint32_t)g->opts.a_mode;
            a.rmode = (uint32_t)g->opts.reduce_mode;
            a.sigma_mode = (g->opts.check_workspace && done == 0) ? 1u : 0u;
            a.affine = affine;
            a.mu = mu;
            a.sigma_out = sig;
            a.out = d_out;
            a.pools = g->pool;
            a.states = g->state;
            a.r_nu = g->r_nu;
            a.queue = nullptr;
            a.N = (int)g->N;
            a.L = g->sched.L;
            a.logL = ilog2((uint64_t)g->sched.L);
            a.C = g->sched.C;
            a.groups_per_block = g->sched.L > 64 ? 1 : 256 / g->sched.L;
            e = launch_pool(g->sched, a, 1, s);
            done += seg;
          }
        }
        if (e != hipSuccess) return hip_fail(e, "pass launch");
        g->cursor = tail;
        g->passes_host += passes;
    } else {
        g->cursor += k0;
    }
    return WALLACE_OK;
}

}  // namespace wallace

extern "C" {

int32_t wallace_fill(wallace_gen *g, float *d_out, uint64_t count, void *stream)
{
    if (!g) return WALLACE_EINVAL;
    return fill_with_scratch(g, d_out, count, 0, 0.0f, 1.0f, stream, workspace_scratch(g));
}

int32_t wallace_fill_normal(wallace_gen *g, float *d_out, uint64_t count,
                            float mu, float sigma, void *stream)
{
    if (!g) return WALLACE_EINVAL;
    return fill_with_scratch(g, d_out, count, 1, mu, sigma, stream, workspace_scratch(g));
}

int32_t wallace_sumsq(wallace_gen *g, double *sigma, uint64_t *passes, void *stream)
{
    if (!g) return WALLACE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GenState st;
    hipError_t e = hipMemcpyAsync(&st, g->state, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "wallace_sumsq");
    if (sigma) *sigma = st.sigma;
    if (passes) *passes = st.passes;
    return WALLACE_OK;
}

int32_t wallace_read_pool(wallace_gen *g, float *host_pool, void *stream)
{
    if (!g || !host_pool) return WALLACE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float *src = g->streaming ? stream_current_pool(g) : g->pool;
    hipError_t e = hipMemcpyAsync(host_pool, src, g->nu * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "wallace_read_pool");
    return WALLACE_OK;
}

int32_t wallace_status(wallace_gen *g, uint32_t *flags, void *stream)
{
    if (!g) return WALLACE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GenState st;
    hipError_t e = hipMemcpyAsync(&st, g->state, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "wallace_status");
    if (flags) *flags = st.flags;
    return (st.flags & WALLACE_FLAG_CORRUPT) ? WALLACE_ECORRUPT : WALLACE_OK;
}

int32_t wallace_destroy(wallace_gen *g)
{
    delete g;
    return WALLACE_OK;
}

}  // extern "C"

