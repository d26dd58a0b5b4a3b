// Batches of independent generators (section 9: independent streams need no
// communication after initialisation). All pools of a batch live in one
// caller-provided workspace; a planned fill runs every generator's passes in
// persistent pool-resident launches (one per (n, N) class).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <thread>
#include <utility>
#include <vector>

#include "wallace.h"
#include "wallace_internal.h"
#include "wallace_runtime.h"
#include "wallace_tune.h"

using namespace wallace;

namespace {

struct BatchLayout {
    size_t states, pools, jobs, total;
    std::vector<uint64_t> pool_off;  // element offsets, 64-float aligned
};

BatchLayout batch_layout(uint32_t G, const int32_t *n, const uint32_t *N)
{
    BatchLayout L;
    size_t off = sizeof(WsHeader);
    L.states = off;
    off = align_up(off + (size_t)G * sizeof(GenState), kAlign);
    L.pools = off;
    L.pool_off.resize(G);
    uint64_t el = 0;
    for (uint32_t g = 0; g < G; ++g) {
        L.pool_off[g] = el;
        el += align_up((size_t)n[g] * N[g], 64);
    }
    off = align_up(off + el * sizeof(float), kAlign);
    L.jobs = off;
    off = align_up(off + (size_t)G * sizeof(Job), kAlign);
    L.total = off;
    return L;
}

struct ClassInfo {
    int n;
    uint32_t N;
    Sched sched;
    std::vector<uint32_t> gens;  // generators of this class
    uint32_t job_begin = 0, job_count = 0;
    int grid = 0;
    double work = 0.0;  // values written by the planned launch (ordering only)
};

// Classes of one batch run concurrently on up to this many streams.
constexpr int kClassLanes = 4;

// Classes whose pools hold at most this many values are latency-bound: a job
// is a chain of passes over a small pool, so the class takes about as long
// as its longest chain however many CUs it gets, while writing little.
// Measured on the uneven batch: these classes first, one after another on
// one stream, beside the bandwidth-bound classes on the others, 14.6 ms
// against 15.4 ms with every class placed by its output size alone.
constexpr uint64_t kLatencyBoundNu = 8192;

}  // namespace

struct wallace_batch {
    uint32_t G;
    std::vector<int32_t> n;
    std::vector<uint32_t> N;
    wallace_opts opts;
    char *ws;
    BatchLayout lay;
    std::vector<ClassInfo> classes;
    bool planned = false;
    uint64_t extent = 0;  // floats of d_out the planned fill writes: max(offset + passes nu)
    int cus = 0;
    // streams and events that let classes of one fill run side by side: the
    // caller's (wallace_batch_set_streams), else the library's own (default
    // priority), created at the first fill that needs them
    std::vector<hipStream_t> side;
    bool own_side = true;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    ~wallace_batch()
    {
        if (own_side)
            for (hipStream_t x : side) (void)hipStreamDestroy(x);
        for (hipEvent_t x : join) (void)hipEventDestroy(x);
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace {

bool same_sched(const Sched &x, const Sched &y)
{
    return x.T == y.T && x.L == y.L && x.C == y.C;
}

hipError_t class_grid(ClassInfo &c, int cus, uint32_t rmode)
{
    int per_cu = 0;
    hipError_t e = pool_max_blocks_per_cu(c.sched, (int)c.N, rmode, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const int gpb = c.sched.L > 64 ? 1 : 256 / c.sched.L;
    // One block per gpb jobs: the dispatcher then hands out jobs in plan
    // order as blocks retire, which streams the output faster than a
    // resident grid looping over jobs. Very large classes loop (the kernel
    // strides by the grid).
    const uint64_t need = (c.job_count + (uint32_t)gpb - 1) / (uint32_t)gpb;
    const uint64_t cap = std::max<uint64_t>((uint64_t)per_cu * (uint64_t)cus, 1u << 20);
    c.grid = (int)std::max<uint64_t>(1, std::min(need, cap));
    return hipSuccess;
}

PoolArgs class_args(const wallace_batch *b, const ClassInfo &c, float *out,
                    uint32_t sigma_mode)
{
    PoolArgs a{};
    a.jobs = reinterpret_cast<const Job *>(b->ws + b->lay.jobs) + c.job_begin;
    a.njobs = c.job_count;
    a.f = 1;
    a.emit_len = (uint32_t)((uint64_t)c.n * c.N);
    a.a_mode = (uint32_t)b->opts.a_mode;
    a.rmode = (uint32_t)b->opts.reduce_mode;
    a.sigma_mode = sigma_mode;
    a.out = out;
    a.pools = reinterpret_cast<float *>(b->ws + b->lay.pools);
    a.states = reinterpret_cast<GenState *>(b->ws + b->lay.states);
    a.r_nu = chi2_root((uint64_t)c.n * c.N);
    a.N = (int)c.N;
    a.L = c.sched.L;
    a.logL = ilog2((uint64_t)c.sched.L);
    a.C = c.sched.C;
    a.groups_per_block = c.sched.L > 64 ? 1 : 256 / c.sched.L;
    return a;
}

// Uploads jobs for every class (class-major order) and sets job ranges.
hipError_t upload_jobs(wallace_batch *b, const std::vector<Job> &jobs, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(b->ws + b->lay.jobs, jobs.data(), jobs.size() * sizeof(Job),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Where a launch's generators keep their states and pools: the workspace,
// or (the autotuner's runs) a copy of that region laid out the same way.
struct StateBase {
    GenState *states = nullptr;
    float *pools = nullptr;
};

// One launch per class. Several classes are spread over up to kClassLanes
// streams (the caller's and side streams forked from it and joined back).
// Latency-bound classes run first, one after another, on the caller's
// stream; the others go largest work first onto the least loaded side
// stream (onto every stream when one kind is missing), so that the long
// chains of the small pools overlap the bandwidth-bound classes instead of
// trailing them. Under graph capture the fork and join become parallel
// branches of the graph.
hipError_t launch_classes(wallace_batch *b, float *out, uint32_t sigma_mode, hipStream_t s,
                          const StateBase *alt = nullptr)
{
    auto args = [&](const ClassInfo &c) {
        PoolArgs a = class_args(b, c, out, sigma_mode);
        if (alt) {
            a.states = alt->states;
            a.pools = alt->pools;
        }
        return a;
    };
    std::vector<const ClassInfo *> live;
    for (const ClassInfo &c : b->classes)
        if (c.job_count) live.push_back(&c);
    int nside = std::min<int>((int)live.size(), kClassLanes) - 1;
    if (!b->own_side) nside = std::min<int>(nside, (int)b->side.size());
    if (nside <= 0) {
        for (const ClassInfo *c : live) {
            hipError_t e = launch_pool(c->sched, args(*c), c->grid, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t e = hipSuccess;
    if (!b->fork) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    while (e == hipSuccess && (int)b->join.size() < nside) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->join.push_back(ev);
    }
    while (e == hipSuccess && b->own_side && (int)b->side.size() < nside) {
        hipStream_t x = nullptr;
        e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e == hipSuccess) b->side.push_back(x);
    }
    if (e != hipSuccess) return e;
    std::stable_sort(live.begin(), live.end(),
                     [](const ClassInfo *x, const ClassInfo *y) { return x->work > y->work; });
    std::vector<const ClassInfo *> small, big;
    for (const ClassInfo *c : live)
        ((uint64_t)c->n * c->N <= kLatencyBoundNu ? small : big).push_back(c);
    const bool split = !small.empty() && !big.empty();
    e = hipEventRecord(b->fork, s);
    for (int i = 0; i < nside && e == hipSuccess; ++i) e = hipStreamWaitEvent(b->side[i], b->fork, 0);
    if (split) {
        for (const ClassInfo *c : small) {
            if (e != hipSuccess) break;
            e = launch_pool(c->sched, args(*c), c->grid, s);
        }
        live = big;
    }
    std::vector<double> load((size_t)nside + 1, 0.0);
    if (split) load[0] = HUGE_VAL;  // the caller's stream holds the latency-bound classes
    for (const ClassInfo *c : live) {
        if (e != hipSuccess) break;
        const int lane = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[lane] += c->work;
        e = launch_pool(c->sched, args(*c), c->grid,
                        lane == 0 ? s : b->side[lane - 1]);
    }
    for (int i = 0; i < nside && e == hipSuccess; ++i) {
        e = hipEventRecord(b->join[i], b->side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[i], 0);
    }
    return e;
}

}  // namespace

extern "C" {

int32_t wallace_batch_workspace_bytes(uint32_t G, const int32_t *n, const uint32_t *N,
                                      size_t *bytes)
{
    if (!bytes || !n || !N || G == 0) return WALLACE_EINVAL;
    for (uint32_t g = 0; g < G; ++g) {
        Sched s;
        if (!shape_ok(n[g], N[g])) return WALLACE_EINVAL;
        if (!default_sched(n[g], N[g], &s)) return WALLACE_EUNSUP;
    }
    *bytes = batch_layout(G, n, N).total;
    return WALLACE_OK;
}

int32_t wallace_batch_init(uint32_t G, const uint64_t *seeds, const int32_t *n,
                           const uint32_t *N, const wallace_opts *opts, void *d_workspace,
                           size_t workspace_bytes, void *stream, wallace_batch **out)
{
    if (!out || !seeds || !n || !N || !d_workspace || G == 0) return WALLACE_EINVAL;
    *out = nullptr;
    wallace_opts o;
    wallace_default_opts(&o);
    if (opts) o = *opts;
    if (o.f != 1 || o.withhold_driver != 0 || o.transform_mode != 0 || o.restart_passes != 0)
        return WALLACE_EUNSUP;
    if (o.a_mode < 0 || o.a_mode > 1 || o.reduce_mode < 0 || o.reduce_mode > 2 ||
        o.check_workspace < 0 || o.check_workspace > 1)
        return WALLACE_EINVAL;
    if (((uintptr_t)d_workspace) & (kAlign - 1)) return WALLACE_EINVAL;
    size_t need = 0;
    int32_t rc = wallace_batch_workspace_bytes(G, n, N, &need);
    if (rc != WALLACE_OK) return rc;
    if (workspace_bytes < need) return WALLACE_ENOSPC;

    wallace_batch *b = new (std::nothrow) wallace_batch();
    if (!b) return WALLACE_EINVAL;
    b->G = G;
    b->n.assign(n, n + G);
    b->N.assign(N, N + G);
    b->opts = o;
    b->ws = static_cast<char *>(d_workspace);
    b->lay = batch_layout(G, n, N);
    hipError_t ec = num_cus(&b->cus);
    if (ec != hipSuccess) {
        delete b;
        return hip_fail(ec, "device query");
    }

    // classes by shape, with the tuned (or default) schedule
    std::map<std::pair<int, uint32_t>, size_t> index;
    for (uint32_t g = 0; g < G; ++g) {
        auto key = std::make_pair((int)n[g], N[g]);
        auto it = index.find(key);
        if (it == index.end()) {
            ClassInfo c;
            c.n = n[g];
            c.N = N[g];
            const int found = tuned_sched(c.n, c.N, &c.sched);
            if (found < 0) {  // WALLACE_SCHED names a shape that is not compiled
                delete b;
                return WALLACE_EINVAL;
            }
            if (found == 0) default_sched(c.n, c.N, &c.sched);
            index[key] = b->classes.size();
            b->classes.push_back(c);
            it = index.find(key);
        }
        b->classes[it->second].gens.push_back(g);
    }

    // initial pools on all host cores (section 5)
    uint64_t total_el = 0;
    for (uint32_t g = 0; g < G; ++g) total_el = std::max<uint64_t>(total_el, b->lay.pool_off[g] + (uint64_t)n[g] * N[g]);
    std::vector<float> host(total_el, 0.0f);
    std::vector<GenState> st(G);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t) {
        th.emplace_back([&, t]() {
            for (uint32_t g = t; g < G; g += nth) {
                st[g] = GenState{};
                host_box_muller(seeds[g], (size_t)n[g] * N[g], host.data() + b->lay.pool_off[g],
                                &st[g].rng);
            }
        });
    }
    for (auto &x : th) x.join();

    hipStream_t s = static_cast<hipStream_t>(stream);
    WsHeader hdr{};
    hdr.magic = kWsMagic;
    hdr.G = G;
    hipError_t e = hipMemcpyAsync(b->ws, &hdr, sizeof(hdr), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + b->lay.states, st.data(), G * sizeof(GenState),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + b->lay.pools, host.data(), total_el * sizeof(float),
                           hipMemcpyHostToDevice, s);
    // sum of squares of every initial pool, by the pass kernels' own tree
    std::vector<Job> jobs;
    jobs.reserve(G);
    for (ClassInfo &c : b->classes) {
        c.job_begin = (uint32_t)jobs.size();
        for (uint32_t g : c.gens) {
            Job j{};
            j.pool_off = b->lay.pool_off[g];
            j.gen = g;
            jobs.push_back(j);
        }
        c.job_count = (uint32_t)c.gens.size();
        c.work = (double)c.job_count * c.n * c.N;
        if (e == hipSuccess) e = class_grid(c, b->cus, (uint32_t)b->opts.reduce_mode);
    }
    if (e == hipSuccess) e = upload_jobs(b, jobs, s);
    if (e == hipSuccess) e = launch_classes(b, nullptr, 2, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "wallace_batch_init");
    }
    *out = b;
    return WALLACE_OK;
}

int32_t wallace_batch_plan(wallace_batch *b, const uint64_t *offsets, const uint32_t *passes,
                           void *stream)
{
    if (!b || !offsets || !passes) return WALLACE_EINVAL;
    // regions must not overlap
    std::vector<std::pair<uint64_t, uint64_t>> reg;
    reg.reserve(b->G);
    uint64_t extent = 0;
    for (uint32_t g = 0; g < b->G; ++g) {
        const uint64_t len = (uint64_t)passes[g] * b->n[g] * b->N[g];
        if (passes[g] && len / passes[g] != (uint64_t)b->n[g] * b->N[g]) return WALLACE_EINVAL;
        if (len && offsets[g] > UINT64_MAX - len) return WALLACE_EINVAL;
        if (len) reg.emplace_back(offsets[g], offsets[g] + len);
        if (len) extent = std::max(extent, offsets[g] + len);
    }
    std::sort(reg.begin(), reg.end());
    for (size_t i = 1; i < reg.size(); ++i)
        if (reg[i].first < reg[i - 1].second) return WALLACE_EINVAL;

    std::vector<Job> jobs;
    jobs.reserve(b->G);
    for (ClassInfo &c : b->classes) {
        c.job_begin = (uint32_t)jobs.size();
        std::vector<uint32_t> order = c.gens;
        // largest jobs first: with static round-robin assignment this keeps
        // the long chains from landing last
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t x, uint32_t y) { return passes[x] > passes[y]; });
        for (uint32_t g : order) {
            Job j{};
            j.out_off = offsets[g];
            j.pool_off = b->lay.pool_off[g];
            j.gen = g;
            j.passes = passes[g];
            j.last_emit = (uint32_t)((uint64_t)b->n[g] * b->N[g]);
            jobs.push_back(j);
        }
        c.job_count = (uint32_t)order.size();
        c.work = 0.0;
        for (uint32_t g : order) c.work += (double)passes[g] * (double)b->n[g] * b->N[g];
        hipError_t e = class_grid(c, b->cus, (uint32_t)b->opts.reduce_mode);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
    }
    hipError_t e = upload_jobs(b, jobs, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "job upload");
    b->extent = extent;
    b->planned = true;
    return WALLACE_OK;
}

int32_t wallace_fill_batched(wallace_batch *b, float *d_out, uint64_t out_len, void *stream)
{
    if (!b || !d_out || (((uintptr_t)d_out) & 15)) return WALLACE_EINVAL;
    if (!b->planned) return WALLACE_ESTATE;
    if (out_len < b->extent) return WALLACE_EINVAL;
    const uint32_t sm = b->opts.check_workspace ? 1u : 0u;
    hipError_t e = launch_classes(b, d_out, sm, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return WALLACE_OK;
}

int32_t wallace_batch_sumsq(wallace_batch *b, uint32_t g, double *sigma, uint64_t *passes,
                            void *stream)
{
    if (!b || g >= b->G) return WALLACE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GenState st;
    const GenState *src = reinterpret_cast<const GenState *>(b->ws + b->lay.states) + g;
    hipError_t e = hipMemcpyAsync(&st, src, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "wallace_batch_sumsq");
    if (sigma) *sigma = st.sigma;
    if (passes) *passes = st.passes;
    return WALLACE_OK;
}

int32_t wallace_batch_status(wallace_batch *b, uint32_t *flags, void *stream)
{
    if (!b) return WALLACE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<GenState> st(b->G);
    hipError_t e = hipMemcpyAsync(st.data(), b->ws + b->lay.states, b->G * sizeof(GenState),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "wallace_batch_status");
    uint32_t f = 0;
    for (const GenState &x : st) f |= x.flags;
    if (flags) *flags = f;
    return (f & WALLACE_FLAG_CORRUPT) ? WALLACE_ECORRUPT : WALLACE_OK;
}

int32_t wallace_batch_classes(wallace_batch *b, uint32_t max, int64_t *desc, uint32_t *count)
{
    if (!b || !count || (max && !desc)) return WALLACE_EINVAL;
    *count = (uint32_t)b->classes.size();
    const uint32_t m = std::min<uint32_t>(max, *count);
    for (uint32_t i = 0; i < m; ++i) {
        const ClassInfo &c = b->classes[i];
        int64_t *d = desc + 7 * (size_t)i;
        d[0] = c.n;
        d[1] = c.N;
        d[2] = c.sched.T;
        d[3] = c.sched.L;
        d[4] = c.sched.C;
        d[5] = (int64_t)c.gens.size();
        d[6] = b->planned ? c.grid : 0;
    }
    return WALLACE_OK;
}

int32_t wallace_batch_set_streams(wallace_batch *b, uint32_t count, void *const *streams)
{
    if (!b || count > (uint32_t)(kClassLanes - 1) || (count && !streams)) return WALLACE_EINVAL;
    for (uint32_t i = 0; i < count; ++i)
        if (!streams[i]) return WALLACE_EINVAL;
    if (b->own_side)
        for (hipStream_t x : b->side) (void)hipStreamDestroy(x);
    b->side.clear();
    for (uint32_t i = 0; i < count; ++i) b->side.push_back(static_cast<hipStream_t>(streams[i]));
    b->own_side = count == 0;
    return WALLACE_OK;
}

int32_t wallace_batch_destroy(wallace_batch *b)
{
    delete b;
    return WALLACE_OK;
}

int32_t wallace_batch_tune_bytes(wallace_batch *b, size_t *bytes)
{
    if (!b || !bytes) return WALLACE_EINVAL;
    size_t m = b->lay.jobs - b->lay.states;  // a copy of every state and pool
    for (const ClassInfo &c : b->classes) m = std::max(m, tune_scratch_bytes(c.n, c.N));
    *bytes = m;
    return WALLACE_OK;
}

int32_t wallace_batch_tune_planned(wallace_batch *b, float *d_out, uint64_t out_len,
                                   void *d_scratch, size_t scratch_bytes, void *stream)
{
    if (!b || !d_out || (((uintptr_t)d_out) & 15) || !d_scratch ||
        (((uintptr_t)d_scratch) & (kAlign - 1)))
        return WALLACE_EINVAL;
    if (!b->planned) return WALLACE_ESTATE;
    if (out_len < b->extent) return WALLACE_EINVAL;
    // the states and pools regions are contiguous in the workspace; the
    // candidates run on a copy of both, laid out the same way, so the plan's
    // job table (state index, pool offset, output offset) serves unchanged
    const size_t region = b->lay.jobs - b->lay.states;
    if (scratch_bytes < region) return WALLACE_ENOSPC;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *copy = static_cast<char *>(d_scratch);
    const uint32_t rm = (uint32_t)b->opts.reduce_mode;
    const uint32_t sm = b->opts.check_workspace ? 1u : 0u;
    const StateBase alt{reinterpret_cast<GenState *>(copy),
                        reinterpret_cast<float *>(copy + (b->lay.pools - b->lay.states))};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipError_t e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    // ms of `run` on a fresh copy of the states and pools: the fastest of
    // two timed runs after an untimed one
    auto timed = [&](auto run, float *ms) {
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipMemcpyAsync(copy, b->ws + b->lay.states, region, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipEventRecord(ev0, s);
            if (e == hipSuccess) e = run();
            if (e == hipSuccess) e = hipEventRecord(ev1, s);
            if (e == hipSuccess) e = hipEventSynchronize(ev1);
            float ts = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ts, ev0, ev1);
            if (rep > 0) *ms = (rep == 1) ? ts : std::min(*ms, ts);
        }
    };
    // Each class alone: every candidate schedule, the fastest kept.
    std::vector<std::vector<std::pair<Sched, float>>> alone(b->classes.size());
    double total_work = 0.0;
    int live = 0;
    for (size_t ci = 0; ci < b->classes.size() && e == hipSuccess; ++ci) {
        ClassInfo &c = b->classes[ci];
        if (c.job_count == 0) continue;
        total_work += c.work;
        ++live;
        Sched forced;
        if (forced_sched(c.n, c.N, &forced) > 0) continue;  // WALLACE_SCHED: kept as forced
        Sched cand[32];
        const int nc = candidate_scheds(c.n, c.N, cand, 32);
        float best_ms = 1e30f;
        int best_i = -1;
        for (int i = 0; i < nc && e == hipSuccess; ++i) {
            ClassInfo t = c;
            t.sched = cand[i];
            e = class_grid(t, b->cus, rm);
            if (e != hipSuccess) break;
            PoolArgs a = class_args(b, t, d_out, sm);
            a.states = alt.states;
            a.pools = alt.pools;
            float ms = 0.0f;
            timed([&]() { return launch_pool(t.sched, a, t.grid, s); }, &ms);
            if (e != hipSuccess) break;
            alone[ci].push_back({cand[i], ms});
            if (ms < best_ms) {
                best_ms = ms;
                best_i = i;
            }
        }
        if (e != hipSuccess || best_i < 0) break;
        c.sched = cand[best_i];
        e = class_grid(c, b->cus, rm);
        record_tuned(c.n, c.N, c.sched, best_ms * 1000.0);
    }
    // Then the whole fill. Its classes run side by side and share the GPU,
    // so a class's fastest schedule alone need not be its best in the fill.
    // Each class with at least 1/20 of the values tries the schedules that
    // came within 25% of its best alone; one replaces the current choice
    // only if the whole fill gets at least 0.5% faster.
    if (e == hipSuccess && live > 1) {
        auto fill = [&]() { return launch_classes(b, d_out, sm, s, &alt); };
        float cur_ms = 0.0f;
        timed(fill, &cur_ms);
        std::vector<size_t> order;
        for (size_t ci = 0; ci < b->classes.size(); ++ci)
            if (b->classes[ci].job_count && b->classes[ci].work >= total_work / 20.0)
                order.push_back(ci);
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            return b->classes[x].work > b->classes[y].work;
        });
        for (size_t ci : order) {
            if (e != hipSuccess) break;
            ClassInfo &c = b->classes[ci];
            float best_alone = 1e30f;
            for (const auto &pr : alone[ci]) best_alone = std::min(best_alone, pr.second);
            const Sched kept = c.sched;
            for (const auto &pr : alone[ci]) {
                if (e != hipSuccess) break;
                const Sched &cs = pr.first;
                if (same_sched(cs, c.sched) || pr.second > 1.25f * best_alone) continue;
                const Sched prev = c.sched;
                c.sched = cs;
                e = class_grid(c, b->cus, rm);
                float ms = 0.0f;
                if (e == hipSuccess) timed(fill, &ms);
                if (e == hipSuccess && ms < 0.995f * cur_ms) {
                    cur_ms = ms;
                } else if (e == hipSuccess) {
                    c.sched = prev;
                    e = class_grid(c, b->cus, rm);
                }
            }
            if (e == hipSuccess && !same_sched(c.sched, kept)) {
                for (const auto &pr : alone[ci])
                    if (same_sched(pr.first, c.sched)) record_tuned(c.n, c.N, c.sched, pr.second * 1000.0);
            }
        }
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (e != hipSuccess) return hip_fail(e, "wallace_batch_tune_planned");
    return WALLACE_OK;
}

int32_t wallace_batch_tune(wallace_batch *b, void *d_scratch, size_t scratch_bytes,
                           void *stream)
{
    if (!b || !d_scratch || (((uintptr_t)d_scratch) & (kAlign - 1))) return WALLACE_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (ClassInfo &c : b->classes) {
        Sched forced;
        if (forced_sched(c.n, c.N, &forced) > 0) continue;  // WALLACE_SCHED: kept as forced
        if (scratch_bytes < tune_scratch_bytes(c.n, c.N)) return WALLACE_ENOSPC;
        const GenState *st = reinterpret_cast<const GenState *>(b->ws + b->lay.states) + c.gens[0];
        const float *pool = reinterpret_cast<const float *>(b->ws + b->lay.pools) +
                            b->lay.pool_off[c.gens[0]];
        Sched best;
        int32_t rc = tune_class(c.n, c.N, b->opts, st, pool, static_cast<char *>(d_scratch),
                                (uint32_t)std::min<size_t>(c.gens.size(), 4096), b->cus, s, &best);
        if (rc != WALLACE_OK) return rc;
        c.sched = best;
    }
    b->planned = false;  // grids depend on the schedule: plan again
    return WALLACE_OK;
}

}  // extern "C"
