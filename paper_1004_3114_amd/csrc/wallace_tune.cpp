// Autotuner of pool-resident schedules. Candidates differ only in how a pool
// is spread over lanes and how many components pass through LDS at a time;
// the arithmetic order (and so every output bit) is the same for all of
// them, so the choice affects speed only.
#include "wallace_tune.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "wallace_runtime.h"

namespace wallace {

namespace {

constexpr uint32_t kTunePasses = 8;

std::mutex g_mu;
bool g_loaded = false;
std::map<std::tuple<std::string, int, int, uint32_t>, Sched> g_cache;

std::string device_key()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
        return "unknown";
    char buf[128];
    std::snprintf(buf, sizeof(buf), "%s-%dcu", p.gcnArchName, p.multiProcessorCount);
    for (char *c = buf; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    return buf;
}

void load_cache_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = std::getenv("WALLACE_TUNE_CACHE");
    if (!path) return;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return;
    char dev[128];
    int n, T, L, C;
    unsigned N;
    double us;
    while (std::fscanf(fp, "%127s %d %u %d %d %d %lf", dev, &n, &N, &T, &L, &C, &us) == 7) {
        Sched s{n, T, L, C};
        if (pool_sched_supported(s, (int)N)) g_cache[std::make_tuple(std::string(dev), 0, n, N)] = s;
    }
    std::fclose(fp);
}

void store_locked(int n, uint32_t N, const Sched &s, double us)
{
    const std::string dev = device_key();
    g_cache[std::make_tuple(dev, 0, n, N)] = s;
    const char *path = std::getenv("WALLACE_TUNE_CACHE");
    if (!path) return;
    FILE *fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp, "%s %d %u %d %d %d %.3f\n", dev.c_str(), n, N, s.T, s.L, s.C, us);
    std::fclose(fp);
}

uint32_t tune_copies(int n, uint32_t N, uint32_t class_size)
{
    const uint64_t nu = (uint64_t)n * N;
    uint64_t c = (1ull << 24) / nu;
    c = std::max<uint64_t>(64, std::min<uint64_t>(4096, c));
    if (class_size) c = std::min<uint64_t>(c, std::max<uint32_t>(class_size, 1u));
    return (uint32_t)c;
}

struct TuneLayout {
    size_t states, pools, jobs, out, total;
};

TuneLayout tune_layout(int n, uint32_t N, uint32_t copies)
{
    const size_t nu = (size_t)n * N;
    TuneLayout L{};
    size_t off = 0;
    L.states = off;
    off = align_up(off + copies * sizeof(GenState), kAlign);
    L.pools = off;
    off = align_up(off + (size_t)copies * align_up(nu, 64) * sizeof(float), kAlign);
    L.jobs = off;
    off = align_up(off + copies * sizeof(Job), kAlign);
    L.out = off;
    off = align_up(off + (size_t)copies * kTunePasses * nu * sizeof(float), kAlign);
    L.total = off;
    return L;
}

}  // namespace

int forced_sched(int n, uint32_t N, Sched *out)
{
    // Explicit override, read at every call: WALLACE_SCHED="n:N:T:L:C,..."
    if (const char *ov = std::getenv("WALLACE_SCHED")) {
        const char *p = ov;
        while (*p) {
            int a, c, T, L, C, used = 0;
            unsigned b;
            if (std::sscanf(p, "%d:%u:%d:%d:%d%n", &a, &b, &T, &L, &C, &used) != 5) break;
            (void)c;
            Sched s{a, T, L, C};
            if (a == n && b == N) {
                if (!pool_sched_supported(s, (int)N)) return -1;
                *out = s;
                return 1;
            }
            p += used;
            if (*p == ',') ++p;
        }
    }
    return 0;
}

void record_tuned(int n, uint32_t N, const Sched &s, double us)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    store_locked(n, N, s, us);
}

int tuned_sched(int n, uint32_t N, Sched *out)
{
    if (const int f = forced_sched(n, N, out)) return f;
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    auto it = g_cache.find(std::make_tuple(device_key(), 0, n, N));
    if (it == g_cache.end()) return 0;
    *out = it->second;
    return 1;
}

size_t tune_scratch_bytes(int n, uint32_t N)
{
    if (!shape_ok(n, N)) return 0;
    return tune_layout(n, N, tune_copies(n, N, 0)).total;
}

int candidate_scheds(int n, uint32_t N, Sched *out, int max)
{
    int cnt = 0;
    for (int T = 1; T <= 16; T *= 2) {
        if (N % (uint32_t)T) continue;
        const uint32_t L = N / (uint32_t)T;
        if (L < (uint32_t)n || L > 1024) continue;
        int taken = 0;
        for (int C = n; C >= 1 && taken < 2; C /= 2) {
            Sched s{n, T, (int)L, C};
            if (!pool_sched_supported(s, (int)N)) continue;
            if ((size_t)C * N * sizeof(float) > 128 * 1024) continue;
            if (cnt < max) out[cnt++] = s;
            ++taken;
        }
    }
    return cnt;
}

int32_t tune_class(int n, uint32_t N, const wallace_opts &opts, const GenState *d_state,
                   const float *d_pool, char *d_scratch, uint32_t class_size, int cus,
                   hipStream_t s, Sched *best)
{
    Sched cand[32];
    const int nc = candidate_scheds(n, N, cand, 32);
    if (nc == 0) return WALLACE_EUNSUP;
    const uint32_t copies = tune_copies(n, N, class_size);
    const TuneLayout lay = tune_layout(n, N, copies);
    const uint64_t nu = (uint64_t)n * N;
    const uint64_t stride = align_up(nu, 64);

    // copies of the class's first generator; jobs of kTunePasses passes
    std::vector<Job> jobs(copies);
    for (uint32_t c = 0; c < copies; ++c) {
        Job &j = jobs[c];
        j.out_off = (uint64_t)c * kTunePasses * nu;
        j.pool_off = (uint64_t)c * stride;
        j.gen = c;
        j.passes = kTunePasses;
        j.last_emit = (uint32_t)nu;
        j.cls = 0;
    }
    hipError_t e = hipMemcpyAsync(d_scratch + lay.jobs, jobs.data(), copies * sizeof(Job),
                                  hipMemcpyHostToDevice, s);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    float best_ms = 1e30f;
    int best_i = -1;
    for (int i = 0; i < nc && e == hipSuccess; ++i) {
        int per_cu = 0;
        e = pool_max_blocks_per_cu(cand[i], (int)N, (uint32_t)opts.reduce_mode, &per_cu);
        if (e != hipSuccess) break;
        const int gpb = cand[i].L > 64 ? 1 : 256 / cand[i].L;
        const int need = (int)((copies + (uint32_t)gpb - 1) / (uint32_t)gpb);
        const int grid = std::max(1, std::min(need, std::max(per_cu, 1) * cus));
        PoolArgs a{};
        a.jobs = reinterpret_cast<const Job *>(d_scratch + lay.jobs);
        a.njobs = copies;
        a.f = 1;
        a.emit_len = (uint32_t)nu;
        a.a_mode = (uint32_t)opts.a_mode;
        a.rmode = (uint32_t)opts.reduce_mode;
        a.out = reinterpret_cast<float *>(d_scratch + lay.out);
        a.pools = reinterpret_cast<float *>(d_scratch + lay.pools);
        a.states = reinterpret_cast<GenState *>(d_scratch + lay.states);
        a.r_nu = chi2_root(nu);
        a.N = (int)N;
        a.L = cand[i].L;
        a.logL = ilog2((uint64_t)cand[i].L);
        a.C = cand[i].C;
        a.groups_per_block = gpb;
        float ms = 0.0f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            // reset every copy to the source generator's state and pool
            e = launch_replicate(reinterpret_cast<GenState *>(d_scratch + lay.states),
                                 reinterpret_cast<float *>(d_scratch + lay.pools), stride,
                                 copies, d_state, d_pool, nu, s);
            if (e == hipSuccess) e = hipEventRecord(ev0, s);
            if (e == hipSuccess) e = launch_pool(cand[i], a, grid, s);
            if (e == hipSuccess) e = hipEventRecord(ev1, s);
            if (e == hipSuccess) e = hipEventSynchronize(ev1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, ev0, ev1);
            if (rep > 0) ms = (rep == 1) ? t : std::min(ms, t);
        }
        if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best_i = i;
        }
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    if (e != hipSuccess) return hip_fail(e, "tuning run");
    *best = cand[best_i];
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    store_locked(n, N, *best, best_ms * 1000.0);
    return WALLACE_OK;
}

}  // namespace wallace
