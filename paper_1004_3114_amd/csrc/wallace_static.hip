// wallace_fill_static: wallace_fill with its per-call scratch in a static
// device array instead of the caller's workspace, for callers that cannot
// allocate device memory.
//
// A fill's per-call scratch (wallace_runtime.h, Scratch) holds the streamed
// passes' partial sums of squares, component nodes and last-value slots, and
// the sum-of-squares tree of a pool in memory (restart refills, workspace
// checks). Every word of it is written before it is read within the call,
// so nothing needs clearing between calls. The largest supported shape
// needs about 2 MiB (n = 16, N = 2^22: 4096 partial nodes per component;
// a 2^26-value tree), below kStaticScratchBytes.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wallace.h"
#include "wallace_internal.h"
#include "wallace_runtime.h"

namespace {

constexpr size_t kStaticScratchBytes = WALLACE_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends. In host code this name is
// a host-side stand-in: kernels and copies only ever see the device address
// obtained below.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_mu;
char *g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device

// The current device's address of `scratch`, looked up once per device with
// that device current.
hipError_t scratch_address(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t wallace_fill_static(wallace_gen *g, float *d_out, uint64_t count, void *stream)
{
    using namespace wallace;
    if (!g) return WALLACE_EINVAL;
    const size_t need = fill_scratch_bytes(g);
    if (need > kStaticScratchBytes) {
        record_error("wallace_fill_static: the generator's per-call scratch exceeds the "
                     "static array");
        return WALLACE_ENOSPC;
    }
    char *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return hip_fail(e, "wallace_fill_static: static scratch address");
    // the workspace's regions, in the same order, carved from the array
    Scratch sc{};
    size_t off = 0;
    if (g->streaming) {
        sc.partials = base + off;
        off += align_up(stream_partials_bytes(g->n, g->N), kAlign);
    }
    sc.tree = reinterpret_cast<double *>(base + off);
    return fill_with_scratch(g, d_out, count, 0, 0.0f, 1.0f, stream, sc);
}

}  // extern "C"
