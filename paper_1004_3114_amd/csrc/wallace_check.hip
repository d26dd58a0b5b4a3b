// libwallace_check.so: kernels that check and measure the generator library
// (include/wallace_check.h). Built with the same flags as libwallace.so, so
// the FP64 scale and rotation run exactly as in the pass kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wallace.h"
#include "wallace_check.h"
#include "wallace_devmath.hpp"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_check_chi2(const double *xstar, const double *sigma,
                                                    const double *r_nu, double *S, double *q,
                                                    double *c, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        // the two steps as the streamed kernels call them, and the composed
        // form the pool-resident kernels call: all must agree
        const double s = wallace::chi2_target(xstar[i], r_nu[i]);
        const double c1 = wallace::chi2_scale_from_S(s, sigma[i]);
        const double c2 = wallace::chi2_scale64(xstar[i], sigma[i], r_nu[i]);
        if (S) S[i] = s;
        if (q) q[i] = s / sigma[i];
        // a disagreement between the two forms is reported as NaN, which no
        // host comparison accepts
        c[i] = (__double_as_longlong(c1) == __double_as_longlong(c2)) ? c1 : __builtin_nan("");
    }
}

__global__ __launch_bounds__(256) void k_check_rotation(const uint64_t *w, double *cs,
                                                        double *sn, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double a, b;
        wallace::rotation(w[i], a, b);
        cs[i] = a;
        sn[i] = b;
    }
}

// Block b writes the 4 KB at out + 1024 b: one 16-byte chunk per thread.
template <bool NT>
__global__ __launch_bounds__(256) void k_store_oneshot(float *out, float value)
{
    v4f *p = reinterpret_cast<v4f *>(out) + (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const v4f v = {value, value, value, value};
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Wave w writes its chunks one after another; each chunk is 4 store
// instructions of 1 KB (lane l stores 16 bytes at 16 l of each KB), as the
// pool kernel stores a returned 4096-value pool. `spin` dependent FP32
// multiply-adds per lane between chunks stand in for a pass's arithmetic;
// their result feeds the stored value so the compiler keeps them.
__global__ __launch_bounds__(256) void k_store_longlived(float *out, uint32_t chunks,
                                                         uint64_t wave_stride,
                                                         uint64_t chunk_stride, uint32_t spin)
{
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    float x = 1.0f + (float)lane * 1e-7f;
    float *base = out + (uint64_t)wave * wave_stride;
    for (uint32_t c = 0; c < chunks; ++c) {
        for (uint32_t s = 0; s < spin; ++s) x = __builtin_fmaf(x, 0.999999f, 1e-7f);
        v4f *p = reinterpret_cast<v4f *>(base + (uint64_t)c * chunk_stride) + lane;
        const v4f v = {x, x, x, x};
#pragma unroll
        for (int q = 0; q < 4; ++q) __builtin_nontemporal_store(v, p + 64 * q);
    }
}

unsigned grid_for(uint64_t count)
{
    uint64_t g = (count + 255) / 256;
    if (g > 8192) g = 8192;
    return (unsigned)(g ? g : 1);
}

}  // namespace

extern "C" {

int32_t wallace_check_chi2(const double *xstar, const double *sigma, const double *r_nu,
                           double *S, double *q, double *c, uint64_t count, void *stream)
{
    if (count == 0) return WALLACE_OK;
    if (!xstar || !sigma || !r_nu || !c) return WALLACE_EINVAL;
    hipLaunchKernelGGL(k_check_chi2, dim3(grid_for(count)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), xstar, sigma, r_nu, S, q, c, count);
    return hipGetLastError() == hipSuccess ? WALLACE_OK : WALLACE_EHIP;
}

int32_t wallace_check_rotation(const uint64_t *w, double *cs, double *sn, uint64_t count,
                               void *stream)
{
    if (count == 0) return WALLACE_OK;
    if (!w || !cs || !sn) return WALLACE_EINVAL;
    hipLaunchKernelGGL(k_check_rotation, dim3(grid_for(count)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), w, cs, sn, count);
    return hipGetLastError() == hipSuccess ? WALLACE_OK : WALLACE_EHIP;
}

int32_t wallace_check_store_oneshot(float *out, uint64_t count, float value,
                                    int32_t nontemporal, void *stream)
{
    if (!out || (((uintptr_t)out) & 15) || count == 0 || (count % 1024) != 0 ||
        count / 1024 > 0x7FFFFFFFull)
        return WALLACE_EINVAL;
    const dim3 grid((unsigned)(count / 1024));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nontemporal)
        hipLaunchKernelGGL(k_store_oneshot<true>, grid, dim3(256), 0, s, out, value);
    else
        hipLaunchKernelGGL(k_store_oneshot<false>, grid, dim3(256), 0, s, out, value);
    return hipGetLastError() == hipSuccess ? WALLACE_OK : WALLACE_EHIP;
}

int32_t wallace_check_store_longlived(float *out, uint64_t out_count, uint32_t waves,
                                      uint32_t chunks, uint64_t wave_stride,
                                      uint64_t chunk_stride, uint32_t spin, void *stream)
{
    if (!out || (((uintptr_t)out) & 15) || waves == 0 || (waves % 4) != 0 || chunks == 0 ||
        (wave_stride % 4) != 0 || (chunk_stride % 4) != 0)
        return WALLACE_EINVAL;
    // end of the last chunk of the last wave, with overflow checks
    const unsigned __int128 end = (unsigned __int128)(waves - 1) * wave_stride +
                                  (unsigned __int128)(chunks - 1) * chunk_stride + 1024u;
    if (end > (unsigned __int128)out_count) return WALLACE_EINVAL;
    hipLaunchKernelGGL(k_store_longlived, dim3(waves / 4), dim3(256), 0,
                       static_cast<hipStream_t>(stream), out, chunks, wave_stride,
                       chunk_stride, spin);
    return hipGetLastError() == hipSuccess ? WALLACE_OK : WALLACE_EHIP;
}

}  // extern "C"
