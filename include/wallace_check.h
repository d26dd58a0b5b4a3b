/*
 * wallace_check.h -- C ABI of libwallace_check.so, a companion library of
 * libwallace.so that is used only to check and to measure it (tests and the
 * benchmark). Nothing in libwallace.so calls it.
 *
 * 1. Device arithmetic checks. The bit-exactness of the generator rests on
 *    the GPU computing the chi-squared scale (Brent 1997, section 4, eq. 3)
 *    and the n = 2 rotation (section 8) with correctly rounded FP64
 *    operations. These entry points run the very device functions the pass
 *    kernels use (wallace_devmath.hpp, same compiler flags) over arrays of
 *    inputs, so a test can compare every result bit with host IEEE
 *    arithmetic.
 * 2. Store ceilings. Section 7 prices a number at one unit-stride store; on
 *    MI355X that store stream is the bound of the batched generator. These
 *    kernels write plain streams in the same patterns as the pass kernels
 *    but compute nothing, so the benchmark can report what the pattern
 *    itself allows on the GPU it runs on.
 *
 * Conventions: as in wallace.h (status codes, `stream` is a hipStream_t or
 * NULL, device pointers from hipMalloc on the current device, nothing
 * synchronises unless stated). Every entry point checks its arguments on
 * the host before enqueueing anything and returns WALLACE_EINVAL for null
 * pointers, misaligned pointers or sizes out of range.
 */
#ifndef WALLACE_CHECK_H
#define WALLACE_CHECK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Chi-squared scale of section 4 (eq. 3) for count independent inputs:
 * S[i] = (xstar[i] + r_nu[i])^2 / 2, q[i] = S[i] / sigma[i] and
 * c[i] = sqrt(q[i]), each step one FP64 operation, computed by the pass
 * kernels' device functions (c is NaN if the composed and the two-step forms
 * of those functions disagree). All arrays are device arrays of `count`
 * doubles (8-byte aligned); S and q may be NULL. count may be 0. */
int32_t wallace_check_chi2(const double *xstar, const double *sigma, const double *r_nu,
                           double *S, double *q, double *c, uint64_t count, void *stream);

/* n = 2 rotation of section 8 for count pass draws w[i] (device uint64
 * array): cs[i], sn[i] = cos and sin of the pass's angle from
 * t = tan(theta/2) by the rational formulas, as the pass kernels compute
 * them. Device arrays of `count` elements. */
int32_t wallace_check_rotation(const uint64_t *w, double *cs, double *sn, uint64_t count,
                               void *stream);

/* One-shot store stream: every thread of a grid of 256-thread blocks writes
 * one 16-byte chunk of `value`, blocks in address order, so the whole grid
 * covers out[0 .. count) once. out must be 16-byte aligned and count a
 * multiple of 1024. nontemporal != 0 uses nontemporal stores. */
int32_t wallace_check_store_oneshot(float *out, uint64_t count, float value,
                                    int32_t nontemporal, void *stream);

/* Long-lived store stream: `waves` waves (64 lanes each, 4 per block) each
 * write `chunks` chunks of 1024 floats (4 KB, one 16-byte store per lane and
 * instruction, each instruction 1 KB of consecutive memory), chunk c of wave
 * w at out + w * wave_stride + c * chunk_stride (element strides, multiples
 * of 4). Between two chunks a wave runs `spin` dependent FP32 operations per
 * lane (0: none), standing in for a pass's arithmetic. out holds out_count
 * floats (16-byte aligned); the host rejects a layout whose last chunk ends
 * beyond it. waves must be a positive multiple of 4. Chunks of different
 * waves should not overlap (the stream would still be in bounds). */
int32_t wallace_check_store_longlived(float *out, uint64_t out_count, uint32_t waves,
                                      uint32_t chunks, uint64_t wave_stride,
                                      uint64_t chunk_stride, uint32_t spin, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* WALLACE_CHECK_H */
