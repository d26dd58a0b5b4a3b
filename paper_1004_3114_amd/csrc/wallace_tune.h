// Autotuner of pool-resident schedules (lanes per pool, tuples per lane,
// components per on-chip stage) for batches of generators.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "wallace.h"
#include "wallace_internal.h"

namespace wallace {

// Schedule forced for (n, N) by WALLACE_SCHED="n:N:T:L:C,..." (read at
// every call): 1 and *out set when the first entry naming (n, N) is a
// compiled shape, -1 when that entry is not, 0 when no entry names (n, N).
int forced_sched(int n, uint32_t N, Sched *out);

// The forced schedule, else the one recorded for (n, N) on this device by an
// earlier tuning run, in this process or in the cache file named by
// WALLACE_TUNE_CACHE: 1 (found), 0 (none) or -1 (forced but not compiled).
int tuned_sched(int n, uint32_t N, Sched *out);

// Scratch bytes tune_class needs for one class.
size_t tune_scratch_bytes(int n, uint32_t N);

// Every supported schedule of the class.
int candidate_scheds(int n, uint32_t N, Sched *out, int max);

// Records a tuned schedule for (n, N) on this device (process cache and the
// WALLACE_TUNE_CACHE file, if set).
void record_tuned(int n, uint32_t N, const Sched &s, double us);

// Times each candidate on copies of one generator (state + pool) placed in
// scratch and stores the fastest in *best (and in the cache).
int32_t tune_class(int n, uint32_t N, const wallace_opts &opts, const GenState *d_state,
                   const float *d_pool, char *d_scratch, uint32_t class_size, int cus,
                   hipStream_t s, Sched *best);

}  // namespace wallace
