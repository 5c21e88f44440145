// sm_wave.h -- wave-level helpers for compacting rare per-lane work.
//
// A lane with a job writes it to a queue private to its wave at the position
// given by a ballot over the wave (its rank among the lanes that want one);
// the ballot and the first position are kept per round so that, after the
// queue has been evaluated by all 64 lanes, each lane finds its own results
// again.  Positions depend only on which lanes want jobs, so the evaluation
// order is deterministic.
#pragma once

#include <hip/hip_runtime.h>

namespace smk {

// One ballot round: the lanes in (hi:lo) queued one job each, from `base` on.
struct alignas(16) JobRound {
    unsigned lo, hi;
    int base, pad;
};

// Number of lanes below this one in mask m.
__device__ __forceinline__ int lane_rank(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Order the wave's LDS writes before its following LDS reads.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace smk
