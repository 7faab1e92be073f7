// Device-side accessors of a step request (included by the step kernels only).
#pragma once

#include "bnb.h"
#include "bound_common.h"

namespace fspbb {

using ReqP = cptr<StepReq>;

// The request of this block's search (blockIdx.y), read through the scalar path.
__device__ __forceinline__ ReqP req_of(const StepReq *reqs) { return as_const(reqs + blockIdx.y); }

// Row and depth of parent p (p-th in pop order).
__device__ __forceinline__ const int32_t *parent_row(ReqP q, int64_t p)
{
    const int64_t r = q->a.parents_reversed ? (q->a.parent_top - 1 - p) : p;
    const int64_t row = q->a.pslot ? (int64_t)q->a.pslot[r] : r;
    return q->a.parents + row * (int64_t)q->a.n;
}
__device__ __forceinline__ int32_t parent_depth(ReqP q, int64_t p)
{
    return q->a.pdepth[q->a.parents_reversed ? (q->a.parent_top - 1 - p) : p];
}

// One wave per parent: the lanes build the parent's scheduled set in a 16-word
// LDS mask (LDS atomics; a returned bit already set means a repeated job).
// Returns, uniformly over the wave, whether the parent is valid: depth in
// 0..n, every job in 0..n-1, no repeat.
__device__ inline bool wave_prefix_set(const int32_t *row, int d, int n, uint32_t *mask, int lane)
{
    if (lane < kMaxJobs / 32) mask[lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    bool bad = d < 0 || d > n;
    if (!bad) {
        for (int t = lane; t < d; t += 64) {
            const int j = row[t];
            if ((unsigned)j >= (unsigned)n) { bad = true; continue; }
            const uint32_t bit = 1u << (j & 31);
            if (atomicOr(&mask[j >> 5], bit) & bit) bad = true;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return __ballot(bad) == 0;
}

}  // namespace fspbb
