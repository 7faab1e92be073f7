// Staging of global tables and rows into LDS with the loads batched.
#pragma once

#include <hip/hip_runtime.h>

namespace fspbb {

// Fills dst[0 .. count) (LDS) with load(e), each thread of the block issuing
// PER loads before its first store.  A loop that stores every element as it
// arrives waits one full memory latency per pass; here the block waits once
// per PER passes.  load is called with e < count only.
template <int PER, class V, class Load>
__device__ __forceinline__ void stage_lds(V *dst, int count, Load load)
{
    const int t = threadIdx.x, nt = blockDim.x;
    for (int b = 0; b < count; b += PER * nt) {
        V v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) v[k] = load(min(b + k * nt + t, count - 1));
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (b + k * nt + t < count) dst[b + k * nt + t] = v[k];
    }
}

// The same with the destination given by store(e, v): dst positions that are
// not a plain copy of the source order.
template <int PER, class V, class Load, class Store>
__device__ __forceinline__ void stage_lds_with(int count, Load load, Store store)
{
    const int t = threadIdx.x, nt = blockDim.x;
    for (int b = 0; b < count; b += PER * nt) {
        V v[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) v[k] = load(min(b + k * nt + t, count - 1));
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (b + k * nt + t < count) store(b + k * nt + t, v[k]);
    }
}

}  // namespace fspbb
