// Device-wide exclusive prefix sum (see scan.h).
#include "scan.h"

namespace fspbb {

// Inclusive scan of one value per thread across a block of kScanThreads.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t a = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    const uint32_t r = sh[t];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanThreads) void scan_tile_sums_kernel(const uint32_t *__restrict__ in,
                                                                      int64_t count, uint32_t *__restrict__ sums)
{
    __shared__ uint32_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < count) v += in[base + i];
    v = block_inclusive_scan(v, sh);
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = v;
}

// Exclusive scan of the tile sums in place (one block); total -> *total.
__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(uint32_t *__restrict__ sums, int64_t nb,
                                                                 uint32_t *__restrict__ total)
{
    __shared__ uint32_t sh[kScanThreads];
    __shared__ uint32_t last;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? sums[b] : 0u;
        const uint32_t inc = block_inclusive_scan(v, sh);
        if (b < nb) sums[b] = carry + inc - v;
        if (threadIdx.x == kScanThreads - 1) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void store_u32_kernel(uint32_t *p, uint32_t v) { *p = v; }

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const uint32_t *in, uint32_t *out, int64_t count,
                                                                  const uint32_t *__restrict__ sums)
{
    __shared__ uint32_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tsum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < count ? in[base + i] : 0u;
        tsum += v[i];
    }
    const uint32_t inc = block_inclusive_scan(tsum, sh);
    uint32_t run = sums[blockIdx.x] + inc - tsum;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < count) out[base + i] = run;
        run += v[i];
    }
}

hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t count, uint32_t *total, void *scratch,
                              hipStream_t s)
{
    const int64_t nb = (count + kScanTile - 1) / kScanTile;
    uint32_t *sums = (uint32_t *)scratch;
    if (count <= 0) {
        store_u32_kernel<<<1, 1, 0, s>>>(total, 0u);
        return hipGetLastError();
    }
    scan_tile_sums_kernel<<<(unsigned)nb, kScanThreads, 0, s>>>(in, count, sums);
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(sums, nb, total);
    scan_apply_kernel<<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, count, sums);
    return hipGetLastError();
}

}  // namespace fspbb
