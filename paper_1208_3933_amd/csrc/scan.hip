// Device-wide exclusive prefix sums over independent segments (see scan.h).
// The grid's y index selects the segment; blocks past a segment's tiles exit.
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

__global__ __launch_bounds__(kScanThreads) void seg_tile_sums_kernel(const ScanSeg *__restrict__ segs)
{
    __shared__ uint32_t sh[kScanThreads];
    const ScanSeg g = segs[blockIdx.y];
    const int64_t tiles = (g.count + kScanTile - 1) / kScanTile;
    if ((int64_t)blockIdx.x >= tiles) return;  // whole block
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < g.count) v += g.in[base + i];
    v = block_inclusive_scan(v, sh);
    if (threadIdx.x == kScanThreads - 1) g.sums[blockIdx.x] = v;
}

// One block per segment: exclusive scan of its tile sums in place; total.
__global__ __launch_bounds__(kScanThreads) void seg_sums_kernel(const ScanSeg *__restrict__ segs)
{
    __shared__ uint32_t sh[kScanThreads];
    __shared__ uint32_t last;
    const ScanSeg g = segs[blockIdx.x];
    const int64_t tiles = (g.count + kScanTile - 1) / kScanTile;
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < tiles; b0 += kScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t v = b < tiles ? g.sums[b] : 0u;
        const uint32_t inc = block_inclusive_scan(v, sh);
        if (b < tiles) g.sums[b] = carry + inc - v;
        if (threadIdx.x == kScanThreads - 1) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    if (threadIdx.x == 0) *g.total = carry;
}

__global__ __launch_bounds__(kScanThreads) void seg_apply_kernel(const ScanSeg *__restrict__ segs)
{
    __shared__ uint32_t sh[kScanThreads];
    const ScanSeg g = segs[blockIdx.y];
    const int64_t tiles = (g.count + kScanTile - 1) / kScanTile;
    if ((int64_t)blockIdx.x >= tiles) return;  // whole block
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tsum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < g.count ? g.in[base + i] : 0u;
        tsum += v[i];
    }
    const uint32_t inc = block_inclusive_scan(tsum, sh);
    uint32_t run = g.sums[blockIdx.x] + inc - tsum;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < g.count) g.out[base + i] = run;
        run += v[i];
    }
}

// Segments of at most one tile: the whole scan in one block per segment.
__global__ __launch_bounds__(kScanThreads) void seg_small_kernel(const ScanSeg *__restrict__ segs)
{
    __shared__ uint32_t sh[kScanThreads];
    const ScanSeg g = segs[blockIdx.x];
    const int64_t base = (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tsum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < g.count ? g.in[base + i] : 0u;
        tsum += v[i];
    }
    const uint32_t inc = block_inclusive_scan(tsum, sh);
    uint32_t run = inc - tsum;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < g.count) g.out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanThreads - 1) *g.total = inc;
}

hipError_t exclusive_scan_segments(const ScanSeg *segs, int R, int64_t max_count, hipStream_t s)
{
    if (R <= 0) return hipSuccess;
    if (max_count <= kScanTile) {
        seg_small_kernel<<<dim3((unsigned)R), kScanThreads, 0, s>>>(segs);
        return hipGetLastError();
    }
    const int64_t tiles = (max_count + kScanTile - 1) / kScanTile;
    if (tiles > 0) seg_tile_sums_kernel<<<dim3((unsigned)tiles, (unsigned)R), kScanThreads, 0, s>>>(segs);
    seg_sums_kernel<<<dim3((unsigned)R), kScanThreads, 0, s>>>(segs);
    if (tiles > 0) seg_apply_kernel<<<dim3((unsigned)tiles, (unsigned)R), kScanThreads, 0, s>>>(segs);
    return hipGetLastError();
}

}  // namespace fspbb
