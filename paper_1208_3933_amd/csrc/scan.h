// Device-wide exclusive prefix sum of uint32 counts (three kernels: block
// sums, scan of the block sums in one block, per-block rescan with offset).
// Used by the branch-and-bound step for child offsets and for the stable
// compaction of surviving children.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fspbb {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;                          // per thread
constexpr int kScanTile = kScanThreads * kScanItems;    // per block

// Bytes of scratch exclusive_scan needs for `count` items.
inline size_t scan_scratch_bytes(int64_t count)
{
    const int64_t blocks = (count + kScanTile - 1) / kScanTile;
    return (size_t)(blocks + 1) * sizeof(uint32_t);
}

// out[i] = sum_{k<i} in[i]; *total (device) = sum of all.  in and out may alias.
// scratch holds scan_scratch_bytes(count) bytes.  Counts must sum below 2^32.
hipError_t exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t count, uint32_t *total,
                              void *scratch, hipStream_t s);

}  // namespace fspbb
