// Device-wide exclusive prefix sums of uint32 counts, for one array or for
// many independent arrays ("segments") in one set of launches (three kernels:
// tile sums, scan of the tile sums, per-tile rescan with offset).  Used by the
// branch-and-bound step for child offsets and for the stable compaction of
// surviving children.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fspbb {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;                          // per thread
constexpr int kScanTile = kScanThreads * kScanItems;    // per block

// Bytes of tile-sum scratch a scan of `count` items needs.
inline size_t scan_scratch_bytes(int64_t count)
{
    const int64_t tiles = (count + kScanTile - 1) / kScanTile;
    return (size_t)(tiles + 1) * sizeof(uint32_t);
}

// One segment: out[i] = sum_{k<i} in[k] for i < count, *total = sum of all.
// in and out may alias; sums holds scan_scratch_bytes(count) bytes.
struct ScanSeg {
    const uint32_t *in;
    uint32_t *out;
    int64_t count;
    uint32_t *total;
    uint32_t *sums;
};

// Scans R segments (device array segs); max_count bounds every count.
hipError_t exclusive_scan_segments(const ScanSeg *segs, int R, int64_t max_count, hipStream_t s);

}  // namespace fspbb
