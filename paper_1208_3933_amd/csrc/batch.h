// Batched bounding of many pools in one persistent launch (host/device shared).
#pragma once

#include "fspbb_internal.h"

namespace fspbb {

// Decode workspace of one pool in the 16-bit path (see bound_packed.hip).
struct Workspace16 {
    uint32_t *dec;    // G x 3 x m x 64 dwords: releases R, closing sums Tk, tails Q
    uint32_t *flg;    // G x NW x 128 dwords: unscheduled-job bits per node
    uint32_t *st;     // G*128: 1 = valid node
    int32_t *order;   // N: node index at each depth-sorted position, or null (identity)
    uint32_t *cnt;    // (n + 2) x B: per-block depth counts, then scatter offsets
};

constexpr int kBatchWaves = 16;  // waves per workgroup of the persistent scan

// One pool of a batch.  wpg = waves per 128-node group (divides 16); a work
// item stages 16 / wpg groups of the pool in LDS at once.
struct BatchPool {
    DevTables T;
    Workspace16 W;
    const int32_t *prefixes;
    const int32_t *depths;
    int32_t *out_lb;
    int64_t N, Npad;
    int32_t wpg;
    int32_t reserved;
};

// A work item: ngroups consecutive 128-node groups of one pool.
struct WorkItem {
    int32_t pool, group0, ngroups, reserved;
};

hipError_t launch_batch_decode(int MV, const BatchPool *pools, const int64_t *blk_off, const int32_t *cls_pools,
                               int ncls, int64_t nblocks, size_t lds_bytes, hipStream_t s);
hipError_t launch_batch_scan(const BatchPool *pools, const WorkItem *items, int n_items, uint32_t *counter,
                             int grid, size_t lds_bytes, hipStream_t s);
int batch_scan_blocks_per_cu(size_t lds_bytes);

// Tile schedule of the scan for an instance shape: waves per group and slots
// per scalar record batch.  Filled by the autotuner, else a rule of thumb.
struct ScanTuning {
    int waves_per_group;
    int unroll;
};
ScanTuning scan_tuning(int n, int m);
void set_scan_tuning(int n, int m, ScanTuning t);

}  // namespace fspbb
