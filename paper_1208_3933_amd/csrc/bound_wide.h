// The 32-bit bound path with masks in LDS (bound_wide.hip): workspace layout
// and launchers.
#pragma once

#include "bound_common.h"
#include "ws16.h"

namespace fspbb {

constexpr int kGroupW = 64;  // nodes per scan group (one per lane)

struct WorkspaceW {
    int32_t *dec;    // G x 3 x m x 64: releases R, closing sums Tk, tails Q
    uint32_t *flg;   // G x NW x 64: unscheduled-job bits per node
    uint32_t *st;    // G*64: 1 = valid node
    int32_t *order;  // N: node at each depth-sorted position, or null (identity)
    uint32_t *cnt;   // (n + 2) x B: depth-sort counts
};

// Bytes of the workspace for N nodes (256-byte aligned sections).
size_t wide_workspace_bytes(const fsp_instance_s *I, int64_t N);

// Depth sort, decode and scan of N nodes over a caller-provided workspace of
// wide_workspace_bytes(I, N) bytes (allocates nothing when marks is false).
hipError_t launch_bound_wide_ws(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N,
                                int32_t *out_lb, hipStream_t s, bool sort_depths, void *ws, bool marks);

// The same with the workspace from the stream-ordered pool.
hipError_t launch_bound_wide(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N,
                             int32_t *out_lb, hipStream_t s, bool sort_depths = true);

}  // namespace fspbb
