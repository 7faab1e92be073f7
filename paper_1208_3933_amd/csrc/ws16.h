// Scan inputs of a pool in the 16-bit path: what the decode (bound_packed.hip)
// or the children's decode (children16.hip) writes and the pair scan reads.
#pragma once

#include "fspbb_internal.h"

namespace fspbb {

struct Workspace16 {
    uint32_t *dec;    // G x 3 x m x 64 dwords: releases R, closing sums Tk, tails Q
    uint32_t *flg;    // G x NW x 128 dwords: unscheduled-job bits per node
    uint32_t *st;     // G*128: 1 = valid node
    int32_t *order;   // N: node index at each depth-sorted position, or null (identity)
    uint32_t *cnt;    // (n + 2) x B: per-block depth counts, then scatter offsets
};

// Counting sort of a pool's node indices by depth (invalid depths last):
// B blocks of `chunk` nodes, per-block counts in cnt ((n + 2) x B words),
// the sorted indices in order (N).  Two launches.
void launch_depth_sort(const int32_t *depths, int64_t N, int n, int B, int64_t chunk, uint32_t *cnt, int32_t *order,
                       hipStream_t s);

// The 16-bit scan alone over a decoded workspace of N nodes (identity order
// unless W.order is set), bounds to out_lb.  splits > 1 divides the machine
// pairs of each group between that many workgroups, which combine their
// maxima into out_lb by atomic max: out_lb must then hold 0 for every valid
// node beforehand.  With Ndev, N only bounds the node count, which the
// kernel reads from Ndev on the device.
hipError_t launch_scan16(const fsp_instance_s *I, const Workspace16 &W, int64_t N, int32_t *out_lb, hipStream_t s,
                         int splits = 1, const int64_t *Ndev = nullptr);

}  // namespace fspbb
