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

// The 16-bit scan alone over a decoded workspace of N nodes (identity order
// unless W.order is set), bounds to out_lb.
hipError_t launch_scan16(const fsp_instance_s *I, const Workspace16 &W, int64_t N, int32_t *out_lb, hipStream_t s);

}  // namespace fspbb
