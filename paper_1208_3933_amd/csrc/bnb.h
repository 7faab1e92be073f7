// Device side of the branch-and-bound step (bnb.hip), for one or many
// independent searches at once: every kernel runs on a 2-D grid whose y index
// selects a search ("request") and reads that request's arguments and scratch
// from a device table.
#pragma once

#include "fspbb_internal.h"
#include "scan.h"

namespace fspbb {

// Arguments of one step of one search.  Parents are rows of n int32 (first d
// entries are the prefix); with parents_reversed the pop order runs downward
// from row parent_top - 1 of a stack, otherwise parent p is row p.  Survivors
// go to out_rows/out_depth/out_lb at out_base + s (or out_base + S - 1 - s when
// out_reversed), for s the survivor's rank in child order.
struct StepArgs {
    int n;
    int32_t ub_in;
    const int32_t *parents;
    const int32_t *pdepth;
    int64_t K;
    int parents_reversed;
    int64_t parent_top;
    int32_t *out_rows;
    int32_t *out_depth;
    int32_t *out_lb;             // may be null
    int64_t out_base, out_cap;
    int out_reversed;
    uint32_t *surv_per_parent;   // K survivor counts per parent (written); may be null
    int32_t *incumbent;          // n; written when a complete child improves ub_in; may be null
};

// Device scratch of one search's step (children capacity C, parents capacity K).
struct StepScratch {
    uint32_t *cnt, *off;         // K
    int32_t *ujob, *upar;        // C: appended job and parent of each child
    int32_t *crow;               // C x n child rows
    int32_t *cdepth, *clb;       // C
    uint32_t *keep, *pos;        // C
    uint32_t *nchild, *nsurv;    // device scalars
    unsigned long long *best;    // (bound << 32) | child index of the best complete child
    unsigned long long *fingerprint;
    unsigned long long *bad;     // invalid parents
};

// One search in a step launch.
struct StepReq {
    StepArgs a;
    StepScratch w;
    int64_t nchild;              // children of this step (set before the branch phase)
    int64_t out_slot;            // offset of this search's survivor counts in the gathered copy
};

// Per-search scalars gathered after a step (one device-to-host copy).
struct StepResultDev {
    unsigned long long best, fingerprint, bad;
    uint32_t nchild, nsurv;
};

// Phase 1: init, validate and count children, child offsets (-> w.nchild).
hipError_t mstep_phase1(const StepReq *reqs, const ScanSeg *segs, int R, int64_t maxK, hipStream_t s);
// Branch: children's job lists and rows (nchild known in each StepReq).
hipError_t mstep_branch(const StepReq *reqs, int R, int64_t maxK, int64_t maxC, hipStream_t s);
// Finish (after the children are bounded into w.clb): upper bound, keep,
// stable compaction, scatter, fingerprint, per-parent counts, incumbent,
// and the gather of the per-search results and survivor counts.
hipError_t mstep_finish(const StepReq *reqs, const ScanSeg *segs, int R, int64_t maxK, int64_t maxC,
                        StepResultDev *results, uint32_t *surv_all, hipStream_t s);

}  // namespace fspbb
