// Device side of the branch-and-bound step (bnb.hip), for one or many
// independent searches at once: every kernel runs on a 2-D grid whose y index
// selects a search ("request") and reads that request's arguments and scratch
// from a device table.
#pragma once

#include "fspbb_internal.h"
#include "scan.h"
#include "ws16.h"

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
    uint32_t *surv_per_parent;   // K survivor counts per parent (written, also for 0 children); may be null
    int32_t *incumbent;          // n; written when a complete child improves ub_in; may be null
    // Row indirection (best-first frontier in a slab of rows); null = direct.
    // Parent p's row is parents + pslot[p] * n.  Survivor rank r's row goes to
    // out_rows + oslot[r * oslot_step] * n (its depth and bound still go to
    // out_depth/out_lb at out_base + r).
    const int32_t *pslot;
    const int32_t *oslot;
    int64_t oslot_step;
};

// Device scratch of one search's step (children capacity C, parents capacity K).
struct StepScratch {
    uint32_t *cnt, *off;         // K
    int32_t *ujob, *upar;        // C: appended job and parent of each child
    int32_t *crow;               // C x n child rows
    int32_t *cdepth, *clb;       // C
    // Survivors of the compaction, for a step of nch children and W =
    // ceil(nch / 32): keep[t] (t < W) holds the survivor bits of children
    // 32t..32t+31, keep[W + t] the survivors of the words before t within its
    // 256-child block, and pos[b] the survivors before block b.
    uint32_t *keep, *pos;        // C
    uint32_t *nchild, *nsurv;    // device scalars
    unsigned long long *best;    // (bound << 32) | child index of the best complete child
    unsigned long long *fingerprint;
    unsigned long long *bad;     // invalid parents
    // Set when the children are bounded from their parents (kids16_bound):
    // K x n copy of the parent rows; child rows are then never written, and
    // survivor rows and the incumbent are built from it and ujob.  Null =
    // child rows in crow.  krec holds the parent records and kw the
    // children's scan inputs (see kids16.h).
    int32_t *prow;
    int32_t *krec;
    Workspace16 kw;
};

// Per-search scalars of a step.  They live in the search's entry of the
// request table: the upload that starts a step sets their initial values
// (best = (ub_in << 32) | 0xffffffff, the rest 0) and the copy back that ends
// it returns them, so no kernel initialises or gathers them.
struct StepResultDev {
    unsigned long long best, fingerprint, bad;
    uint32_t nchild, nsurv;
};

// One search in a step launch.  The kernels read the request through the
// constant (scalar) path and write the results only through the w pointers,
// which the host points at `res` of the same entry on the device.
struct StepReq {
    StepArgs a;
    StepScratch w;
    DevTables T;                 // the search's instance tables
    int64_t nchild;              // children of this step (set before the branch phase)
    int64_t reserved;
    StepResultDev res;
};

// Phase 1: validate and count children, child offsets (-> w.nchild).
hipError_t mstep_phase1(const StepReq *reqs, const ScanSeg *segs, int R, int64_t maxK, hipStream_t s);
// Branch: children's job lists and rows (nchild known in each StepReq).
hipError_t mstep_branch(const StepReq *reqs, int R, int64_t maxK, int64_t maxC, hipStream_t s);
// Branch without rows: the children's appended jobs and parents only.
hipError_t mstep_list(const StepReq *reqs, int R, int64_t maxK, int64_t maxC, hipStream_t s);
// Finish (after the children are bounded into w.clb): upper bound, keep and
// stable compaction (survivor bits and block counts, then one block per
// search scans the block counts), scatter, fingerprint, per-parent counts,
// incumbent.
// leaves_done: the leaf step was taken by the child decode (see kids16.h).
hipError_t mstep_finish(const StepReq *reqs, int R, int64_t maxK, int64_t maxC, hipStream_t s,
                        bool leaves_done = false);

}  // namespace fspbb
