// Device side of one branch-and-bound step (bnb.hip) and its scratch.
#pragma once

#include "fspbb_internal.h"

namespace fspbb {

// Arguments of one step.  Parents are rows of n int32 (first d entries are
// the prefix); with parents_reversed the pop order runs downward from row
// parent_top - 1 of a stack, otherwise parent p is row p.  Survivors go to
// out_rows/out_depth/out_lb at out_base + s (or out_base + S - 1 - s when
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

// Device scratch of one step (children capacity C, parents capacity K).
struct StepScratch {
    uint32_t *cnt, *off;         // K
    int32_t *ujob, *upar;        // C: appended job and parent of each child
    int32_t *crow;               // C x n child rows
    int32_t *cdepth, *clb;       // C
    uint32_t *keep, *pos;        // C
    void *scan_scratch;
    uint32_t *nchild, *nsurv;    // device scalars
    unsigned long long *best;    // (bound << 32) | child index of the best complete child
    unsigned long long *fingerprint;
    unsigned long long *bad;     // invalid parents
};

// Children counts and offsets; *w.nchild receives the total.
hipError_t step_phase1(const StepArgs &a, const StepScratch &w, hipStream_t s);
// Branch, bound, update, compact (nchild from phase 1).
hipError_t step_phase2(fsp_instance_s *I, const StepArgs &a, const StepScratch &w, int64_t nchild,
                       hipStream_t s);

}  // namespace fspbb
