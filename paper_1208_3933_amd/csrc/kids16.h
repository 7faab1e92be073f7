// Bounding a step's children from their parents (children16.hip), for
// instances on the 16-bit path with the plain releases.
#pragma once

#include "batch.h"
#include "bnb.h"

namespace fspbb {

// Per-parent record, kKidRec int32 words:
//   [kKidC, +32)   completion times of the parent's prefix on each machine
//   [kKidU, +32)   time of the parent's unscheduled jobs on each machine
//   [kKidM, +16)   the parent's unscheduled-job bits
//   [kKidQ1, +32)  least tail on each machine over the unscheduled jobs
//   [kKidJ1, +32)  the job holding it (the smallest id on ties)
//   [kKidQ2, +32)  least tail over the unscheduled jobs other than that one
constexpr int kKidC = 0, kKidU = 32, kKidM = 64, kKidQ1 = 96, kKidJ1 = 128, kKidQ2 = 160, kKidRec = 192;

// Step scratch of the incremental path: a copy of the K parent rows (the
// survivors may overwrite the parents' rows on a stack), the parent records
// and the children's scan workspace (identity order).
// The buffers only grow: a search keeps one across its steps.
struct Kids16 {
    void *blob = nullptr;
    int32_t *prow = nullptr;  // capK x n
    int32_t *rec = nullptr;   // capK x kKidRec
    Workspace16 W{};          // for capC children
    int64_t K = 0, nch = 0;   // the current step
    int64_t capK = 0, capC = 0;
    size_t bytes = 0;
    int n = 0, m = 0;
};

// Whether children of this instance are bounded from their parents.
bool kids16_eligible(const fsp_instance_s *I);
// Sets the step's sizes, growing the buffers if needed (stream ordered).
hipError_t kids16_ensure(Kids16 &k, const fsp_instance_s *I, int64_t K, int64_t nch, hipStream_t s);
void kids16_release(Kids16 &k, hipStream_t s);
// After mstep_list of the single search in dreq (whose w.prow is k.prow):
// decodes its parents, then its children into k.W, writes the children's
// depths (w.cdepth) and their bounds to clb (its w.clb).
hipError_t kids16_bound(const StepReq *dreq, fsp_instance_s *I, Kids16 &k, int32_t *clb, hipStream_t s);

}  // namespace fspbb
