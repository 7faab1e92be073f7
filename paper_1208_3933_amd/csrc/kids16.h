// Bounding a step's children from their parents (children16.hip), for
// instances on the 16-bit path with the plain releases.
#pragma once

#include <algorithm>
#include <vector>

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

// One region holding the scratch of every search of a merged step, laid out
// anew at each step.  It grows by doubling and is kept: searches that live a
// few dozen steps would otherwise allocate on every few steps.
struct KidsArena {
    void *blob = nullptr;
    size_t cap = 0;
    // out[i] views the region for a search of instance I[i] with K[i] parents
    // and nch[i] children.
    hipError_t layout(const std::vector<const fsp_instance_s *> &I, const std::vector<int64_t> &K,
                      const std::vector<int64_t> &nch, std::vector<Kids16> &out, hipStream_t s);
    void release(hipStream_t s);
    // Bytes of one search's scratch in the region, and the region's size
    // once a layout has needed `need` bytes.
    static size_t step_bytes(const fsp_instance_s *I, int64_t K, int64_t nch);
    size_t cap_after(size_t need) const { return need > cap ? std::max(need, 2 * cap) : cap; }
};

// Whether children of this instance are bounded from their parents.
bool kids16_eligible(const fsp_instance_s *I);
// Sets the step's sizes, growing the buffers if needed (stream ordered).
hipError_t kids16_ensure(Kids16 &k, const fsp_instance_s *I, int64_t K, int64_t nch, hipStream_t s);
void kids16_release(Kids16 &k, hipStream_t s);
// Points a request's scratch at the buffers (w.prow, w.krec, w.kw); a request
// whose w.prow is null bounds its children from rows instead.
void kids16_point(StepScratch &w, const Kids16 &k);
// After mstep_list: for every request of the R in dreqs whose w.prow is set,
// decodes its parents, then its children into w.kw, and writes the children's
// depths (w.cdepth).  maxK / maxC bound the requests' parents and children;
// nmax / mmax their jobs and machines.
// With segs (the offset scan segments of every request, all of which have
// w.prow set), it replaces the step's phase 1 and list as well: the parent
// launch validates and counts the children, the segments are scanned, and
// the child launch writes each child's parent and appended job and takes the
// leaf step (mstep_finish then runs with leaves_done).
hipError_t kids16_decode(const StepReq *dreqs, int R, int64_t maxK, int64_t maxC, int nmax, int mmax, hipStream_t s,
                         const ScanSeg *segs = nullptr);
// The single search in dreq: kids16_decode, then the plain scan of its
// children, bounds to clb (its w.clb).
hipError_t kids16_bound(const StepReq *dreq, fsp_instance_s *I, Kids16 &k, int32_t *clb, hipStream_t s);

// Pair splits for a scan of N children decoded by kids16_decode (which
// zeroes each child's bound in the request's clb, so that the splits can
// combine by atomic max): more than one when N fills too few workgroups.
int scan_splits_for(const fsp_instance_s *I, int64_t N);

}  // namespace fspbb
