// Host-side state of depth-first branch-and-bound searches whose stacks live
// on the device, and the step ("tick") that advances any number of them with
// one set of launches: the step kernels run on 2-D grids (one row per
// search) and the children of all searches are bounded by one merged batched
// launch.  fsp_solve drives one search; the server drives many.
#pragma once

#include <utility>
#include <vector>

#include "batch.h"
#include "bnb.h"
#include "kids16.h"

namespace fspbb {

// Stack rows a depth-first search allocates at its start: room for a few
// pools' worth of survivors before the first doubling (each doubling copies
// the stack).
inline int64_t initial_stack_rows(int64_t pool_cap) { return pool_cap > 128 ? 8 * pool_cap : 1024; }

// Device scratch of one search's steps: the parent part (K) and the child
// part (C) grow independently, so the parent outputs survive a child resize.
struct StepBuffers {
    StepScratch w{};
    uint32_t *sums_k = nullptr;  // tile sums of the separate offset scan
    void *kblob = nullptr, *cblob = nullptr;
    int64_t Kcap = 0, Ccap = 0;
    int n = 0;
    bool rows = true;  // child rows (crow); off for instances whose children are bounded from their parents
    hipError_t ensure_k(int64_t K, hipStream_t s);
    hipError_t ensure_c(int64_t C, int n, hipStream_t s);
    void release(hipStream_t s);
    size_t bytes() const;
    static size_t bytes_for(int64_t Kcap, int64_t Ccap, int n, bool rows);
};

// Per-tick device table and its pinned host image: StepReq[R], the phase-1
// and finish scan segments, then the gathered results and survivor counts.
struct TickContext {
    hipStream_t s = nullptr;
    void *dtab = nullptr, *htab = nullptr;
    size_t dcap = 0, hcap = 0;
    BatchArena arena;
    KidsArena kids;  // the incremental scratch of a step's searches
    hipError_t reserve(size_t bytes);
    void release();
    size_t device_bytes() const;  // the request table and both arenas
};

// Bounds the children of K parents (device rows and depths, taken in order;
// each parent valid with depth < n) into B.w.clb: nch children (known to the
// caller), in parent order and then by increasing appended job.  The table
// upload goes through ctx's pinned buffer, so the caller synchronizes s
// before its next call.
hipError_t bound_children_of(fsp_instance_s *I, const int32_t *parents, const int32_t *pdepth, int64_t K,
                             int64_t nch, StepBuffers &B, Kids16 &kids, TickContext &ctx, hipStream_t s);

struct Search {
    fsp_instance_s *inst = nullptr;
    int n = 0;
    int64_t pool_cap = 0, node_budget = 0;
    int32_t UB = 0, ub0 = 0;
    std::vector<int32_t> inc;                         // host copy of the incumbent
    int32_t *srows = nullptr, *sdep = nullptr;        // stack, cap_stack rows
    int32_t *dinc = nullptr;                          // device incumbent (n)
    uint32_t *dsurv = nullptr;                        // survivors per popped parent
    int64_t cap_stack = 0;
    StepBuffers B;
    std::vector<std::pair<int32_t, int64_t>> runs;    // run-length mirror of stack depths
    std::vector<std::pair<int32_t, int64_t>> taken;   // this step's pops (depth, count)
    int64_t top = 0, nodes = 0, steps = 0, max_stack = 0;
    int32_t improvements = 0;
    int64_t *steplog = nullptr;                        // optional, 6 int64 per step
    int64_t steplog_cap = 0;
    int64_t K = 0, nch = 0, base = 0;                  // the step in flight
    bool done = false;
    fsp_status status = FSP_OK;
    // A search moved out of device memory (swap_out) keeps its live stack
    // rows here; its stack and step buffers are freed, the incumbent stays.
    bool swapped = false;
    std::vector<int32_t> host_rows, host_dep;

    // NEH or the given upper bound, device state, and the root bound.
    // Synchronous on s.
    hipError_t start(fsp_instance_s *I, int32_t ub0_in, int64_t pool_cap, int64_t node_budget, hipStream_t s);
    // The parts of start: everything but the root bound (async on s), and the
    // state once the root's bound lb0 is known.
    hipError_t begin(fsp_instance_s *I, int32_t ub0_in, int64_t pool_cap, int64_t node_budget, hipStream_t s);
    void finish_root(int32_t lb0);
    void release(hipStream_t s);
    size_t device_bytes() const;
    void result(fsp_solve_result *res, int32_t *perm_out) const;
    // Copies the live stack rows to host memory, then frees the stack and the
    // step buffers.  Synchronous on s.  The search's state is otherwise kept,
    // so its later steps are those it would have taken without the move.
    hipError_t swap_out(hipStream_t s);
    // Reallocates the stack (cap_stack rows) and pool-sized step buffers and
    // copies the rows back.  Synchronous on s; on failure the search stays
    // swapped out and holds no stack.
    hipError_t swap_in(hipStream_t s);
};

constexpr int kDevSelChunk = 1024;  // stack entries per block of the device selection

// Device-side state of a depth-first search stepped on the device
// (dsteps.hip): the host's counters and stack top, and the step in flight.
// A step whose worst case (maxC more rows) would not fit the stack's
// cap_stack rows is not started: the search pauses until the host grows the
// stack and clears `paused`.
struct DevSearch {
    int64_t top, nodes, steps, max_stack;
    int64_t node_budget, pool_cap, maxK, steplog_cap;
    int64_t K, nch, base;
    int64_t cap_stack, maxC;
    int32_t UB, improvements, done, status;
    int32_t n, paused;
};

// The two host-side parts of a step as kernels: choose the step's parents
// from the stack's top depths (writing the request's sizes and initial
// results), and account for the step once its kernels ran.  sums holds
// nchunks = ceil(maxK / 1024) words.
hipError_t launch_device_step_select(DevSearch *ds, const int32_t *sdep, int64_t *sums, int nchunks, StepReq *req,
                                     ScanSeg *seg, hipStream_t s);
hipError_t launch_device_step_update(DevSearch *ds, const StepReq *req, int64_t *steplog, hipStream_t s);

// Runs a started depth-first search (16-bit instance with the plain
// releases) to its end with steps chosen on the device, several steps per
// host synchronisation.  Synchronous on ctx.s.
hipError_t run_device_steps(Search &S, TickContext &ctx);

struct StartArgs {
    fsp_instance_s *inst;
    int32_t ub0;
    int64_t pool_cap, node_budget;
};

// Starts several searches with their root bounds in one merged launch and one
// copy back (Search::start for each, with one synchronization).
hipError_t start_many(std::vector<Search *> &ss, const std::vector<StartArgs> &args, TickContext &ctx);
// ctx.device_bytes() after start_many of these searches.
size_t start_scratch_after(const std::vector<StartArgs> &args, const TickContext &ctx);

// The parents a search's next step pops (its K parents and nch children),
// without popping them.
struct StepSel {
    int64_t K = 0, nch = 0;
};
StepSel select_step(const Search &S);
// S.device_bytes() once the step q has made room for its children.
size_t bytes_after_step(const Search &S, const StepSel &q);
// ctx.device_bytes() after a tick of these searches, whose steps are qs.
size_t tick_scratch_after(const std::vector<Search *> &sel, const std::vector<StepSel> &qs, const TickContext &ctx);

// Advances every search in `active` (not done, same device) by one step.
// Synchronous on ctx.s.  A search whose step fails gets done = true and a
// status; a returned error means the device state of all of them is lost.
hipError_t tick(std::vector<Search *> &active, TickContext &ctx);

int32_t neh(const int32_t *p, int n, int m, int32_t *perm);

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

inline fsp_status fail_status(hipError_t e)
{
    set_last_error(e);
    return e == hipErrorOutOfMemory ? FSP_E_NOMEM : FSP_E_DEVICE;
}

}  // namespace fspbb
