// Depth-first steps chosen and accounted for on the device, so that a search
// runs several steps per host synchronisation (FSP_SOLVE_DEVICE_STEPS).
//
// A host-driven step takes one round trip: the host pops parents from its
// run-length view of the stack, uploads the step's sizes, and reads the
// survivor counts back to update that view.  Here two small kernels take the
// host's part:
//   select  the parents of the step under the rule of the host-driven search
//           (pop from the top while the children so far plus the next
//           parent's n - d fit in pool_cap; the first parent always), from the
//           depths at the top of the device stack: per-chunk child sums of up
//           to pool_cap entries, then one block finds the cut;
//   update  after the step's kernels: nodes, the upper bound, improvements,
//           the stack top (base + survivors), the step log and the stop rule
//           (empty stack: proven; nodes >= budget: stopped).
// The step's own kernels (children from parents, the pair scan, the
// compaction) read every size from the request table and run on grids sized
// for pool_cap children, so a stopped search's later steps are empty.  The
// results, node counts and step log are those of the host-driven search.
#include <algorithm>
#include <cstring>

#include "search.h"

namespace fspbb {

namespace {

constexpr int kSelThreads = kDevSelChunk;

// Block-wide inclusive scan of one value per thread (1,024 threads: 16
// waves): a scan within each wave by lane shuffles, then each wave adds the
// totals of the waves before it.  sh: at least 16 words.
__device__ int64_t block_scan_incl(int64_t v, int64_t *sh)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) sh[w] = v;
    __syncthreads();
    int64_t before = 0;
    for (int k = 0; k < w; ++k) before += sh[k];
    __syncthreads();  // sh is free again when the call returns
    return v + before;
}

// Children of stack entry i counted from the top (i = 0 is the top), or 0 past
// the stack or past maxK entries.
__device__ __forceinline__ int64_t kids_from_top(const DevSearch *ds, const int32_t *sdep, int64_t i)
{
    const int64_t idx = ds->top - 1 - i;
    return (i < ds->maxK && idx >= 0) ? (int64_t)(ds->n - sdep[idx]) : 0;
}

// No step runs: the search ended, or the stack has no room for the next
// step's worst case.
__device__ __forceinline__ bool idle(const DevSearch *ds) { return ds->done || ds->paused; }

__global__ __launch_bounds__(kSelThreads) void dsel_sums_kernel(const DevSearch *__restrict__ ds,
                                                                const int32_t *__restrict__ sdep,
                                                                int64_t *__restrict__ sums)
{
    __shared__ int64_t sh[kSelThreads];
    const int64_t i = (int64_t)blockIdx.x * kSelThreads + threadIdx.x;
    const int64_t v = idle(ds) ? 0 : kids_from_top(ds, sdep, i);
    const int64_t tot = block_scan_incl(v, sh);
    if (threadIdx.x == kSelThreads - 1) sums[blockIdx.x] = tot;
}

// One block: the step's parents K and children nch, and the request's sizes
// and initial results.  Pauses the search first when the stack has no room
// for the step's worst case.
__global__ __launch_bounds__(kSelThreads) void dsel_finish_kernel(DevSearch *__restrict__ ds,
                                                                  const int32_t *__restrict__ sdep,
                                                                  const int64_t *__restrict__ sums, int nchunks,
                                                                  StepReq *__restrict__ req, ScanSeg *__restrict__ seg)
{
    __shared__ int64_t sh[kSelThreads];
    __shared__ unsigned long long s_chunk, s_K;
    __shared__ int64_t s_before, s_tile, s_nch;
    __shared__ int s_off;
    const int t = threadIdx.x;
    const int64_t cap = ds->pool_cap;
    if (t == 0) {
        if (!ds->done && !ds->paused && ds->top + ds->maxC > ds->cap_stack) ds->paused = 1;
        s_off = idle(ds) ? 1 : 0;
        s_chunk = (unsigned long long)nchunks;
        s_before = 0;
        s_tile = 0;
    }
    __syncthreads();
    const bool off = s_off != 0;
    // the first chunk whose running sum passes pool_cap (chunk sums scanned a
    // block-width at a time), and the children in the chunks before it
    int64_t base = 0;
    for (int c0 = 0; c0 < nchunks && !off; c0 += kSelThreads) {
        const int c = c0 + t;
        const int64_t v = c < nchunks ? sums[c] : 0;
        const int64_t incl = base + block_scan_incl(v, sh);
        if (t == kSelThreads - 1) s_tile = incl;  // the running sum through this tile
        if (c < nchunks && incl > cap) atomicMin(&s_chunk, (unsigned long long)c);
        __syncthreads();
        if ((unsigned long long)c == s_chunk) s_before = incl - v;
        base = s_tile;
        __syncthreads();
        if (s_chunk < (unsigned long long)nchunks) break;
    }
    const int64_t c = (int64_t)s_chunk;
    if (t == 0) {
        // every entry of the chunks before the cut fits; when no chunk passes
        // pool_cap, so does every entry within reach, with all their children
        s_K = c < nchunks ? (unsigned long long)(c * kSelThreads) : (unsigned long long)min(ds->top, ds->maxK);
        s_nch = c < nchunks ? s_before : s_tile;
    }
    __syncthreads();
    if (!off && c < nchunks) {
        const int64_t i = c * kSelThreads + t;
        const int64_t v = kids_from_top(ds, sdep, i);
        const int64_t pre = s_before + block_scan_incl(v, sh);  // children up to and including entry i
        // entries of the chunk that fit: those with prefix <= cap (and a parent)
        const int fits = (v > 0 && pre <= cap) ? 1 : 0;
        if (fits) atomicMax(&s_K, (unsigned long long)(i + 1));
        __syncthreads();
        if (fits && (unsigned long long)(i + 1) == s_K) s_nch = pre;
        __syncthreads();
    }
    if (t == 0) {
        int64_t K = off ? 0 : (int64_t)s_K, nch = off ? 0 : s_nch;
        if (!off && K == 0 && ds->top > 0) {  // the first parent alone passes pool_cap: it is taken
            K = 1;
            nch = ds->n - sdep[ds->top - 1];
        }
        ds->K = K;
        ds->nch = nch;
        ds->base = ds->top - K;
        req->a.K = K;
        req->a.parent_top = ds->top;
        req->a.out_base = ds->base;
        req->a.ub_in = ds->UB;
        req->nchild = nch;
        req->res.best = ((unsigned long long)(uint32_t)ds->UB << 32) | 0xffffffffull;
        req->res.fingerprint = 0;
        req->res.bad = 0;
        req->res.nchild = 0;
        req->res.nsurv = 0;
        seg->count = K;
    }
}

__global__ void dstep_update_kernel(DevSearch *__restrict__ ds, const StepReq *__restrict__ req,
                                    int64_t *__restrict__ steplog)
{
    if (threadIdx.x != 0 || idle(ds) || ds->K == 0) return;
    const StepResultDev o = req->res;
    if (o.bad || (int64_t)o.nchild != ds->nch) {
        ds->done = 1;
        ds->status = FSP_E_BADNODE;
        return;
    }
    ds->nodes += ds->nch;
    const uint32_t idx = (uint32_t)(o.best & 0xffffffffu);
    if (idx != 0xffffffffu) {
        ds->UB = (int32_t)(o.best >> 32);
        ++ds->improvements;
    }
    ds->top = ds->base + o.nsurv;
    ds->max_stack = max(ds->max_stack, ds->top);
    if (steplog && ds->steps < ds->steplog_cap) {
        int64_t *L = steplog + ds->steps * 6;
        L[0] = ds->K;
        L[1] = ds->nch;
        L[2] = ds->UB;
        L[3] = o.nsurv;
        L[4] = ds->top;
        L[5] = (int64_t)o.fingerprint;
    }
    ++ds->steps;
    if (ds->top == 0) {
        ds->done = 1;
        ds->status = FSP_OK;
    } else if (ds->nodes >= ds->node_budget) {
        ds->done = 1;
        ds->status = FSP_BUDGET;
    }
}

}  // namespace

hipError_t launch_device_step_select(DevSearch *ds, const int32_t *sdep, int64_t *sums, int nchunks, StepReq *req,
                                     ScanSeg *seg, hipStream_t s)
{
    dsel_sums_kernel<<<nchunks, kSelThreads, 0, s>>>(ds, sdep, sums);
    dsel_finish_kernel<<<1, kSelThreads, 0, s>>>(ds, sdep, sums, nchunks, req, seg);
    return hipGetLastError();
}

hipError_t launch_device_step_update(DevSearch *ds, const StepReq *req, int64_t *steplog, hipStream_t s)
{
    dstep_update_kernel<<<1, 64, 0, s>>>(ds, req, steplog);
    return hipGetLastError();
}

}  // namespace fspbb
