// One pool-synchronous branch-and-bound step on the device (Sec. II-A
// operators: branching, bounding, elimination; Sec. III-A: the pool of
// sub-problems is bounded in parallel).
//
// Given K parents in pop order, the step
//   1. validates each parent and counts its children (n - d),
//   2. takes child offsets by an exclusive prefix sum,
//   3. lists each parent's unscheduled jobs in increasing id (forward
//      branching: child k appends the k-th unscheduled job, Sec. II-B),
//   4. writes the child rows and bounds them with the bound kernels,
//   5. takes the best complete child below the upper bound with a 64-bit
//      atomic minimum over (bound << 32 | child index), so the first child in
//      child order wins ties whatever the order of the atomics,
//   6. keeps the non-leaf children whose bound is below the new upper bound
//      and compacts them stably (prefix sum), optionally in reverse child
//      order so that pushing them on a stack leaves the first child on top.
#include "bnb.h"
#include "scan.h"

namespace fspbb {

__device__ __forceinline__ const int32_t *parent_row(const StepArgs &a, int64_t p)
{
    return a.parents + (a.parents_reversed ? (a.parent_top - 1 - p) : p) * (int64_t)a.n;
}
__device__ __forceinline__ int32_t parent_depth(const StepArgs &a, int64_t p)
{
    return a.pdepth[a.parents_reversed ? (a.parent_top - 1 - p) : p];
}

// One wave per parent: the lanes build the parent's scheduled set in a 16-word
// LDS mask (LDS atomics; a returned bit already set means a repeated job).
// Returns, uniformly over the wave, whether the parent is valid: depth in
// 0..n, every job in 0..n-1, no repeat.
__device__ inline bool wave_prefix_set(const int32_t *row, int d, int n, uint32_t *mask, int lane)
{
    if (lane < kMaxJobs / 32) mask[lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    bool bad = d < 0 || d > n;
    if (!bad) {
        for (int t = lane; t < d; t += 64) {
            const int j = row[t];
            if ((unsigned)j >= (unsigned)n) { bad = true; continue; }
            const uint32_t bit = 1u << (j & 31);
            if (atomicOr(&mask[j >> 5], bit) & bit) bad = true;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return __ballot(bad) == 0;
}

__global__ __launch_bounds__(256) void step_count_kernel(StepArgs a, StepScratch w)
{
    __shared__ uint32_t mask[4][kMaxJobs / 32];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + wv;
    if (p >= a.K) return;  // whole wave
    const int d = parent_depth(a, p);
    const bool ok = wave_prefix_set(parent_row(a, p), d, a.n, mask[wv], lane);
    if (lane == 0) {
        w.cnt[p] = (ok && d < a.n) ? (uint32_t)(a.n - d) : 0u;
        if (!ok) atomicAdd(w.bad, 1ull);
    }
}

// One wave per parent: each unscheduled job j goes to slot off[p] + (number
// of unscheduled jobs below j), i.e. children in increasing job id.
__global__ __launch_bounds__(256) void step_ulist_kernel(StepArgs a, StepScratch w)
{
    __shared__ uint32_t mask[4][kMaxJobs / 32];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + wv;
    if (p >= a.K) return;  // whole wave
    if (w.cnt[p] == 0) return;  // whole wave (uniform load)
    const int d = parent_depth(a, p);
    wave_prefix_set(parent_row(a, p), d, a.n, mask[wv], lane);
    const int64_t base = w.off[p];
    for (int j = lane; j < a.n; j += 64) {
        const int wj = j >> 5;
        const uint32_t mw = mask[wv][wj];
        if ((mw >> (j & 31)) & 1u) continue;
        int below = __popc(mw & ((1u << (j & 31)) - 1u));
        for (int q = 0; q < wj; ++q) below += __popc(mask[wv][q]);
        const int64_t slot = base + (j - below);
        w.ujob[slot] = j;
        w.upar[slot] = (int32_t)p;
    }
}

// One wave per child: child row = parent prefix followed by the appended job.
__global__ __launch_bounds__(256) void step_rows_kernel(StepArgs a, StepScratch w, int64_t nchild)
{
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= nchild) return;
    const int64_t p = w.upar[c];
    const int d = parent_depth(a, p);
    const int32_t *prow = parent_row(a, p);
    int32_t *crow = w.crow + c * (int64_t)a.n;
    for (int t = lane; t <= d; t += 64) crow[t] = t < d ? prow[t] : w.ujob[c];
    if (lane == 0) w.cdepth[c] = d + 1;
}

__global__ __launch_bounds__(256) void step_leaf_kernel(StepArgs a, StepScratch w, int64_t nchild)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nchild) return;
    const int32_t lb = w.clb[c];
    if (w.cdepth[c] == a.n && lb >= 0 && lb < a.ub_in)
        atomicMin(w.best, ((unsigned long long)(uint32_t)lb << 32) | (unsigned long long)c);
}

__global__ __launch_bounds__(256) void step_keep_kernel(StepArgs a, StepScratch w, int64_t nchild)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nchild) return;
    const int32_t ub = (int32_t)(*w.best >> 32);
    w.keep[c] = (w.cdepth[c] < a.n && w.clb[c] >= 0 && w.clb[c] < ub) ? 1u : 0u;
}

// One wave per child: survivors are copied to their compacted slot.
__global__ __launch_bounds__(256) void step_scatter_kernel(StepArgs a, StepScratch w, int64_t nchild)
{
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= nchild) return;
    if (!w.keep[c]) return;
    const int64_t S = *w.nsurv;
    const int64_t s = w.pos[c];
    const int64_t dst = a.out_reversed ? a.out_base + (S - 1 - s) : a.out_base + s;
    if (dst < 0 || dst >= a.out_cap) return;  // overflow is reported by the host
    const int d = w.cdepth[c];
    const int32_t *src = w.crow + c * (int64_t)a.n;
    int32_t *out = a.out_rows + dst * (int64_t)a.n;
    for (int t = lane; t < d; t += 64) out[t] = src[t];
    if (lane == 0) {
        a.out_depth[dst] = d;
        if (a.out_lb) a.out_lb[dst] = w.clb[c];
    }
}

// Fingerprint of the survivor order: sum over survivors of (S - rank) * (job + 1),
// one block reduction and one atomic per block.
__global__ __launch_bounds__(256) void step_fingerprint_kernel(StepScratch w, int64_t nchild)
{
    __shared__ unsigned long long part[256];
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long v = 0;
    if (c < nchild && w.keep[c]) {
        const unsigned long long S = *w.nsurv;
        v = (S - w.pos[c]) * (unsigned long long)(w.ujob[c] + 1);
    }
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part[0]) atomicAdd(w.fingerprint, part[0]);
}

// Survivors per parent: a parent's children are contiguous in child order, so
// its survivor count is the difference of the compaction offsets at the ends
// of its children.
__global__ __launch_bounds__(256) void step_per_parent_kernel(StepArgs a, StepScratch w, int64_t nchild)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.K || !a.surv_per_parent) return;
    const uint32_t cnt = w.cnt[p];
    if (cnt == 0) { a.surv_per_parent[p] = 0u; return; }
    const int64_t lo = w.off[p], hi = lo + cnt;
    const uint32_t end = hi < nchild ? w.pos[hi] : *w.nsurv;
    a.surv_per_parent[p] = end - w.pos[lo];
}

__global__ void step_incumbent_kernel(StepArgs a, StepScratch w)
{
    const unsigned long long b = *w.best;
    const uint32_t idx = (uint32_t)(b & 0xffffffffu);
    if (idx == 0xffffffffu || !a.incumbent) return;
    for (int t = threadIdx.x; t < a.n; t += blockDim.x) a.incumbent[t] = w.crow[(int64_t)idx * a.n + t];
}

__global__ void step_init_kernel(StepArgs a, StepScratch w)
{
    *w.best = ((unsigned long long)(uint32_t)a.ub_in << 32) | 0xffffffffull;
    *w.fingerprint = 0ull;
    *w.bad = 0ull;
}

__global__ void store_zero_kernel(uint32_t *p) { *p = 0u; }

static unsigned blocks_for(int64_t items, int per_block) { return (unsigned)((items + per_block - 1) / per_block); }

hipError_t step_phase1(const StepArgs &a, const StepScratch &w, hipStream_t s)
{
    step_init_kernel<<<1, 1, 0, s>>>(a, w);
    if (a.K > 0) {
        step_count_kernel<<<blocks_for(a.K, 4), 256, 0, s>>>(a, w);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return exclusive_scan_u32(w.cnt, w.off, a.K, w.nchild, w.scan_scratch, s);
}

hipError_t step_phase2(fsp_instance_s *I, const StepArgs &a, const StepScratch &w, int64_t nchild, hipStream_t s)
{
    if (nchild > 0) {
        step_ulist_kernel<<<blocks_for(a.K, 4), 256, 0, s>>>(a, w);
        step_rows_kernel<<<blocks_for(nchild, 4), 256, 0, s>>>(a, w, nchild);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = I->packed16 ? launch_bound_packed(I, w.crow, w.cdepth, nchild, w.clb, s)
                        : launch_bound_lane32(I, w.crow, w.cdepth, nchild, w.clb, s);
        if (e != hipSuccess) return e;
        step_leaf_kernel<<<blocks_for(nchild, 256), 256, 0, s>>>(a, w, nchild);
        step_keep_kernel<<<blocks_for(nchild, 256), 256, 0, s>>>(a, w, nchild);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = exclusive_scan_u32(w.keep, w.pos, nchild, w.nsurv, w.scan_scratch, s);
        if (e != hipSuccess) return e;
        step_scatter_kernel<<<blocks_for(nchild, 4), 256, 0, s>>>(a, w, nchild);
        step_fingerprint_kernel<<<blocks_for(nchild, 256), 256, 0, s>>>(w, nchild);
        step_per_parent_kernel<<<blocks_for(a.K, 256), 256, 0, s>>>(a, w, nchild);
        step_incumbent_kernel<<<1, 256, 0, s>>>(a, w);
    } else {
        store_zero_kernel<<<1, 1, 0, s>>>(w.nsurv);
    }
    return hipGetLastError();
}

}  // namespace fspbb
