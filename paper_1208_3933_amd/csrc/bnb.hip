// Pool-synchronous branch-and-bound steps on the device, for R independent
// searches at once (Sec. II-A operators: branching, bounding, elimination;
// Sec. III-A: the pool of sub-problems is bounded in parallel).  Every kernel
// has a 2-D grid: y selects the search, x covers its parents or children;
// blocks past a search's size return at once.
//
// For each search, given K parents in pop order, the step
//   1. validates each parent and counts its children (n - d),
//   2. takes child offsets by an exclusive prefix sum,
//   3. lists each parent's unscheduled jobs in increasing id (forward
//      branching: child k appends the k-th unscheduled job, Sec. II-B),
//   4. writes the child rows (they are then bounded by the bound kernels),
//   5. takes the best complete child below the upper bound with a 64-bit
//      atomic minimum over (bound << 32 | child index), so the first child in
//      child order wins ties whatever the order of the atomics,
//   6. keeps the non-leaf children whose bound is below the new upper bound
//      and compacts them stably (prefix sum), optionally in reverse child
//      order so that pushing them on a stack leaves the first child on top.
// The compaction of step 6 keeps survivor bits and per-block counts; one
// small launch scans the block counts, and a survivor's rank is its block's
// offset plus the bits before it within the block.
#include <algorithm>

#include "step_dev.h"

namespace fspbb {

// ---- block-level helpers (blocks of 256 threads)

// Inclusive prefix sum of one value per thread over the block: within each
// wave by shuffles, then the sums of the waves before.  sh holds 4 words.
__device__ inline uint32_t block_inclusive_sum(uint32_t v, uint32_t *sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    for (int w = 0; w < wv; ++w) x += sh[w];
    __syncthreads();
    return x;
}

// out[i] = in[0] + ... + in[i - 1] for i < count (in and out may be the same
// array), the sum of all to *total; one block, 4,096 items per round.
__device__ inline void block_scan_array(const uint32_t *in, uint32_t *out, int64_t count, uint32_t *total,
                                        uint32_t *sh, uint32_t *round_total)
{
    constexpr int kItems = 16;
    uint32_t carry = 0;
    for (int64_t base = 0; base < count; base += 256 * kItems) {
        const int64_t i0 = base + (int64_t)threadIdx.x * kItems;
        uint32_t v[kItems], sum = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            v[k] = i0 + k < count ? in[i0 + k] : 0u;
            sum += v[k];
        }
        const uint32_t inc = block_inclusive_sum(sum, sh);
        uint32_t run = carry + inc - sum;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (i0 + k < count) out[i0 + k] = run;
            run += v[k];
        }
        if (threadIdx.x == 255) *round_total = inc;
        __syncthreads();
        carry += *round_total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// One wave per parent: validation and child count.
__global__ __launch_bounds__(256) void mstep_count_kernel(const StepReq *__restrict__ reqs)
{
    __shared__ uint32_t mask[4][kMaxJobs / 32];
    ReqP q = req_of(reqs);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + wv;
    if (p >= q->a.K) return;  // whole wave
    const int n = q->a.n;
    const int d = parent_depth(q, p);
    const bool ok = wave_prefix_set(parent_row(q, p), d, n, mask[wv], lane);
    if (lane == 0) {
        q->w.cnt[p] = (ok && d < n) ? (uint32_t)(n - d) : 0u;
        if (!ok) atomicAdd(q->w.bad, 1ull);
    }
}

// One wave per parent: each unscheduled job j goes to slot off[p] + (number
// of unscheduled jobs below j), i.e. children in increasing job id.
__global__ __launch_bounds__(256) void mstep_ulist_kernel(const StepReq *__restrict__ reqs)
{
    __shared__ uint32_t mask[4][kMaxJobs / 32];
    ReqP q = req_of(reqs);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + wv;
    if (p >= q->a.K) return;      // whole wave
    if (q->w.cnt[p] == 0) return;  // whole wave
    const int n = q->a.n;
    const int d = parent_depth(q, p);
    wave_prefix_set(parent_row(q, p), d, n, mask[wv], lane);
    const int64_t base = q->w.off[p];
    int32_t *ujob = q->w.ujob, *upar = q->w.upar;
    for (int j = lane; j < n; j += 64) {
        const int wj = j >> 5;
        const uint32_t mw = mask[wv][wj];
        if ((mw >> (j & 31)) & 1u) continue;
        int below = __popc(mw & ((1u << (j & 31)) - 1u));
        for (int t = 0; t < wj; ++t) below += __popc(mask[wv][t]);
        const int64_t slot = base + (j - below);
        ujob[slot] = j;
        upar[slot] = (int32_t)p;
    }
}

// Rows and survivor copies run kRowLanes lanes per child (8 children per
// wave): a wave per child would leave most lanes idle on shallow rows and make
// the dispatch of one wave per child the cost.
constexpr int kRowLanes = 8;
constexpr int kRowsPerBlock = 256 / kRowLanes;

// Child row = parent prefix followed by the appended job.
__global__ __launch_bounds__(256) void mstep_rows_kernel(const StepReq *__restrict__ reqs)
{
    ReqP q = req_of(reqs);
    if (q->w.prow) return;  // whole block: children bounded from their parents
    const int64_t c = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x / kRowLanes);
    const int sub = threadIdx.x % kRowLanes;
    if (c >= q->nchild) return;
    const int n = q->a.n;
    const int64_t p = q->w.upar[c];
    const int d = parent_depth(q, p);
    const int32_t *prow = parent_row(q, p);
    int32_t *crow = q->w.crow + c * (int64_t)n;
    const int32_t j = q->w.ujob[c];
    for (int t = sub; t <= d; t += kRowLanes) crow[t] = t < d ? prow[t] : j;
    if (sub == 0) q->w.cdepth[c] = d + 1;
}

__global__ __launch_bounds__(256) void mstep_leaf_kernel(const StepReq *__restrict__ reqs)
{
    ReqP q = req_of(reqs);
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= q->nchild) return;
    const int32_t lb = q->w.clb[c];
    if (q->w.cdepth[c] == q->a.n && lb >= 0 && lb < q->a.ub_in)
        atomicMin(q->w.best, ((unsigned long long)(uint32_t)lb << 32) | (unsigned long long)c);
}

// Keep, one block per 256 children: each wave's ballot gives two words of
// survivor bits; thread 0 writes the words' offsets within the block and the
// block's count.
__global__ __launch_bounds__(256) void mstep_keep_kernel(const StepReq *__restrict__ reqs)
{
    __shared__ uint32_t wcnt[8];
    ReqP q = req_of(reqs);
    const int64_t nch = q->nchild;
    const int64_t nblk = (nch + 255) >> 8;
    if ((int64_t)blockIdx.x >= nblk) return;  // whole block
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t W = (nch + 31) >> 5;
    uint32_t *kb = q->w.keep;
    bool k = false;
    if (c < nch) {
        const int32_t ub = (int32_t)(*q->w.best >> 32);
        const int32_t lb = q->w.clb[c];
        k = q->w.cdepth[c] < q->a.n && lb >= 0 && lb < ub;
    }
    const unsigned long long bal = __ballot(k);
    if ((lane & 31) == 0) {
        const uint32_t bits = lane ? (uint32_t)(bal >> 32) : (uint32_t)bal;
        if ((c >> 5) < W) kb[c >> 5] = bits;
        wcnt[wv * 2 + (lane >> 5)] = __popc(bits);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int t = 0; t < 8; ++t) {
            const int64_t g = (int64_t)blockIdx.x * 8 + t;
            if (g < W) kb[W + g] = run;
            run += wcnt[t];
        }
        q->w.pos[blockIdx.x] = run;
    }
}

// One block per search: block counts -> block offsets, and the survivor count.
__global__ __launch_bounds__(256) void mstep_blockscan_kernel(const StepReq *__restrict__ reqs)
{
    __shared__ uint32_t sh[4];
    __shared__ uint32_t round_total;
    ReqP q = req_of(reqs);
    const int64_t nblk = (q->nchild + 255) >> 8;
    block_scan_array(q->w.pos, q->w.pos, nblk, q->w.nsurv, sh, &round_total);
}

// Whether child c survives, and its rank among the survivors (c < nchild).
__device__ __forceinline__ bool surv_kept(ReqP q, int64_t c) { return (q->w.keep[c >> 5] >> (c & 31)) & 1u; }
__device__ __forceinline__ uint32_t surv_rank(ReqP q, int64_t c)
{
    const int64_t W = (q->nchild + 31) >> 5;
    const uint32_t *kb = q->w.keep;
    return q->w.pos[c >> 8] + kb[W + (c >> 5)] + (uint32_t)__popc(kb[c >> 5] & ((1u << (c & 31)) - 1u));
}

// The step's tail after the compaction, in one launch over disjoint block
// ranges (all four parts only read the compaction and write disjoint outputs):
//   survivor rows to their compacted slots (kRowLanes lanes per child),
//   the fingerprint of the survivor order, survivors per parent, and the
//   incumbent row.

// Block blk of the survivor copies.
__device__ inline void tail_scatter(ReqP q, int64_t blk)
{
    const int64_t c = blk * kRowsPerBlock + (threadIdx.x / kRowLanes);
    const int sub = threadIdx.x % kRowLanes;
    if (c >= q->nchild) return;
    if (!surv_kept(q, c)) return;
    const int n = q->a.n;
    const int64_t S = *q->w.nsurv;
    const int64_t s = surv_rank(q, c);
    const int64_t dst = q->a.out_reversed ? q->a.out_base + (S - 1 - s) : q->a.out_base + s;
    if (dst < 0 || dst >= q->a.out_cap) return;  // overflow is reported by the host
    const int d = q->w.cdepth[c];
    const int64_t orow = q->a.oslot ? (int64_t)q->a.oslot[s * q->a.oslot_step] : dst;
    int32_t *out = q->a.out_rows + orow * (int64_t)n;
    if (q->w.prow) {  // parent prefix (from the step's copy of the parent rows) + appended job
        const int32_t *src = q->w.prow + (int64_t)q->w.upar[c] * n;
        const int32_t j = q->w.ujob[c];
        for (int t = sub; t < d; t += kRowLanes) out[t] = t + 1 < d ? src[t] : j;
    } else {
        const int32_t *src = q->w.crow + c * (int64_t)n;
        for (int t = sub; t < d; t += kRowLanes) out[t] = src[t];
    }
    if (sub == 0) {
        q->a.out_depth[dst] = d;
        if (q->a.out_lb) q->a.out_lb[dst] = q->w.clb[c];
    }
}

// Fingerprint of the survivor order: sum over survivors of (S - rank) *
// (job + 1); block blk of nblk strides over the children, one block reduction
// and one atomic per block.
__device__ inline void tail_fingerprint(ReqP q, int64_t blk, int64_t nblk, unsigned long long *part)
{
    const int64_t nch = q->nchild;
    if (blk * 256 >= nch) return;  // whole block
    unsigned long long v = 0;
    const unsigned long long S = *q->w.nsurv;
    for (int64_t c = blk * 256 + threadIdx.x; c < nch; c += nblk * 256)
        if (surv_kept(q, c)) v += (S - surv_rank(q, c)) * (unsigned long long)(q->w.ujob[c] + 1);
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part[0]) atomicAdd(q->w.fingerprint, part[0]);
}

// Survivors per parent: a parent's children are contiguous in child order, so
// its survivor count is the difference of the compaction offsets at the ends
// of its children.  Block blk of nblk strides over the parents.
__device__ inline void tail_per_parent(ReqP q, int64_t blk, int64_t nblk)
{
    if (!q->a.surv_per_parent) return;
    for (int64_t p = blk * 256 + threadIdx.x; p < q->a.K; p += nblk * 256) {
        const uint32_t cnt = q->w.cnt[p];
        uint32_t v = 0u;
        if (cnt) {
            const int64_t lo = q->w.off[p], hi = lo + cnt;
            const uint32_t end = hi < q->nchild ? surv_rank(q, hi) : *q->w.nsurv;
            v = end - surv_rank(q, lo);
        }
        q->a.surv_per_parent[p] = v;
    }
}

// The best complete child, when it lowered the upper bound, becomes the incumbent.
__device__ inline void tail_incumbent(ReqP q)
{
    const unsigned long long b = *q->w.best;
    const uint32_t idx = (uint32_t)(b & 0xffffffffu);
    int32_t *inc = q->a.incumbent;
    if (idx == 0xffffffffu || !inc) return;
    const int n = q->a.n;
    if (q->w.prow) {  // a complete child: n - 1 parent jobs and the appended one
        const int32_t *src = q->w.prow + (int64_t)q->w.upar[idx] * n;
        const int32_t j = q->w.ujob[idx];
        for (int t = threadIdx.x; t < n; t += blockDim.x) inc[t] = t + 1 < n ? src[t] : j;
    } else {
        for (int t = threadIdx.x; t < n; t += blockDim.x) inc[t] = q->w.crow[(int64_t)idx * n + t];
    }
}

constexpr int kPrintBlocks = 128, kParentBlocks = 64;

// Blocks [0, bs) copy survivors, [bs, bs + bf) take the fingerprint,
// [bs + bf, bs + bf + bp) count survivors per parent, the last one writes the
// incumbent.  Block-uniform branches: every barrier is reached by a whole block.
__global__ __launch_bounds__(256) void mstep_tail_kernel(const StepReq *__restrict__ reqs, int bs, int bf, int bp)
{
    __shared__ unsigned long long part[256];
    ReqP q = req_of(reqs);
    const int b = blockIdx.x;
    if (b < bs) tail_scatter(q, b);
    else if (b < bs + bf) tail_fingerprint(q, b - bs, bf, part);
    else if (b < bs + bf + bp) tail_per_parent(q, b - bs - bf, bp);
    else tail_incumbent(q);
}

static unsigned blocks_for(int64_t items, int per_block)
{
    const int64_t b = (items + per_block - 1) / per_block;
    return (unsigned)(b > 0 ? b : 1);
}

hipError_t mstep_phase1(const StepReq *reqs, const ScanSeg *segs, int R, int64_t maxK, hipStream_t s)
{
    if (R <= 0) return hipSuccess;
    if (maxK > 0) mstep_count_kernel<<<dim3(blocks_for(maxK, 4), R), 256, 0, s>>>(reqs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return exclusive_scan_segments(segs, R, maxK, s);
}

hipError_t mstep_list(const StepReq *reqs, int R, int64_t maxK, int64_t maxC, hipStream_t s)
{
    if (R <= 0 || maxC <= 0) return hipSuccess;
    mstep_ulist_kernel<<<dim3(blocks_for(maxK, 4), R), 256, 0, s>>>(reqs);
    return hipGetLastError();
}

hipError_t mstep_branch(const StepReq *reqs, int R, int64_t maxK, int64_t maxC, hipStream_t s)
{
    if (R <= 0 || maxC <= 0) return hipSuccess;
    hipError_t e = mstep_list(reqs, R, maxK, maxC, s);
    if (e != hipSuccess) return e;
    mstep_rows_kernel<<<dim3(blocks_for(maxC, kRowsPerBlock), R), 256, 0, s>>>(reqs);
    return hipGetLastError();
}

hipError_t mstep_finish(const StepReq *reqs, int R, int64_t maxK, int64_t maxC, hipStream_t s, bool leaves_done)
{
    if (R <= 0) return hipSuccess;
    if (maxC > 0) {
        if (!leaves_done) mstep_leaf_kernel<<<dim3(blocks_for(maxC, 256), R), 256, 0, s>>>(reqs);
        mstep_keep_kernel<<<dim3(blocks_for(maxC, 256), R), 256, 0, s>>>(reqs);
        mstep_blockscan_kernel<<<dim3(1, R), 256, 0, s>>>(reqs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // without children the tail only writes the per-parent counts (all zero)
    const int bs = maxC > 0 ? (int)blocks_for(maxC, kRowsPerBlock) : 0;
    const int bf = maxC > 0 ? (int)std::min<int64_t>(blocks_for(maxC, 256), kPrintBlocks) : 0;
    const int bp = maxK > 0 ? (int)std::min<int64_t>(blocks_for(maxK, 256), kParentBlocks) : 0;
    mstep_tail_kernel<<<dim3((unsigned)(bs + bf + bp + 1), R), 256, 0, s>>>(reqs, bs, bf, bp);
    return hipGetLastError();
}

}  // namespace fspbb
