// Host side of the branch-and-bound: the C ABI step call, the NEH initial
// upper bound, the depth-first search state with its stack on the device, and
// the step that advances one or many searches with one set of launches.
//
// A search is pool-synchronous (Sec. III-A: the CPU selects a pool, the GPU
// bounds it): each step pops parents from the top of the stack while their
// children fit in pool_cap (the first parent is always taken), branches them
// in pop order with children in increasing job id, bounds every child,
// lowers the upper bound with the best complete child (the first in child
// order on ties), and pushes the children whose bound is below the upper
// bound in reverse child order, so the first child is popped first.  With a
// fixed (instance, initial upper bound, pool_cap) every count is a
// deterministic function of the search, step by step, whichever other
// searches share its launches.
#include <algorithm>
#include <cstring>
#include <vector>

#include "best_first.h"
#include "bound_wide.h"
#include "kids16.h"
#include "search.h"

using namespace fspbb;

namespace fspbb {

namespace {
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

// ---------------------------------------------------------------- scratch

hipError_t StepBuffers::ensure_k(int64_t K, hipStream_t s)
{
    if (kblob && K <= Kcap) return hipSuccess;
    if (kblob) stream_free(kblob, s);
    kblob = nullptr;
    Kcap = std::max<int64_t>(K, 1);
    const size_t kb = al256((size_t)Kcap * 4), sb = al256(scan_scratch_bytes(Kcap));
    hipError_t e = stream_alloc((void **)&kblob, 2 * kb + sb, s);
    if (e != hipSuccess) { kblob = nullptr; Kcap = 0; return e; }
    char *p = (char *)kblob;
    w.cnt = (uint32_t *)p; p += kb;
    w.off = (uint32_t *)p; p += kb;
    sums_k = (uint32_t *)p;
    return hipSuccess;
}

hipError_t StepBuffers::ensure_c(int64_t C, int n_, hipStream_t s)
{
    if (cblob && C <= Ccap && n_ == n) return hipSuccess;
    if (cblob) stream_free(cblob, s);
    cblob = nullptr;
    Ccap = std::max<int64_t>(C, 1);
    n = n_;
    // (each array holds at least 64 words, so keep also fits the word offsets
    // of a step with fewer than 64 children)
    const size_t cb = al256((size_t)Ccap * 4), rows_b = rows ? al256((size_t)Ccap * n * 4) : 0;
    hipError_t e = stream_alloc((void **)&cblob, 6 * cb + rows_b, s);
    if (e != hipSuccess) { cblob = nullptr; Ccap = 0; return e; }
    char *p = (char *)cblob;
    w.ujob = (int32_t *)p; p += cb;
    w.upar = (int32_t *)p; p += cb;
    w.cdepth = (int32_t *)p; p += cb;
    w.clb = (int32_t *)p; p += cb;
    w.keep = (uint32_t *)p; p += cb;
    w.pos = (uint32_t *)p; p += cb;
    w.crow = rows ? (int32_t *)p : nullptr;
    return hipSuccess;
}

void StepBuffers::release(hipStream_t s)
{
    if (kblob) stream_free(kblob, s);
    if (cblob) stream_free(cblob, s);
    kblob = cblob = nullptr;
    Kcap = Ccap = 0;
}

size_t StepBuffers::bytes_for(int64_t Kc, int64_t Cc, int n_, bool rows_)
{
    return (size_t)Kc * 8 + (size_t)Cc * (24 + (rows_ ? 4 * (size_t)n_ : 0)) + scan_scratch_bytes(Kc);
}

size_t StepBuffers::bytes() const { return bytes_for(Kcap, Ccap, n, rows); }

hipError_t TickContext::reserve(size_t bytes)
{
    if (bytes > dcap) {
        if (dtab) stream_free(dtab, s);
        dtab = nullptr;
        dcap = 0;
        const size_t c = std::max(bytes, (size_t)64 * 1024);
        hipError_t e = stream_alloc((void **)&dtab, c, s);
        if (e != hipSuccess) return e;
        dcap = c;
    }
    if (bytes > hcap) {
        // the previous tick ended with a stream synchronization: no copy reads htab
        pinned_put(htab, hcap);
        htab = nullptr;
        hcap = 0;
        hipError_t e = pinned_get(&htab, &hcap, std::max(bytes, (size_t)64 * 1024));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t TickContext::device_bytes() const { return dcap + arena.dev_bytes + kids.cap; }

void TickContext::release()
{
    if (dtab) stream_free(dtab, s);
    arena.release(s);
    kids.release(s);
    hipStreamSynchronize(s);
    pinned_put(htab, hcap);
    dtab = htab = nullptr;
    dcap = hcap = 0;
}

// ---------------------------------------------------------------- NEH

// NEH (Nawaz, Enscore and Ham 1983) with Taillard's evaluation of all
// insertion positions in O(L m) per job: e = heads of the current sequence,
// q = tails, f = completion of the inserted job.  Jobs by decreasing total
// time (smaller id first on ties); the earliest best position wins.
int32_t neh(const int32_t *p, int n, int m, int32_t *perm)
{
    std::vector<int> jobs(n);
    std::vector<int64_t> tot(n, 0);
    for (int j = 0; j < n; ++j) {
        jobs[j] = j;
        for (int k = 0; k < m; ++k) tot[j] += p[j * m + k];
    }
    std::stable_sort(jobs.begin(), jobs.end(), [&](int a, int b) { return tot[a] > tot[b]; });
    std::vector<int> seq;
    seq.reserve(n);
    std::vector<int64_t> e((size_t)(n + 1) * m), q((size_t)(n + 2) * m), f(m);
    for (int x : jobs) {
        const int L = (int)seq.size();
        for (int k = 0; k < m; ++k) e[k] = 0;                      // e[0][k]
        for (int i = 1; i <= L; ++i)
            for (int k = 0; k < m; ++k) {
                const int64_t up = e[(size_t)(i - 1) * m + k], left = k ? e[(size_t)i * m + k - 1] : 0;
                e[(size_t)i * m + k] = std::max(up, left) + p[seq[i - 1] * m + k];
            }
        for (int k = 0; k < m; ++k) q[(size_t)L * m + k] = 0;      // nothing after the end
        for (int i = L - 1; i >= 0; --i)
            for (int k = m - 1; k >= 0; --k) {
                const int64_t down = q[(size_t)(i + 1) * m + k], right = k + 1 < m ? q[(size_t)i * m + k + 1] : 0;
                q[(size_t)i * m + k] = std::max(down, right) + p[seq[i] * m + k];
            }
        int best_pos = 0;
        int64_t best = -1;
        for (int i = 0; i <= L; ++i) {
            int64_t ms = 0, prev = 0;
            for (int k = 0; k < m; ++k) {
                prev = std::max(prev, e[(size_t)i * m + k]) + p[x * m + k];
                f[k] = prev;
                ms = std::max(ms, f[k] + q[(size_t)i * m + k]);
            }
            if (best < 0 || ms < best) { best = ms; best_pos = i; }
        }
        seq.insert(seq.begin() + best_pos, x);
    }
    // makespan of the final sequence
    std::vector<int64_t> C(m, 0);
    for (int i = 0; i < n; ++i) {
        C[0] += p[seq[i] * m];
        for (int k = 1; k < m; ++k) C[k] = std::max(C[k], C[k - 1]) + p[seq[i] * m + k];
    }
    if (perm) std::copy(seq.begin(), seq.end(), perm);
    return (int32_t)C[m - 1];
}

// ---------------------------------------------------------------- search

// sort_depths as in launch_bound_packed: off for the children of a depth-first
// step, which come from parents popped off the top of one stack and so sit at
// one or a few depths.
static hipError_t bound_rows(fsp_instance_s *I, const int32_t *rows, const int32_t *depths, int64_t N, int32_t *lb,
                             hipStream_t s, bool sort_depths = true)
{
    if (N <= 0) return hipSuccess;
    return I->packed16 ? launch_bound_packed(I, rows, depths, N, lb, s, sort_depths)
                       : launch_bound_wide(I, rows, depths, N, lb, s, sort_depths);
}

// Whether one step bounds its children from their parents, with the
// (persistent, grow-only) scratch it uses.
struct KidsStep {
    Kids16 &k;
    bool on = false;
    explicit KidsStep(Kids16 &buf) : k(buf) {}
    hipError_t start(const fsp_instance_s *I, int64_t K, int64_t nch, hipStream_t s)
    {
        on = kids16_eligible(I) && nch > 0;
        return on ? kids16_ensure(k, I, K, nch, s) : hipSuccess;
    }
};

// Branch and bound the children of the single search in dreq: from their
// parents on the incremental path, else through child rows and the plain
// bound launch.
static hipError_t branch_and_bound1(const StepReq *dreq, fsp_instance_s *I, KidsStep &ks, int64_t K, int64_t nch,
                                    const StepScratch &w, hipStream_t s, bool sort_depths)
{
    hipError_t e;
    if (ks.on) {
        e = mstep_list(dreq, 1, K, nch, s);
        if (e == hipSuccess) e = kids16_bound(dreq, I, ks.k, w.clb, s);
    } else {
        e = mstep_branch(dreq, 1, K, nch, s);
        if (e == hipSuccess) e = bound_rows(I, w.crow, w.cdepth, nch, w.clb, s, sort_depths);
    }
    return e;
}

// Phase 1, branching and bounding of the single search in dreq, whose nch
// children the host has counted: on the incremental path with validation,
// counts, lists and the leaf step folded into the child launches (the finish
// then runs with leaves_done), else phase 1 and branch_and_bound1.
static hipError_t phase1_and_bound1(const StepReq *dreq, const ScanSeg *seg1, fsp_instance_s *I, KidsStep &ks,
                                    int64_t K, int64_t nch, const StepScratch &w, hipStream_t s, bool *leaves_done)
{
    *leaves_done = false;
    if (ks.on) {
        hipError_t e = kids16_decode(dreq, 1, K, nch, I->n, I->m, s, seg1);
        if (e == hipSuccess) e = launch_scan16(I, ks.k.W, nch, w.clb, s);
        *leaves_done = true;
        return e;
    }
    hipError_t e = mstep_phase1(dreq, seg1, 1, K, s);
    if (e == hipSuccess) e = branch_and_bound1(dreq, I, ks, K, nch, w, s, true);
    return e;
}

hipError_t Search::begin(fsp_instance_s *I, int32_t ub0_in, int64_t pool_cap_in, int64_t node_budget_in,
                         hipStream_t s)
{
    inst = I;
    n = I->n;
    pool_cap = pool_cap_in;
    node_budget = node_budget_in;
    inc.assign(n, -1);
    UB = ub0_in == FSP_UB_NEH ? neh(I->p_host, n, I->m, inc.data()) : ub0_in;
    ub0 = UB;
    cap_stack = initial_stack_rows(pool_cap);
    hipError_t e = stream_alloc((void **)&srows, (size_t)cap_stack * n * 4, s);
    if (e == hipSuccess) e = stream_alloc((void **)&sdep, (size_t)cap_stack * 4, s);
    if (e == hipSuccess) e = stream_alloc((void **)&dinc, (size_t)n * 4, s);
    B.rows = !kids16_eligible(I);
    if (e == hipSuccess) e = B.ensure_k(pool_cap, s);
    if (e == hipSuccess) e = B.ensure_c(pool_cap, n, s);
    // the root: an all-zero row of depth 0 at the bottom of the stack
    if (e == hipSuccess) e = hipMemsetAsync(srows, 0, (size_t)n * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(sdep, 0, 4, s);
    return e;
}

void Search::finish_root(int32_t lb0)
{
    nodes = 1;
    if (lb0 < UB) {
        top = 1;
        runs.push_back({0, 1});
        max_stack = 1;
    }
    done = top == 0 || nodes >= node_budget;
    status = top == 0 ? FSP_OK : (done ? FSP_BUDGET : FSP_OK);
}

hipError_t Search::start(fsp_instance_s *I, int32_t ub0_in, int64_t pool_cap_in, int64_t node_budget_in,
                         hipStream_t s)
{
    hipError_t e = begin(I, ub0_in, pool_cap_in, node_budget_in, s);
    if (e == hipSuccess) e = bound_rows(I, srows, sdep, 1, B.w.clb, s);
    int32_t lb0 = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&lb0, B.w.clb, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    finish_root(lb0);
    return hipSuccess;
}

hipError_t start_many(std::vector<Search *> &ss, const std::vector<StartArgs> &args, TickContext &ctx)
{
    hipStream_t s = ctx.s;
    const size_t R = ss.size();
    if (R == 0) return hipSuccess;
    for (size_t i = 0; i < R; ++i) {
        hipError_t e = ss[i]->begin(args[i].inst, args[i].ub0, args[i].pool_cap, args[i].node_budget, s);
        if (e != hipSuccess) return e;
    }
    if (R == 1) {
        Search &S = *ss[0];
        hipError_t e = bound_rows(S.inst, S.srows, S.sdep, 1, S.B.w.clb, s);
        int32_t lb0 = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&lb0, S.B.w.clb, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        S.finish_root(lb0);
        return hipSuccess;
    }
    // every root bounded into one contiguous array: one merged launch, one copy back
    const size_t bytes = al256(R * 4);
    hipError_t e = ctx.reserve(bytes);
    if (e != hipSuccess) return e;
    int32_t *dlb = (int32_t *)ctx.dtab;
    std::vector<fsp_pool_desc> descs;
    for (size_t i = 0; i < R; ++i) {
        Search &S = *ss[i];
        if (S.inst->packed16)
            descs.push_back(fsp_pool_desc{S.inst, S.srows, S.sdep, 1, dlb + i});
        else if (e == hipSuccess)
            e = bound_rows(S.inst, S.srows, S.sdep, 1, dlb + i, s);
    }
    if (e == hipSuccess && !descs.empty()) e = ctx.arena.run(descs.data(), (int32_t)descs.size(), s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctx.htab, dlb, R * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < R; ++i) ss[i]->finish_root(((const int32_t *)ctx.htab)[i]);
    return hipSuccess;
}

size_t start_scratch_after(const std::vector<StartArgs> &args, const TickContext &ctx)
{
    if (args.size() <= 1) return ctx.device_bytes();  // one root is bounded on its own
    const size_t tab = al256(args.size() * 4);
    const size_t dcap = tab > ctx.dcap ? std::max(tab, (size_t)64 * 1024) : ctx.dcap;
    std::vector<fsp_pool_desc> descs;
    for (const StartArgs &a : args)
        if (a.inst->packed16) descs.push_back(fsp_pool_desc{a.inst, nullptr, nullptr, 1, nullptr});
    size_t arena = ctx.arena.dev_bytes;
    if (!descs.empty()) {
        BatchPlan pl;
        plan_batch(descs.data(), (int32_t)descs.size(), 0, false, pl);
        arena = ctx.arena.bytes_after(pl.ws_bytes + pl.meta_bytes);
    }
    return dcap + arena + ctx.kids.cap;
}

void Search::release(hipStream_t s)
{
    if (srows) stream_free(srows, s);
    if (sdep) stream_free(sdep, s);
    if (dinc) stream_free(dinc, s);
    srows = sdep = dinc = nullptr;
    B.release(s);
}

size_t Search::device_bytes() const
{
    return (swapped ? 0 : (size_t)cap_stack * (n + 1) * 4) + (size_t)n * 4 + B.bytes();
}

hipError_t Search::swap_out(hipStream_t s)
{
    if (swapped) return hipSuccess;
    host_rows.resize((size_t)top * n);
    host_dep.resize((size_t)top);
    hipError_t e = hipSuccess;
    if (top > 0) {
        e = hipMemcpyAsync(host_rows.data(), srows, (size_t)top * n * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(host_dep.data(), sdep, (size_t)top * 4, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    stream_free(srows, s);
    stream_free(sdep, s);
    srows = sdep = nullptr;
    B.release(s);
    swapped = true;
    return hipSuccess;
}

hipError_t Search::swap_in(hipStream_t s)
{
    if (!swapped) return hipSuccess;
    hipError_t e = stream_alloc((void **)&srows, (size_t)cap_stack * n * 4, s);
    if (e == hipSuccess) e = stream_alloc((void **)&sdep, (size_t)cap_stack * 4, s);
    if (e == hipSuccess) e = B.ensure_k(pool_cap, s);
    if (e == hipSuccess) e = B.ensure_c(pool_cap, n, s);
    if (e == hipSuccess && top > 0) {
        e = hipMemcpyAsync(srows, host_rows.data(), (size_t)top * n * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(sdep, host_dep.data(), (size_t)top * 4, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        if (srows) stream_free(srows, s);
        if (sdep) stream_free(sdep, s);
        srows = sdep = nullptr;
        B.release(s);
        return e;
    }
    std::vector<int32_t>().swap(host_rows);
    std::vector<int32_t>().swap(host_dep);
    swapped = false;
    return hipSuccess;
}

void Search::result(fsp_solve_result *res, int32_t *perm_out) const
{
    std::memset(res, 0, sizeof(*res));
    res->opt = UB;
    res->proven = top == 0;
    res->nodes_bounded = nodes;
    res->steps = steps;
    res->ub0 = ub0;
    res->improvements = improvements;
    res->max_stack = max_stack;
    if (perm_out) std::copy(inc.begin(), inc.end(), perm_out);
}

StepSel select_step(const Search &S)
{
    StepSel q;
    for (auto it = S.runs.rbegin(); it != S.runs.rend(); ++it) {
        const int64_t c = S.n - it->first;
        int64_t x = (S.pool_cap - q.nch) / c;
        if (q.K == 0) x = std::max<int64_t>(x, 1);
        x = std::min(x, it->second);
        if (x <= 0) break;
        q.K += x;
        q.nch += x * c;
        if (x < it->second) break;
    }
    return q;
}

// The stack and step buffers prepare_step leaves for the step q (the same
// growth rules: the stack doubles, the buffers take the requested size).
size_t bytes_after_step(const Search &S, const StepSel &q)
{
    int64_t cs = S.cap_stack;
    const int64_t base = S.top - q.K;
    while (base + q.nch > cs) cs *= 2;
    const int64_t k = std::max(S.pool_cap, q.K), c = std::max(S.pool_cap, q.nch);
    const int64_t Kc = (S.B.kblob && k <= S.B.Kcap) ? S.B.Kcap : std::max<int64_t>(k, 1);
    const int64_t Cc = (S.B.cblob && c <= S.B.Ccap && S.B.n == S.n) ? S.B.Ccap : std::max<int64_t>(c, 1);
    return (size_t)cs * (S.n + 1) * 4 + (size_t)S.n * 4 + StepBuffers::bytes_for(Kc, Cc, S.n, S.B.rows);
}

// Pops parents for one step and makes room for their children.
static hipError_t prepare_step(Search &S, hipStream_t s)
{
    S.taken.clear();
    int64_t K = 0, nch = 0;
    while (!S.runs.empty()) {
        auto &r = S.runs.back();
        const int64_t c = S.n - r.first;
        int64_t x = (S.pool_cap - nch) / c;
        if (K == 0) x = std::max<int64_t>(x, 1);
        x = std::min(x, r.second);
        if (x <= 0) break;
        S.taken.push_back({r.first, x});
        K += x;
        nch += x * c;
        r.second -= x;
        if (r.second > 0) break;
        S.runs.pop_back();
    }
    S.K = K;
    S.nch = nch;
    S.base = S.top - K;
    if (S.base + nch > S.cap_stack) {
        int64_t nc = S.cap_stack;
        while (S.base + nch > nc) nc *= 2;
        int32_t *r2 = nullptr, *d2 = nullptr;
        hipError_t e = stream_alloc((void **)&r2, (size_t)nc * S.n * 4, s);
        if (e == hipSuccess) e = stream_alloc((void **)&d2, (size_t)nc * 4, s);
        if (e == hipSuccess) e = hipMemcpyAsync(r2, S.srows, (size_t)S.top * S.n * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d2, S.sdep, (size_t)S.top * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            if (r2) stream_free(r2, s);
            if (d2) stream_free(d2, s);
            return e;
        }
        stream_free(S.srows, s);
        stream_free(S.sdep, s);
        S.srows = r2;
        S.sdep = d2;
        S.cap_stack = nc;
    }
    hipError_t e = S.B.ensure_k(std::max(S.pool_cap, K), s);
    if (e == hipSuccess) e = S.B.ensure_c(std::max(S.pool_cap, nch), S.n, s);  // one parent may exceed pool_cap
    return e;
}

namespace {
// Request table of a step: StepReq[R] (with their results), the phase-1 scan
// segments, the metadata of a merged bound launch (meta bytes, possibly 0),
// then the survivor counts of every popped parent.  Everything before surv
// goes up in one copy.
struct TabLayout {
    size_t req, seg1, meta, surv, total;
    TabLayout(int R, int64_t sumK, size_t meta_bytes = 0)
    {
        req = 0;
        seg1 = al256(sizeof(StepReq) * R);
        meta = seg1 + al256(sizeof(ScanSeg) * R);
        surv = meta + al256(meta_bytes);
        total = surv + al256((size_t)std::max<int64_t>(sumK, 1) * 4);
    }
};

// Points the request's scalar outputs at its entry of the device table.
void point_results(StepReq &q, StepReq *dq_entry)
{
    q.w.best = &dq_entry->res.best;
    q.w.fingerprint = &dq_entry->res.fingerprint;
    q.w.bad = &dq_entry->res.bad;
    q.w.nchild = &dq_entry->res.nchild;
    q.w.nsurv = &dq_entry->res.nsurv;
}

// point_results, and the initial values in the host image.
void bind_results(StepReq &q, StepReq *dq_entry, int32_t ub_in)
{
    q.res = StepResultDev{};
    q.res.best = ((unsigned long long)(uint32_t)ub_in << 32) | 0xffffffffull;
    point_results(q, dq_entry);
}
}  // namespace

// ---------------------------------------------------------------- children of parents

hipError_t bound_children_of(fsp_instance_s *I, const int32_t *parents, const int32_t *pdepth, int64_t K,
                             int64_t nch, StepBuffers &B, Kids16 &kids, TickContext &ctx, hipStream_t s)
{
    if (K <= 0 || nch <= 0) return hipSuccess;
    const int n = I->n;
    B.rows = !kids16_eligible(I);
    hipError_t e = B.ensure_k(K, s);
    if (e == hipSuccess) e = B.ensure_c(nch, n, s);
    KidsStep ks(kids);
    if (e == hipSuccess) e = ks.start(I, K, nch, s);
    const TabLayout L(1, K);
    if (e == hipSuccess) e = ctx.reserve(L.total);
    if (e != hipSuccess) return e;
    char *h = (char *)ctx.htab, *d = (char *)ctx.dtab;
    StepReq *dentry = (StepReq *)(d + L.req);
    StepReq q;
    std::memset(&q, 0, sizeof(q));
    q.a.n = n;
    q.a.ub_in = 0x7fffffff;
    q.a.parents = parents;
    q.a.pdepth = pdepth;
    q.a.K = K;
    q.w = B.w;
    if (ks.on) kids16_point(q.w, ks.k);
    q.T = I->dt;
    q.nchild = nch;
    bind_results(q, dentry, 0x7fffffff);
    *(StepReq *)(h + L.req) = q;
    *(ScanSeg *)(h + L.seg1) = ScanSeg{q.w.cnt, q.w.off, K, q.w.nchild, B.sums_k};
    e = hipMemcpyAsync(d, h, L.surv, hipMemcpyHostToDevice, s);
    bool leaves_done = false;
    if (e == hipSuccess)
        e = phase1_and_bound1(dentry, (const ScanSeg *)(d + L.seg1), I, ks, K, nch, q.w, s, &leaves_done);
    return e;
}

size_t tick_scratch_after(const std::vector<Search *> &sel, const std::vector<StepSel> &qs, const TickContext &ctx)
{
    const int R = (int)sel.size();
    size_t kids_need = 0;
    int64_t sumK = 0;
    std::vector<fsp_pool_desc> descs;
    std::vector<Workspace16> ready;
    for (int r = 0; r < R; ++r) {
        const Search &S = *sel[r];
        sumK += qs[r].K;
        const bool k = kids16_eligible(S.inst) && qs[r].nch > 0;
        if (k) kids_need += KidsArena::step_bytes(S.inst, qs[r].K, qs[r].nch);
        if (R > 1 && S.inst->packed16) {
            // only sizes matter to the plan; a non-null dec marks a decoded pool
            descs.push_back(fsp_pool_desc{S.inst, nullptr, nullptr, qs[r].nch, nullptr});
            Workspace16 w{};
            if (k) w.dec = reinterpret_cast<uint32_t *>(uintptr_t(256));
            ready.push_back(w);
        }
    }
    size_t arena = ctx.arena.dev_bytes, meta = 0;
    if (!descs.empty()) {
        BatchPlan pl;
        plan_batch(descs.data(), (int32_t)descs.size(), 0, false, pl, -1, ready.data());
        arena = ctx.arena.bytes_after(pl.ws_bytes);
        meta = pl.meta_bytes;
    }
    const size_t tab = TabLayout(R, sumK, meta).total;
    const size_t dcap = tab > ctx.dcap ? std::max(tab, (size_t)64 * 1024) : ctx.dcap;
    return dcap + arena + (kids_need ? ctx.kids.cap_after(kids_need) : ctx.kids.cap);
}

hipError_t tick(std::vector<Search *> &act, TickContext &ctx)
{
    hipStream_t s = ctx.s;
    const int R = (int)act.size();
    if (R == 0) return hipSuccess;
    int64_t maxK = 0, maxC = 0, sumK = 0;
    for (Search *S : act) {
        hipError_t e = prepare_step(*S, s);
        if (e != hipSuccess) return e;
        maxK = std::max(maxK, S->K);
        maxC = std::max(maxC, S->nch);
        sumK += S->K;
    }
    hipError_t e = hipSuccess;
    // searches on the 16-bit path with the plain releases bound their
    // children from their parents; the others from child rows
    std::vector<int> kid_of(R, -1);  // index into kv, or -1 (child rows)
    std::vector<const fsp_instance_s *> kI;
    std::vector<int64_t> kKs, kCs;
    int64_t kK = 0, kC = 0;
    int knmax = 0, kmmax = 0;
    bool any_rows = false;
    for (int r = 0; r < R; ++r) {
        Search &S = *act[r];
        if (kids16_eligible(S.inst) && S.nch > 0) {
            kid_of[r] = (int)kI.size();
            kI.push_back(S.inst);
            kKs.push_back(S.K);
            kCs.push_back(S.nch);
            kK = std::max(kK, S.K);
            kC = std::max(kC, S.nch);
            knmax = std::max(knmax, S.n);
            kmmax = std::max(kmmax, (int)S.inst->m);
        } else {
            any_rows = true;
        }
    }
    std::vector<Kids16> kv;
    if (!kI.empty()) {
        e = ctx.kids.layout(kI, kKs, kCs, kv, s);
        if (e != hipSuccess) return e;
    }
    // a merged step bounds its 16-bit searches in one batched launch, planned
    // here so that its metadata goes up with the request table
    std::vector<fsp_pool_desc> descs;
    std::vector<Workspace16> ready;
    size_t meta_bytes = 0;
    if (R > 1) {
        descs.reserve(R);
        ready.reserve(R);
        for (int r = 0; r < R; ++r) {
            Search *S = act[r];
            if (!S->inst->packed16) continue;
            const bool k = kid_of[r] >= 0;
            descs.push_back(fsp_pool_desc{S->inst, k ? nullptr : S->B.w.crow, S->B.w.cdepth, S->nch, S->B.w.clb});
            ready.push_back(k ? kv[kid_of[r]].W : Workspace16{});
        }
        if (!descs.empty()) e = ctx.arena.plan_only(descs.data(), (int32_t)descs.size(), s, ready.data(), &meta_bytes);
        if (e != hipSuccess) return e;
    }
    const TabLayout L(R, sumK, meta_bytes);
    e = ctx.reserve(L.total);
    if (e != hipSuccess) return e;
    char *h = (char *)ctx.htab, *d = (char *)ctx.dtab;
    if (meta_bytes) ctx.arena.stage(d + L.meta, h + L.meta);
    StepReq *hq = (StepReq *)(h + L.req);
    ScanSeg *hs1 = (ScanSeg *)(h + L.seg1);
    int64_t slot = 0;
    std::vector<int64_t> slots(R);
    for (int r = 0; r < R; ++r) {
        Search &S = *act[r];
        StepReq q;
        std::memset(&q, 0, sizeof(q));
        q.a.n = S.n;
        q.a.ub_in = S.UB;
        q.a.parents = S.srows;
        q.a.pdepth = S.sdep;
        q.a.K = S.K;
        q.a.parents_reversed = 1;
        q.a.parent_top = S.top;
        q.a.out_rows = S.srows;
        q.a.out_depth = S.sdep;
        q.a.out_lb = nullptr;
        q.a.out_base = S.base;
        q.a.out_cap = S.cap_stack;
        q.a.out_reversed = 1;
        q.a.surv_per_parent = (uint32_t *)(d + L.surv) + slot;
        q.a.incumbent = S.dinc;
        q.w = S.B.w;
        if (kid_of[r] >= 0) kids16_point(q.w, kv[kid_of[r]]);
        q.T = S.inst->dt;
        q.nchild = S.nch;
        bind_results(q, (StepReq *)(d + L.req) + r, S.UB);
        slots[r] = slot;
        slot += S.K;
        hq[r] = q;
        hs1[r] = ScanSeg{q.w.cnt, q.w.off, S.K, q.w.nchild, S.B.sums_k};
    }
    const StepReq *dq = (const StepReq *)(d + L.req);
    const ScanSeg *ds1 = (const ScanSeg *)(d + L.seg1);
    e = hipMemcpyAsync(d, h, L.surv, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    if (!any_rows) {
        // every search decodes its children from its parents: validation,
        // counts and child lists are folded into those launches
        e = kids16_decode(dq, R, kK, kC, knmax, kmmax, s, ds1);
    } else {
        e = mstep_phase1(dq, ds1, R, maxK, s);
        // branching: job lists for all, child rows for the searches without
        // the incremental path; the others decode their children from their parents
        if (e == hipSuccess) e = mstep_branch(dq, R, maxK, maxC, s);
        if (e == hipSuccess && kK > 0) e = kids16_decode(dq, R, kK, kC, knmax, kmmax, s);
    }
    if (e != hipSuccess) return e;
    // bounding: one plain launch for a search alone, else one merged batch
    // (decoded workspaces go straight to its scan)
    if (R == 1) {
        Search &S = *act[0];
        e = kid_of[0] >= 0 ? launch_scan16(S.inst, kv[0].W, S.nch, S.B.w.clb, s, scan_splits_for(S.inst, S.nch))
                           : bound_rows(S.inst, S.B.w.crow, S.B.w.cdepth, S.nch, S.B.w.clb, s, false);
    } else {
        for (int r = 0; r < R && e == hipSuccess; ++r) {
            Search *S = act[r];
            if (!S->inst->packed16) e = bound_rows(S->inst, S->B.w.crow, S->B.w.cdepth, S->nch, S->B.w.clb, s);
        }
        if (e == hipSuccess && !descs.empty()) e = ctx.arena.launch(s);
    }
    if (e == hipSuccess) e = mstep_finish(dq, R, maxK, maxC, s, !any_rows);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, L.total, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;

    const uint32_t *hsurv = (const uint32_t *)(h + L.surv);
    bool copies = false;
    for (int r = 0; r < R; ++r) {
        Search &S = *act[r];
        const StepResultDev o = hq[r].res;
        if (o.bad || (int64_t)o.nchild != S.nch) {
            S.done = true;
            S.status = FSP_E_BADNODE;
            continue;
        }
        S.nodes += S.nch;
        const uint32_t idx = (uint32_t)(o.best & 0xffffffffu);
        if (idx != 0xffffffffu) {
            S.UB = (int32_t)(o.best >> 32);
            ++S.improvements;
            e = hipMemcpyAsync(S.inc.data(), S.dinc, (size_t)S.n * 4, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return e;
            copies = true;
        }
        // survivors sit bottom-to-top as: children of the last popped parent ... of the first
        const uint32_t *sv = hsurv + slots[r];
        int64_t p = S.K;
        for (auto it = S.taken.rbegin(); it != S.taken.rend(); ++it) {
            for (int64_t x = 0; x < it->second; ++x) {
                --p;
                const int64_t cnt = sv[p];
                if (!cnt) continue;
                const int32_t dd = it->first + 1;
                if (!S.runs.empty() && S.runs.back().first == dd) S.runs.back().second += cnt;
                else S.runs.push_back({dd, cnt});
            }
        }
        S.top = S.base + o.nsurv;
        S.max_stack = std::max(S.max_stack, S.top);
        if (S.steplog && S.steps < S.steplog_cap) {
            int64_t *Lg = S.steplog + S.steps * 6;
            Lg[0] = S.K; Lg[1] = S.nch; Lg[2] = S.UB; Lg[3] = o.nsurv; Lg[4] = S.top; Lg[5] = (int64_t)o.fingerprint;
        }
        ++S.steps;
        if (S.top == 0) {
            S.done = true;
            S.status = FSP_OK;
        } else if (S.nodes >= S.node_budget) {
            S.done = true;
            S.status = FSP_BUDGET;
        }
    }
    if (copies) e = hipStreamSynchronize(s);
    return e;
}

// ---------------------------------------------------------------- device-chosen steps

hipError_t run_device_steps(Search &S, TickContext &ctx)
{
    hipStream_t s = ctx.s;
    fsp_instance_s *I = S.inst;
    const int n = S.n;
    // grids for the largest step: at most pool_cap parents, and pool_cap
    // children unless one parent alone has more (at most n)
    const int64_t maxK = S.pool_cap, maxC = std::max<int64_t>(S.pool_cap, n);
    hipError_t e = S.B.ensure_k(maxK, s);
    if (e == hipSuccess) e = S.B.ensure_c(maxC, n, s);
    std::vector<Kids16> kv;
    if (e == hipSuccess) e = ctx.kids.layout({I}, {maxK}, {maxC}, kv, s);
    if (e != hipSuccess) return e;
    // the request table of one search, then the device state, the selection's
    // chunk sums and the step log
    const TabLayout L(1, maxK, 0);
    const int nchunks = (int)((maxK + kDevSelChunk - 1) / kDevSelChunk);
    const size_t off_ds = L.total, off_sums = off_ds + al256(sizeof(DevSearch)),
                 off_log = off_sums + al256((size_t)nchunks * 8);
    const int64_t logcap = S.steplog ? S.steplog_cap : 0;
    e = ctx.reserve(off_log + al256((size_t)std::max<int64_t>(logcap, 1) * 6 * 8));
    if (e != hipSuccess) return e;
    char *h = (char *)ctx.htab, *d = (char *)ctx.dtab;
    StepReq *dq = (StepReq *)(d + L.req);
    ScanSeg *ds1 = (ScanSeg *)(d + L.seg1);
    DevSearch *dds = (DevSearch *)(d + off_ds);
    int64_t *dsums = (int64_t *)(d + off_sums);
    int64_t *dlog = logcap ? (int64_t *)(d + off_log) : nullptr;

    // the table's fixed fields (the selection writes the sizes of each step)
    auto upload_table = [&]() -> hipError_t {
        StepReq q;
        std::memset(&q, 0, sizeof(q));
        q.a.n = n;
        q.a.ub_in = S.UB;
        q.a.parents = S.srows;
        q.a.pdepth = S.sdep;
        q.a.parents_reversed = 1;
        q.a.parent_top = S.top;
        q.a.out_rows = S.srows;
        q.a.out_depth = S.sdep;
        q.a.out_cap = S.cap_stack;
        q.a.out_reversed = 1;
        q.a.surv_per_parent = (uint32_t *)(d + L.surv);
        q.a.incumbent = S.dinc;
        q.w = S.B.w;
        kids16_point(q.w, kv[0]);
        q.T = I->dt;
        bind_results(q, dq, S.UB);
        *(StepReq *)(h + L.req) = q;
        *(ScanSeg *)(h + L.seg1) = ScanSeg{q.w.cnt, q.w.off, 0, q.w.nchild, S.B.sums_k};
        return hipMemcpyAsync(d, h, L.surv, hipMemcpyHostToDevice, s);
    };
    DevSearch st{};
    st.top = S.top;
    st.nodes = S.nodes;
    st.steps = S.steps;
    st.max_stack = S.max_stack;
    st.node_budget = S.node_budget;
    st.pool_cap = S.pool_cap;
    st.maxK = maxK;
    st.maxC = maxC;
    st.cap_stack = S.cap_stack;
    st.steplog_cap = logcap;
    st.UB = S.UB;
    st.improvements = S.improvements;
    st.done = S.done ? 1 : 0;
    st.status = S.status;
    st.n = n;
    st.paused = 0;
    auto upload_state = [&]() -> hipError_t {
        std::memcpy(h + off_ds, &st, sizeof(st));
        return hipMemcpyAsync(dds, h + off_ds, sizeof(st), hipMemcpyHostToDevice, s);
    };
    e = upload_state();
    if (e == hipSuccess) e = upload_table();
    // steps per synchronisation: 1, 2, 4, ... up to 16, and fewer when the
    // steps are large (at most about 2^20 children per synchronisation), so
    // that a search does not run many empty steps after its end
    const int chunk_max = (int)std::max<int64_t>(1, std::min<int64_t>(16, ((int64_t)1 << 20) / maxC));
    const int splits = scan_splits_for(I, maxC);  // for the largest step
    int chunk = 1;
    while (e == hipSuccess && !st.done) {
        // the device pauses a search whose next step might not fit the stack
        // (maxC more rows): grow it, doubling, until the coming chunk of
        // steps fits whole (a pause idles the rest of its chunk), and resume
        const int64_t need = st.top + (int64_t)chunk * maxC;
        if (st.paused || need > S.cap_stack) {
            int64_t nc = S.cap_stack;
            while (need > nc) nc *= 2;
            if (nc > S.cap_stack) {
                int32_t *r2 = nullptr, *d2 = nullptr;
                e = stream_alloc((void **)&r2, (size_t)nc * n * 4, s);
                if (e == hipSuccess) e = stream_alloc((void **)&d2, (size_t)nc * 4, s);
                if (e == hipSuccess) e = hipMemcpyAsync(r2, S.srows, (size_t)st.top * n * 4, hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess) e = hipMemcpyAsync(d2, S.sdep, (size_t)st.top * 4, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) {
                    if (r2) stream_free(r2, s);
                    if (d2) stream_free(d2, s);
                    break;
                }
                stream_free(S.srows, s);
                stream_free(S.sdep, s);
                S.srows = r2;
                S.sdep = d2;
                S.cap_stack = nc;
                e = upload_table();
                if (e != hipSuccess) break;
            }
            st.cap_stack = S.cap_stack;
            st.paused = 0;
            e = upload_state();
            if (e != hipSuccess) break;
        }
        for (int k = 0; k < chunk && e == hipSuccess; ++k) {
            e = launch_device_step_select(dds, S.sdep, dsums, nchunks, dq, ds1, s);
            if (e == hipSuccess) e = kids16_decode(dq, 1, maxK, maxC, n, I->m, s, ds1);
            if (e == hipSuccess) e = launch_scan16(I, kv[0].W, maxC, S.B.w.clb, s, splits, &dq->nchild);
            if (e == hipSuccess) e = mstep_finish(dq, 1, maxK, maxC, s, true);
            if (e == hipSuccess) e = launch_device_step_update(dds, dq, dlog, s);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(h + off_ds, dds, sizeof(st), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) std::memcpy(&st, h + off_ds, sizeof(st));
        chunk = std::min(2 * chunk, chunk_max);
    }
    if (e != hipSuccess) return e;
    S.top = st.top;
    S.nodes = st.nodes;
    S.steps = st.steps;
    S.max_stack = st.max_stack;
    S.UB = st.UB;
    S.improvements = st.improvements;
    S.done = true;
    S.status = st.status;
    S.runs.clear();  // the host view of the stack is not kept in this mode
    if (S.improvements > 0) e = hipMemcpyAsync(S.inc.data(), S.dinc, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    const int64_t nlog = std::min(S.steps, logcap);
    if (e == hipSuccess && nlog > 0)
        e = hipMemcpyAsync(S.steplog, dlog, (size_t)nlog * 6 * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// ---------------------------------------------------------------- best first

namespace {

// Device state of a best-first search: the row slab, the free-slot stack, the
// frontier records (ping-pong), and the per-step survivor and sort buffers.
struct BestFirst {
    hipStream_t s = nullptr;
    int n = 0;
    int64_t C = 0;              // slots
    int32_t *slab = nullptr;    // C x n
    int32_t *fl = nullptr;      // C: free slots, the top nfree in use
    int32_t *rec[2] = {nullptr, nullptr};  // each 3 x C: bound, depth, slot
    int64_t nfree = 0;
    int64_t Scap = 0;           // survivor buffers: depth, bound, keys, ranks, sorted keys, sorted ranks
    int32_t *sbuf = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int64_t *sel = nullptr;     // 3 scalars of the selection
    int32_t *dinc = nullptr;

    Frontier F(int i) const { return Frontier{rec[i], rec[i] + C, rec[i] + 2 * C}; }
    int32_t *S(int k) const { return sbuf + (size_t)k * Scap; }

    hipError_t alloc(int64_t slots)
    {
        C = slots;
        hipError_t e = stream_alloc((void **)&slab, (size_t)C * n * 4, s);
        if (e == hipSuccess) e = stream_alloc((void **)&fl, (size_t)C * 4, s);
        if (e == hipSuccess) e = stream_alloc((void **)&rec[0], (size_t)C * 12, s);
        if (e == hipSuccess) e = stream_alloc((void **)&rec[1], (size_t)C * 12, s);
        if (e == hipSuccess) e = stream_alloc((void **)&sel, 64, s);
        if (e == hipSuccess) e = stream_alloc((void **)&dinc, (size_t)n * 4, s);
        return e;
    }

    // Room for `need` more rows: double the slot count until it fits, keep
    // every slot's row, the live records of frontier `cur` and the free stack.
    hipError_t grow(int64_t need, int cur, int64_t M)
    {
        if (nfree >= need) return hipSuccess;
        int64_t C2 = C;
        while (nfree + (C2 - C) < need) C2 *= 2;
        int32_t *slab2 = nullptr, *fl2 = nullptr, *r0 = nullptr, *r1 = nullptr;
        hipError_t e = stream_alloc((void **)&slab2, (size_t)C2 * n * 4, s);
        if (e == hipSuccess) e = stream_alloc((void **)&fl2, (size_t)C2 * 4, s);
        if (e == hipSuccess) e = stream_alloc((void **)&r0, (size_t)C2 * 12, s);
        if (e == hipSuccess) e = stream_alloc((void **)&r1, (size_t)C2 * 12, s);
        if (e != hipSuccess) return e;
        const Frontier a = F(cur), b{r0, r0 + C2, r0 + 2 * C2};
        e = hipMemcpyAsync(slab2, slab, (size_t)C * n * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(fl2, fl, (size_t)nfree * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = bf_fill_slots(fl2 + nfree, C2 - C, (int32_t)C, s);
        if (e == hipSuccess && M > 0) e = hipMemcpyAsync(b.lb, a.lb, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && M > 0) e = hipMemcpyAsync(b.depth, a.depth, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && M > 0) e = hipMemcpyAsync(b.slot, a.slot, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        stream_free(slab, s);
        stream_free(fl, s);
        stream_free(rec[0], s);
        stream_free(rec[1], s);
        slab = slab2;
        fl = fl2;
        rec[cur] = r0;
        rec[cur ^ 1] = r1;
        nfree += C2 - C;
        C = C2;
        return hipSuccess;
    }

    hipError_t ensure_survivors(int64_t cap)
    {
        if (cap <= Scap) return hipSuccess;
        if (sbuf) stream_free(sbuf, s);
        sbuf = nullptr;
        Scap = std::max<int64_t>(cap, 1024);
        hipError_t e = stream_alloc((void **)&sbuf, (size_t)Scap * 6 * 4, s);
        if (e != hipSuccess) Scap = 0;
        return e;
    }

    void release()
    {
        for (void *ptr : {(void *)slab, (void *)fl, (void *)rec[0], (void *)rec[1], (void *)sbuf, tmp, (void *)sel,
                          (void *)dinc})
            if (ptr) stream_free(ptr, s);
        slab = fl = nullptr;
        rec[0] = rec[1] = sbuf = dinc = nullptr;
        tmp = nullptr;
        sel = nullptr;
    }
};

// Pool-synchronous best-first search (Sec. III-A), with the frontier on the
// device.  Each step: drop the frontier records the upper bound eliminates,
// take parents from the front while their children fit in pool_cap (the
// first always), branch, bound and update the upper bound as the depth-first
// step does, then merge the survivors (child order kept on equal bounds) into
// the frontier.  Stops when the frontier is empty after the drop (proven) or
// the node budget is reached.
fsp_status best_first_solve(fsp_instance_s *inst, int32_t ub0, int64_t pool_cap, int64_t node_budget,
                            fsp_solve_result *res, int32_t *perm_out, int64_t *steplog, int64_t steplog_cap,
                            hipStream_t s)
{
    const int n = inst->n;
    std::vector<int32_t> inc(n, -1);
    int32_t UB = ub0 == FSP_UB_NEH ? neh(inst->p_host, n, inst->m, inc.data()) : ub0;
    const int32_t ub_start = UB;
    BestFirst bf;
    bf.s = s;
    bf.n = n;
    StepBuffers B;
    Kids16 kids;
    TickContext ctx;
    ctx.s = s;
    auto cleanup = [&]() {
        bf.release();
        B.release(s);
        kids16_release(kids, s);
        ctx.release();
    };
    // slots for sixteen pools of survivors before the first doubling (a
    // doubling allocates a slab twice the size and copies the rows: about 5 ms
    // at 200 x 20 with 262,144-child pools, where a step takes 0.8 ms)
    hipError_t e = bf.alloc(std::max<int64_t>(4096, 16 * pool_cap));
    // step buffers at their usual size up front (a parent with more children
    // than pool_cap grows them later)
    B.rows = !kids16_eligible(inst);
    if (e == hipSuccess) e = B.ensure_k(pool_cap, s);
    if (e == hipSuccess) e = B.ensure_c(pool_cap, n, s);
    if (e == hipSuccess) e = bf.ensure_survivors(pool_cap);
    // the root: slot 0 holds an all-zero row; record 0 = (bound, depth 0, slot 0)
    Frontier F0 = bf.F(0);
    if (e == hipSuccess) e = hipMemsetAsync(bf.slab, 0, (size_t)n * 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(F0.depth, 0, 4, s);
    if (e == hipSuccess) e = hipMemsetAsync(F0.slot, 0, 4, s);
    if (e == hipSuccess) e = bound_rows(inst, bf.slab, F0.depth, 1, F0.lb, s);
    int32_t lb0 = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&lb0, F0.lb, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { cleanup(); return fail_status(e); }
    int64_t M = lb0 < UB ? 1 : 0;
    e = bf_fill_slots(bf.fl, bf.C - M, (int32_t)M, s);
    bf.nfree = bf.C - M;
    int64_t nodes = 1, steps = 0, max_front = M;
    int32_t improvements = 0;
    int cur = 0;
    bool proven = false;
    while (e == hipSuccess) {
        int64_t sel[3] = {0, 0, 0};
        if (M > 0) {
            e = bf_select(bf.F(cur), M, UB, n, pool_cap, bf.sel, s);
            if (e == hipSuccess) e = hipMemcpyAsync(sel, bf.sel, sizeof(sel), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) break;
        }
        const int64_t Mp = sel[0], K = sel[1], nch = sel[2];
        if (Mp == 0) {
            proven = true;
            break;
        }
        if (nodes >= node_budget) break;
        const TabLayout L(1, 1);
        e = bf.grow(nch, cur, M);
        if (e == hipSuccess) e = B.ensure_k(K, s);
        if (e == hipSuccess) e = B.ensure_c(nch, n, s);
        if (e == hipSuccess) e = bf.ensure_survivors(nch);
        if (e == hipSuccess) e = ctx.reserve(L.total);
        if (e != hipSuccess) break;
        KidsStep ks(kids);
        e = ks.start(inst, K, nch, s);
        if (e != hipSuccess) break;
        const Frontier Fc = bf.F(cur), Fn = bf.F(cur ^ 1);
        char *h = (char *)ctx.htab, *d = (char *)ctx.dtab;
        StepReq *dentry = (StepReq *)(d + L.req);
        StepReq q;
        std::memset(&q, 0, sizeof(q));
        q.a.n = n;
        q.a.ub_in = UB;
        q.a.parents = bf.slab;
        q.a.pslot = Fc.slot;
        q.a.pdepth = Fc.depth;
        q.a.K = K;
        q.a.out_rows = bf.slab;
        q.a.oslot = bf.fl + bf.nfree - 1;
        q.a.oslot_step = -1;
        q.a.out_depth = bf.S(0);
        q.a.out_lb = bf.S(1);
        q.a.out_base = 0;
        q.a.out_cap = nch;
        q.a.incumbent = bf.dinc;
        q.w = B.w;
        if (ks.on) kids16_point(q.w, ks.k);
        q.T = inst->dt;
        q.nchild = nch;
        bind_results(q, dentry, UB);
        *(StepReq *)(h + L.req) = q;
        *(ScanSeg *)(h + L.seg1) = ScanSeg{q.w.cnt, q.w.off, K, q.w.nchild, B.sums_k};
        const uint32_t *dnsurv = &dentry->res.nsurv;
        e = hipMemcpyAsync(d, h, L.surv, hipMemcpyHostToDevice, s);
        bool leaves_done = false;
        // parents of mixed depths: the row path sorts its children by depth
        if (e == hipSuccess)
            e = phase1_and_bound1(dentry, (const ScanSeg *)(d + L.seg1), inst, ks, K, nch, q.w, s, &leaves_done);
        if (e == hipSuccess) e = mstep_finish(dentry, 1, K, nch, s, leaves_done);
        if (e == hipSuccess)
            e = bf_sort_survivors(bf.S(1), dnsurv, nch, UB, bf.S(2), bf.S(3), bf.S(4), bf.S(5), &bf.tmp,
                                  &bf.tmp_bytes, s);
        if (e == hipSuccess)
            e = bf_merge(Fc, K, Mp - K, bf.S(4), bf.S(5), bf.S(0), dnsurv, nch, bf.fl, bf.nfree, Fn, s);
        if (e == hipSuccess) e = bf_free_slots(Fc, K, Mp, M, bf.fl, bf.nfree, dnsurv, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h + L.req, d + L.req, sizeof(StepReq), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        const StepResultDev o = ((const StepReq *)(h + L.req))->res;
        if (o.bad || (int64_t)o.nchild != nch) {
            cleanup();
            return FSP_E_BADNODE;
        }
        const int64_t S = o.nsurv;
        nodes += nch;
        const uint32_t idx = (uint32_t)(o.best & 0xffffffffu);
        if (idx != 0xffffffffu) {
            UB = (int32_t)(o.best >> 32);
            ++improvements;
            e = hipMemcpyAsync(inc.data(), bf.dinc, (size_t)n * 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) break;
        }
        bf.nfree = bf.nfree - S + K + (M - Mp);
        M = (Mp - K) + S;
        cur ^= 1;
        max_front = std::max(max_front, M);
        if (steplog && steps < steplog_cap) {
            int64_t *Lg = steplog + steps * 6;
            Lg[0] = K; Lg[1] = nch; Lg[2] = UB; Lg[3] = S; Lg[4] = M; Lg[5] = (int64_t)o.fingerprint;
        }
        ++steps;
    }
    cleanup();
    if (e != hipSuccess) return fail_status(e);
    res->opt = UB;
    res->proven = proven ? 1 : 0;
    res->nodes_bounded = nodes;
    res->steps = steps;
    res->ub0 = ub_start;
    res->improvements = improvements;
    res->max_stack = max_front;
    if (perm_out) std::copy(inc.begin(), inc.end(), perm_out);
    return proven ? FSP_OK : FSP_BUDGET;
}

}  // namespace

}  // namespace fspbb

extern "C" {

fsp_status fsp_neh(fsp_instance inst, int32_t *perm_out, int32_t *makespan)
{
    if (!inst || !makespan) return FSP_E_INVAL;
    *makespan = neh(inst->p_host, inst->n, inst->m, perm_out);
    return FSP_OK;
}

fsp_status fsp_branch_and_prune(fsp_instance inst, const int32_t *parents, const int32_t *parent_depths, int64_t K,
                                int32_t ub_in, int32_t *children, int32_t *child_depths, int32_t *child_lb,
                                int64_t cap, int32_t *incumbent, fsp_step_result *res, void *stream)
{
    if (!inst || !res || K < 0 || cap < 0 || ub_in < 0) return FSP_E_INVAL;
    std::memset(res, 0, sizeof(*res));
    res->ub_out = ub_in;
    if (K == 0) return FSP_OK;
    if (!parents || !parent_depths || (cap > 0 && (!children || !child_depths))) return FSP_E_INVAL;
    DeviceGuard g(inst->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    StepBuffers B;
    Kids16 kids;
    TickContext ctx;
    ctx.s = s;
    auto cleanup = [&]() {
        B.release(s);
        kids16_release(kids, s);
        ctx.release();
    };
    const TabLayout L(1, K);
    B.rows = !kids16_eligible(inst);
    hipError_t e = B.ensure_k(K, s);
    if (e == hipSuccess) e = B.ensure_c(1, inst->n, s);
    if (e == hipSuccess) e = ctx.reserve(L.total);
    if (e != hipSuccess) { cleanup(); return fail_status(e); }
    StepReq q;
    std::memset(&q, 0, sizeof(q));
    q.a.n = inst->n;
    q.a.ub_in = ub_in;
    q.a.parents = parents;
    q.a.pdepth = parent_depths;
    q.a.K = K;
    q.a.out_rows = children;
    q.a.out_depth = child_depths;
    q.a.out_lb = child_lb;
    q.a.out_base = 0;
    q.a.out_cap = cap;
    q.a.incumbent = incumbent;
    q.w = B.w;
    q.T = inst->dt;
    char *h = (char *)ctx.htab, *d = (char *)ctx.dtab;
    StepReq *dentry = (StepReq *)(d + L.req);
    const StepReq *dq = dentry;
    bind_results(q, dentry, ub_in);
    *(StepReq *)(h + L.req) = q;
    *(ScanSeg *)(h + L.seg1) = ScanSeg{q.w.cnt, q.w.off, K, q.w.nchild, B.sums_k};
    e = hipMemcpyAsync(d, h, L.surv, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = mstep_phase1(dq, (const ScanSeg *)(d + L.seg1), 1, K, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + L.req, d + L.req, sizeof(StepReq), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    uint32_t nchild = 0;
    if (e == hipSuccess) {
        nchild = ((const StepReq *)(h + L.req))->res.nchild;
        e = B.ensure_c(nchild, inst->n, s);  // the child scratch may move; phase-1 results stay
    }
    if (e != hipSuccess) { cleanup(); return fail_status(e); }
    const StepResultDev after1 = ((const StepReq *)(h + L.req))->res;
    KidsStep ks(kids);
    e = ks.start(inst, K, nchild, s);
    if (e != hipSuccess) { cleanup(); return fail_status(e); }
    q.w = B.w;
    if (ks.on) kids16_point(q.w, ks.k);
    point_results(q, dentry);
    q.res = after1;
    q.nchild = nchild;
    *(StepReq *)(h + L.req) = q;
    e = hipMemcpyAsync(d, h, L.surv, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = branch_and_bound1(dq, inst, ks, K, nchild, q.w, s, true);
    if (e == hipSuccess) e = mstep_finish(dq, 1, K, nchild, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + L.req, d + L.req, sizeof(StepReq), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { cleanup(); return fail_status(e); }
    const StepResultDev o = ((const StepReq *)(h + L.req))->res;
    cleanup();
    res->n_children = nchild;
    res->n_survivors = o.nsurv;
    const uint32_t idx = (uint32_t)(o.best & 0xffffffffu);
    res->improved = idx != 0xffffffffu;
    res->ub_out = (int32_t)(o.best >> 32);
    res->fingerprint = (int64_t)o.fingerprint;
    if (o.bad) return FSP_E_BADNODE;
    if ((int64_t)o.nsurv > cap) return FSP_E_RANGE;
    return FSP_OK;
}

fsp_status fsp_solve(fsp_instance inst, int32_t ub0, int64_t pool_cap, int64_t node_budget,
                     fsp_solve_result *res, int32_t *perm_out, int64_t *steplog, int64_t steplog_cap,
                     void *stream)
{
    return fsp_solve_ex(inst, ub0, pool_cap, node_budget, 0, res, perm_out, steplog, steplog_cap, stream);
}

fsp_status fsp_solve_ex(fsp_instance inst, int32_t ub0, int64_t pool_cap, int64_t node_budget, int32_t flags,
                        fsp_solve_result *res, int32_t *perm_out, int64_t *steplog, int64_t steplog_cap,
                        void *stream)
{
    if (!inst || !res || pool_cap < 1 || node_budget < 1 || (ub0 < 0 && ub0 != FSP_UB_NEH)) return FSP_E_INVAL;
    if (flags & ~(FSP_SOLVE_BEST_FIRST | FSP_SOLVE_DEVICE_STEPS)) return FSP_E_INVAL;
    if ((flags & FSP_SOLVE_BEST_FIRST) && (flags & FSP_SOLVE_DEVICE_STEPS)) return FSP_E_INVAL;
    std::memset(res, 0, sizeof(*res));
    DeviceGuard g(inst->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    if (flags & FSP_SOLVE_BEST_FIRST)
        return best_first_solve(inst, ub0, pool_cap, node_budget, res, perm_out, steplog, steplog ? steplog_cap : 0,
                                s);
    Search S;
    TickContext ctx;
    ctx.s = s;
    auto cleanup = [&]() {
        S.release(s);
        ctx.release();
    };
    hipError_t e = S.start(inst, ub0, pool_cap, node_budget, s);
    if (e != hipSuccess) { cleanup(); return fail_status(e); }
    S.steplog = steplog;
    S.steplog_cap = steplog ? steplog_cap : 0;
    std::vector<Search *> act{&S};
    if ((flags & FSP_SOLVE_DEVICE_STEPS) && kids16_eligible(inst) && !S.done) {
        e = run_device_steps(S, ctx);
        if (e != hipSuccess) { cleanup(); return fail_status(e); }
    }
    while (!S.done) {
        e = tick(act, ctx);
        if (e != hipSuccess) { cleanup(); return fail_status(e); }
    }
    cleanup();
    if (S.status != FSP_OK && S.status != FSP_BUDGET) return S.status;
    S.result(res, perm_out);
    return res->proven ? FSP_OK : FSP_BUDGET;
}

}  // extern "C"
