// Host side of the branch-and-bound: the C ABI step call, the NEH initial
// upper bound, and the depth-first solve loop that keeps the search stack on
// the device.
//
// The solve is pool-synchronous (Sec. III-A: the CPU selects a pool, the GPU
// bounds it): each step pops parents from the top of the stack while their
// children fit in pool_cap (the first parent is always taken), branches them
// in pop order with children in increasing job id, bounds every child,
// lowers the upper bound with the best complete child (the first in child
// order on ties), and pushes the children whose bound is below the upper
// bound in reverse child order, so the first child is popped first.  With a
// fixed (instance, initial upper bound, pool_cap) every count is a
// deterministic function of the search, step by step.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bnb.h"
#include "scan.h"

using namespace fspbb;

namespace {

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

// Owns the device scratch of steps with up to Kcap parents and Ccap children.
struct StepBuffers {
    StepScratch w{};
    void *blob = nullptr;
    int64_t Kcap = 0, Ccap = 0;
    int n = 0;

    hipError_t ensure(int64_t K, int64_t C, int n_, hipStream_t s)
    {
        if (K <= Kcap && C <= Ccap && n_ == n && blob) return hipSuccess;
        release(s);
        Kcap = std::max<int64_t>(K, 1);
        Ccap = std::max<int64_t>(C, 1);
        n = n_;
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t kb = al((size_t)Kcap * 4), cb = al((size_t)Ccap * 4);
        const size_t rows = al((size_t)Ccap * n * 4);
        const size_t scan = al(scan_scratch_bytes(std::max(Kcap, Ccap)));
        const size_t total = 2 * kb + 6 * cb + rows + scan + 256 * 2;
        hipError_t e = hipMallocAsync(&blob, total, s);
        if (e != hipSuccess) { blob = nullptr; Kcap = Ccap = 0; return e; }
        char *p = (char *)blob;
        w.cnt = (uint32_t *)p; p += kb;
        w.off = (uint32_t *)p; p += kb;
        w.ujob = (int32_t *)p; p += cb;
        w.upar = (int32_t *)p; p += cb;
        w.cdepth = (int32_t *)p; p += cb;
        w.clb = (int32_t *)p; p += cb;
        w.keep = (uint32_t *)p; p += cb;
        w.pos = (uint32_t *)p; p += cb;
        w.crow = (int32_t *)p; p += rows;
        w.scan_scratch = p; p += scan;
        w.nchild = (uint32_t *)p;
        w.nsurv = (uint32_t *)(p + 4);
        w.best = (unsigned long long *)(p + 64);
        w.fingerprint = (unsigned long long *)(p + 128);
        w.bad = (unsigned long long *)(p + 192);
        return hipSuccess;
    }
    void release(hipStream_t s)
    {
        if (blob) hipFreeAsync(blob, s);
        blob = nullptr;
        Kcap = Ccap = 0;
    }
};

// Scalars read back after each step.
struct StepOut {
    uint32_t nchild, nsurv;
    unsigned long long best, fingerprint, bad;
};

hipError_t read_step_out(const StepScratch &w, StepOut &o, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(&o.nchild, w.nchild, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&o.nsurv, w.nsurv, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&o.best, w.best, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&o.fingerprint, w.fingerprint, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&o.bad, w.bad, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

fsp_status fail(hipError_t e)
{
    set_last_error(e);
    return e == hipErrorOutOfMemory ? FSP_E_NOMEM : FSP_E_DEVICE;
}

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

}  // namespace

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
    hipError_t e = B.ensure(K, 1, inst->n, s);
    if (e != hipSuccess) return fail(e);
    StepArgs a{};
    a.n = inst->n;
    a.ub_in = ub_in;
    a.parents = parents;
    a.pdepth = parent_depths;
    a.K = K;
    a.out_rows = children;
    a.out_depth = child_depths;
    a.out_lb = child_lb;
    a.out_base = 0;
    a.out_cap = cap;
    a.incumbent = incumbent;
    e = step_phase1(a, B.w, s);
    StepOut o{};
    if (e == hipSuccess) e = read_step_out(B.w, o, s);
    if (e != hipSuccess) { B.release(s); return fail(e); }
    const int64_t nchild = o.nchild;
    e = B.ensure(K, nchild, inst->n, s);
    if (e == hipSuccess) e = step_phase1(a, B.w, s);  // the scratch may have moved
    if (e == hipSuccess) e = step_phase2(inst, a, B.w, nchild, s);
    if (e == hipSuccess) e = read_step_out(B.w, o, s);
    B.release(s);
    hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return fail(e);
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
    if (!inst || !res || pool_cap < 1 || node_budget < 1 || (ub0 < 0 && ub0 != FSP_UB_NEH)) return FSP_E_INVAL;
    std::memset(res, 0, sizeof(*res));
    DeviceGuard g(inst->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int n = inst->n;
    std::vector<int32_t> inc(n, -1);
    int32_t UB = ub0;
    if (ub0 == FSP_UB_NEH) UB = neh(inst->p_host, n, inst->m, inc.data());
    res->ub0 = UB;

    // device state: stack rows and depths, parents' survivor counts, incumbent
    int64_t cap_stack = std::max<int64_t>(1024, 2 * pool_cap);
    int32_t *srows = nullptr, *sdep = nullptr, *dinc = nullptr, *root_lb = nullptr;
    uint32_t *surv = nullptr;
    StepBuffers B;
    auto cleanup = [&]() {
        if (srows) hipFreeAsync(srows, s);
        if (sdep) hipFreeAsync(sdep, s);
        if (surv) hipFreeAsync(surv, s);
        if (dinc) hipFreeAsync(dinc, s);
        if (root_lb) hipFreeAsync(root_lb, s);
        B.release(s);
        hipStreamSynchronize(s);
    };
    hipError_t e = hipMallocAsync((void **)&srows, (size_t)cap_stack * n * 4, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&sdep, (size_t)cap_stack * 4, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&surv, (size_t)pool_cap * 4, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&dinc, (size_t)n * 4, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&root_lb, 4, s);
    if (e == hipSuccess) e = B.ensure(pool_cap, pool_cap, n, s);
    if (e != hipSuccess) { cleanup(); return fail(e); }

    // root: an all-zero row of depth 0
    std::vector<int32_t> zrow(n, 0);
    const int32_t zdepth = 0;
    e = hipMemcpyAsync(srows, zrow.data(), (size_t)n * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sdep, &zdepth, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = inst->packed16 ? launch_bound_packed(inst, srows, sdep, 1, root_lb, s)
                           : launch_bound_lane32(inst, srows, sdep, 1, root_lb, s);
    int32_t lb0 = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&lb0, root_lb, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { cleanup(); return fail(e); }

    int64_t nodes = 1, steps = 0, top = 0, max_stack = 0;
    int32_t improvements = 0;
    // run-length mirror of the stack depths, bottom to top
    std::vector<std::pair<int32_t, int64_t>> runs;
    if (lb0 < UB) {
        top = 1;
        runs.push_back({0, 1});
        max_stack = 1;
    }
    std::vector<uint32_t> hsurv;
    std::vector<std::pair<int32_t, int64_t>> taken;  // (depth, count) in pop order
    while (top > 0 && nodes < node_budget) {
        // selection
        taken.clear();
        int64_t K = 0, nch = 0;
        while (!runs.empty()) {
            auto &r = runs.back();
            const int64_t c = n - r.first;
            int64_t x = (pool_cap - nch) / c;
            if (K == 0) x = std::max<int64_t>(x, 1);
            x = std::min(x, r.second);
            if (x <= 0) break;
            taken.push_back({r.first, x});
            K += x;
            nch += x * c;
            r.second -= x;
            if (r.second > 0) break;
            runs.pop_back();
        }
        const int64_t base = top - K;
        // room for every child on the stack
        if (base + nch > cap_stack) {
            int64_t nc = cap_stack;
            while (base + nch > nc) nc *= 2;
            int32_t *r2 = nullptr, *d2 = nullptr;
            e = hipMallocAsync((void **)&r2, (size_t)nc * n * 4, s);
            if (e == hipSuccess) e = hipMallocAsync((void **)&d2, (size_t)nc * 4, s);
            if (e == hipSuccess) e = hipMemcpyAsync(r2, srows, (size_t)top * n * 4, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(d2, sdep, (size_t)top * 4, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) { cleanup(); return fail(e); }
            hipFreeAsync(srows, s);
            hipFreeAsync(sdep, s);
            srows = r2;
            sdep = d2;
            cap_stack = nc;
        }
        e = B.ensure(pool_cap, std::max(pool_cap, nch), n, s);  // one parent may exceed pool_cap
        if (e != hipSuccess) { cleanup(); return fail(e); }
        StepArgs a{};
        a.n = n;
        a.ub_in = UB;
        a.parents = srows;
        a.pdepth = sdep;
        a.K = K;
        a.parents_reversed = 1;
        a.parent_top = top;
        a.out_rows = srows;
        a.out_depth = sdep;
        a.out_lb = nullptr;
        a.out_base = base;
        a.out_cap = cap_stack;
        a.out_reversed = 1;
        a.surv_per_parent = surv;
        a.incumbent = dinc;
        e = step_phase1(a, B.w, s);
        if (e == hipSuccess) e = step_phase2(inst, a, B.w, nch, s);
        StepOut o{};
        if (e == hipSuccess) e = read_step_out(B.w, o, s);
        if (e != hipSuccess) { cleanup(); return fail(e); }
        if (o.bad || (int64_t)o.nchild != nch) { cleanup(); return FSP_E_BADNODE; }
        hsurv.resize(K);
        e = hipMemcpyAsync(hsurv.data(), surv, (size_t)K * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { cleanup(); return fail(e); }
        nodes += nch;
        const uint32_t idx = (uint32_t)(o.best & 0xffffffffu);
        if (idx != 0xffffffffu) {
            UB = (int32_t)(o.best >> 32);
            ++improvements;
            e = hipMemcpyAsync(inc.data(), dinc, (size_t)n * 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { cleanup(); return fail(e); }
        }
        // survivors sit bottom-to-top as: children of the last popped parent ... of the first
        int64_t p = K;
        for (auto it = taken.rbegin(); it != taken.rend(); ++it) {
            for (int64_t x = 0; x < it->second; ++x) {
                --p;
                const int64_t cnt = hsurv[p];
                if (!cnt) continue;
                const int32_t d = it->first + 1;
                if (!runs.empty() && runs.back().first == d) runs.back().second += cnt;
                else runs.push_back({d, cnt});
            }
        }
        top = base + o.nsurv;
        max_stack = std::max(max_stack, top);
        if (steplog && steps < steplog_cap) {
            int64_t *L = steplog + steps * 6;
            L[0] = K; L[1] = nch; L[2] = UB; L[3] = o.nsurv; L[4] = top; L[5] = (int64_t)o.fingerprint;
        }
        ++steps;
    }
    cleanup();
    res->opt = UB;
    res->proven = top == 0;
    res->nodes_bounded = nodes;
    res->steps = steps;
    res->improvements = improvements;
    res->max_stack = max_stack;
    if (perm_out) std::copy(inc.begin(), inc.end(), perm_out);
    return res->proven ? FSP_OK : FSP_BUDGET;
}

}  // extern "C"
