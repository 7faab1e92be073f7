// Hybrid search: host threads explore the tree, the GPU bounds their pools
// (the host-driven scheme of Sec. III: the CPU selects and branches, the GPU
// evaluates the bounds of each pool; several host explorers share the device,
// the multi-threaded CPU exploration the paper leaves to future work).
//
// Each explorer runs its own depth-first search on a host stack: it pops
// parents while their children fit in pool_cap and hands the parents to the
// bounding service, which returns the bounds of all their children (in
// parent order, then by increasing appended job).  The explorer then updates
// the shared upper bound with complete children and pushes the others whose
// bound is below it (reverse child order), building only those rows.  When
// its stack is empty it takes the next subtree from a shared list: the first
// levels of the tree, expanded breadth first until there are four subtrees
// per explorer.
//
// The bounding service is one thread that owns every HIP call: it takes all
// requests waiting at that moment, copies their parents (not their children:
// n - d times fewer rows cross PCIe) to the device in one pinned transfer,
// lists and bounds the children of all of them as one step (children bounded
// from their parents on the 16-bit path) and copies the bounds back, so the
// explorers' pools are merged into large launches.  Node counts depend on
// thread timing; the optimum and the proof do not.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "search.h"

using namespace fspbb;

namespace {

struct PoolReq {
    const int32_t *parents;  // K x n, host: the first depth entries of each row
    const int32_t *depths;   // K, each < n
    int64_t K, nch;          // nch = sum over parents of (n - depth)
    int32_t *lb;             // nch, host (written by the service), child order
    bool done = false;
};

class BoundService {
public:
    BoundService(fsp_instance_s *I, hipStream_t s) : I_(I), s_(s) { ctx_.s = s; }

    // Sizes every buffer for K parents and C children before the thread
    // starts (the buffers only grow; growing pinned memory mid-search costs
    // milliseconds per step early on).
    hipError_t presize(int64_t K, int64_t C)
    {
        hipError_t e = reserve(K, C);
        B_.rows = !kids16_eligible(I_);
        if (e == hipSuccess) e = B_.ensure_k(K, s_);
        if (e == hipSuccess) e = B_.ensure_c(C, I_->n, s_);
        if (e == hipSuccess && !B_.rows) e = kids16_ensure(kids_, I_, K, C, s_);
        if (e == hipSuccess) e = ctx_.reserve((size_t)K * 4 + (64 << 10));
        if (e == hipSuccess) e = hipStreamSynchronize(s_);
        return e;
    }

    hipError_t start()
    {
        th_ = std::thread([this] { loop(); });
        return hipSuccess;
    }

    void stop()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        if (th_.joinable()) th_.join();
        release();
    }

    // Blocks until the children's bounds are written; false if the device failed.
    bool bound(PoolReq &r)
    {
        std::unique_lock<std::mutex> lk(mu_);
        if (err_ != hipSuccess) return false;
        q_.push_back(&r);
        cv_work_.notify_one();
        cv_done_.wait(lk, [&] { return r.done || err_ != hipSuccess; });
        return r.done;
    }

    hipError_t error() const { return err_; }
    int64_t launches() const { return launches_.load(); }

private:
    void loop()
    {
        hipSetDevice(I_->device);
        for (;;) {
            std::vector<PoolReq *> batch;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_work_.wait(lk, [&] { return stop_ || !q_.empty(); });
                if (stop_ && q_.empty()) return;
                batch.assign(q_.begin(), q_.end());
                q_.clear();
            }
            hipError_t e = run(batch);
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (e != hipSuccess) err_ = e;
                else
                    for (PoolReq *r : batch) r->done = true;
            }
            cv_done_.notify_all();
            if (e != hipSuccess) return;
        }
    }

    hipError_t reserve(int64_t K, int64_t C)
    {
        if (K > capK_) {
            // the previous batch ended with a stream synchronization
            pinned_put(h_par_, hb_par_);
            pinned_put(h_dep_, hb_dep_);
            if (d_par_) stream_free(d_par_, s_);
            if (d_dep_) stream_free(d_dep_, s_);
            h_par_ = h_dep_ = d_par_ = d_dep_ = nullptr;
            hb_par_ = hb_dep_ = 0;
            capK_ = 0;
            const int64_t c = std::max<int64_t>(K, 1024);
            const size_t rb = (size_t)c * I_->n * 4, db = (size_t)c * 4;
            hipError_t e = pinned_get((void **)&h_par_, &hb_par_, rb);
            if (e == hipSuccess) e = pinned_get((void **)&h_dep_, &hb_dep_, db);
            if (e == hipSuccess) e = stream_alloc((void **)&d_par_, rb, s_);
            if (e == hipSuccess) e = stream_alloc((void **)&d_dep_, db, s_);
            if (e != hipSuccess) return e;
            capK_ = c;
        }
        if (C > capC_) {
            pinned_put(h_lb_, hb_lb_);
            h_lb_ = nullptr;
            hb_lb_ = 0;
            capC_ = 0;
            const int64_t c = std::max<int64_t>(C, 4096);
            hipError_t e = pinned_get((void **)&h_lb_, &hb_lb_, (size_t)c * 4);
            if (e != hipSuccess) return e;
            capC_ = c;
        }
        return hipSuccess;
    }

    void release()
    {
        hipStreamSynchronize(s_);
        pinned_put(h_par_, hb_par_);
        pinned_put(h_dep_, hb_dep_);
        pinned_put(h_lb_, hb_lb_);
        if (d_par_) stream_free(d_par_, s_);
        if (d_dep_) stream_free(d_dep_, s_);
        h_par_ = h_dep_ = h_lb_ = d_par_ = d_dep_ = nullptr;
        hb_par_ = hb_dep_ = hb_lb_ = 0;
        capK_ = capC_ = 0;
        B_.release(s_);
        kids16_release(kids_, s_);
        ctx_.release();
    }

    hipError_t run(const std::vector<PoolReq *> &batch)
    {
        const int n = I_->n;
        int64_t K = 0, C = 0;
        for (PoolReq *r : batch) {
            K += r->K;
            C += r->nch;
        }
        if (C == 0) return hipSuccess;
        hipError_t e = reserve(K, C);
        if (e != hipSuccess) return e;
        int64_t off = 0;
        for (PoolReq *r : batch) {
            for (int64_t k = 0; k < r->K; ++k)
                std::memcpy(h_par_ + (off + k) * n, r->parents + k * n, (size_t)r->depths[k] * 4);
            std::memcpy(h_dep_ + off, r->depths, (size_t)r->K * 4);
            off += r->K;
        }
        e = hipMemcpyAsync(d_par_, h_par_, (size_t)K * n * 4, hipMemcpyHostToDevice, s_);
        if (e == hipSuccess) e = hipMemcpyAsync(d_dep_, h_dep_, (size_t)K * 4, hipMemcpyHostToDevice, s_);
        if (e == hipSuccess) e = bound_children_of(I_, d_par_, d_dep_, K, C, B_, kids_, ctx_, s_);
        if (e == hipSuccess) e = hipMemcpyAsync(h_lb_, B_.w.clb, (size_t)C * 4, hipMemcpyDeviceToHost, s_);
        if (e == hipSuccess) e = hipStreamSynchronize(s_);
        if (e != hipSuccess) return e;
        off = 0;
        for (PoolReq *r : batch) {
            std::memcpy(r->lb, h_lb_ + off, (size_t)r->nch * 4);
            off += r->nch;
        }
        ++launches_;
        return hipSuccess;
    }

    fsp_instance_s *I_;
    hipStream_t s_;
    std::thread th_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<PoolReq *> q_;
    bool stop_ = false;
    hipError_t err_ = hipSuccess;
    int64_t capK_ = 0, capC_ = 0;
    std::atomic<int64_t> launches_{0};  // read by the caller while the thread may run
    int32_t *h_par_ = nullptr, *h_dep_ = nullptr, *h_lb_ = nullptr;
    size_t hb_par_ = 0, hb_dep_ = 0, hb_lb_ = 0;  // their capacities in bytes
    int32_t *d_par_ = nullptr, *d_dep_ = nullptr;
    StepBuffers B_;
    Kids16 kids_;
    TickContext ctx_;
};

// Upper bound and incumbent shared by the explorers.
struct Shared {
    std::atomic<int32_t> ub;
    std::mutex inc_mu;
    std::vector<int32_t> inc;
    std::atomic<int64_t> nodes{0};
    std::atomic<bool> out_of_budget{false};
    std::atomic<bool> failed{false};
    int64_t budget = 0;
    std::mutex work_mu;
    std::deque<std::vector<int32_t>> work;  // subtree roots: depth, then its prefix

    // A complete schedule of makespan lb: the new upper bound and incumbent
    // when it is below the current one (ub is also read without the lock).
    void offer(int32_t lb, const int32_t *row, int n)
    {
        std::lock_guard<std::mutex> lk(inc_mu);
        if (lb < ub.load()) {
            ub.store(lb);
            inc.assign(row, row + n);
        }
    }
};

// Bounds the children of the K parents in prow (K x n, the first pdep[k]
// entries of row k) through the service: lb receives them in child order.
bool bound_children(int n, int64_t K, const std::vector<int32_t> &prow, const std::vector<int32_t> &pdep,
                    BoundService &svc, std::vector<int32_t> &lb, int64_t &nch)
{
    nch = 0;
    for (int64_t k = 0; k < K; ++k) nch += n - pdep[k];
    lb.resize((size_t)std::max<int64_t>(nch, 1));
    PoolReq r{prow.data(), pdep.data(), K, nch, lb.data()};
    return svc.bound(r);
}

// Calls f(child index, parent k, appended job) over the children of the K
// parents in child order (reverse: from the last child back).
template <class F>
void for_children(int n, int64_t K, const std::vector<int32_t> &prow, const std::vector<int32_t> &pdep, int64_t nch,
                  bool reverse, std::vector<unsigned char> &sched, F f)
{
    int64_t c = reverse ? nch - 1 : 0;
    for (int64_t kk = 0; kk < K; ++kk) {
        const int64_t k = reverse ? K - 1 - kk : kk;
        const int32_t *row = prow.data() + k * n;
        std::fill(sched.begin(), sched.end(), 0);
        for (int t = 0; t < pdep[k]; ++t) sched[row[t]] = 1;
        for (int jj = 0; jj < n; ++jj) {
            const int j = reverse ? n - 1 - jj : jj;
            if (sched[j]) continue;
            f(c, k, j);
            c += reverse ? -1 : 1;
        }
    }
}

// An explorer's stack holds compact entries: a child is its parent (an
// expanded node of the explorer's arena), its appended job and its depth.
// A prefix is rebuilt only when its node is popped as a parent, by walking
// the arena up to the subtree root, so a pushed child costs 12 bytes instead
// of a row of n + 1 ints.
struct Entry {
    int32_t parent;  // arena index; kRootEntry: the subtree root itself
    int32_t job;
    int32_t depth;
};
constexpr int32_t kRootEntry = -2;

struct Arena {
    std::vector<int32_t> root;                     // the subtree root: depth, then its prefix
    std::vector<std::pair<int32_t, int32_t>> rec;  // expanded nodes: (parent index, job); -1 = the root

    // Appends the expanded node of stack entry e; returns its index.
    int32_t expand(const Entry &e)
    {
        rec.push_back(e.parent == kRootEntry ? std::make_pair(-1, -1) : std::make_pair(e.parent, e.job));
        return (int32_t)rec.size() - 1;
    }
    // Writes the prefix (depth d) of expanded node a into out.
    void prefix(int32_t a, int d, int32_t *out) const
    {
        int t = d;
        while (rec[a].first >= 0) {
            out[--t] = rec[a].second;
            a = rec[a].first;
        }
        std::memcpy(out, root.data() + 1, (size_t)t * 4);  // t is the root's depth
    }
};

void explorer(int n, int64_t pool_cap, Shared &sh, BoundService &svc)
{
    std::vector<Entry> stack;
    Arena ar;
    std::vector<int32_t> prow, pdep, pidx, lbs, row(n);
    std::vector<unsigned char> sched(n);
    for (;;) {
        if (stack.empty()) {
            std::lock_guard<std::mutex> lk(sh.work_mu);
            if (sh.work.empty()) return;
            ar.root = std::move(sh.work.front());
            sh.work.pop_front();
            ar.rec.clear();
            stack.push_back(Entry{kRootEntry, -1, ar.root[0]});
        }
        if (sh.failed.load() || sh.out_of_budget.load()) return;
        // pop parents while their children fit (the first always)
        int64_t K = 0, nch = 0;
        pdep.clear();
        pidx.clear();
        while (!stack.empty()) {
            const Entry e = stack.back();
            const int64_t c = n - e.depth;
            if (K > 0 && nch + c > pool_cap) break;
            stack.pop_back();
            const int32_t a = ar.expand(e);
            prow.resize((size_t)(K + 1) * n);
            ar.prefix(a, e.depth, prow.data() + K * n);
            pdep.push_back(e.depth);
            pidx.push_back(a);
            ++K;
            nch += c;
        }
        if (!bound_children(n, K, prow, pdep, svc, lbs, nch)) {
            sh.failed = true;
            return;
        }
        if (sh.nodes.fetch_add(nch) + nch >= sh.budget) sh.out_of_budget = true;
        // complete children first (they may lower the bound), then the pushes
        for_children(n, K, prow, pdep, nch, false, sched, [&](int64_t c, int64_t k, int j) {
            const int d = pdep[k];
            if (d + 1 == n && lbs[c] < sh.ub.load()) {
                std::memcpy(row.data(), prow.data() + k * n, (size_t)d * 4);
                row[d] = j;
                sh.offer(lbs[c], row.data(), n);
            }
        });
        const int32_t ub = sh.ub.load();
        for_children(n, K, prow, pdep, nch, true, sched, [&](int64_t c, int64_t k, int j) {
            if (pdep[k] + 1 == n || lbs[c] >= ub) return;
            stack.push_back(Entry{pidx[k], j, pdep[k] + 1});
        });
    }
}

}  // namespace

extern "C" {

fsp_status fsp_explore(fsp_instance inst, int32_t ub0, int32_t threads, int64_t pool_cap, int64_t node_budget,
                       fsp_explore_result *res, int32_t *perm_out, void *stream)
{
    if (!inst || !res || threads < 1 || threads > 256 || pool_cap < 1 || node_budget < 1 ||
        (ub0 < 0 && ub0 != FSP_UB_NEH))
        return FSP_E_INVAL;
    std::memset(res, 0, sizeof(*res));
    DeviceGuard g(inst->device);
    if (!g.ok) return FSP_E_DEVICE;
    const int n = inst->n;
    const auto t0 = std::chrono::steady_clock::now();
    Shared sh;
    sh.inc.assign(n, -1);
    int32_t UB = ub0 == FSP_UB_NEH ? neh(inst->p_host, n, inst->m, sh.inc.data()) : ub0;
    sh.ub = UB;
    sh.budget = node_budget;
    res->ub0 = UB;
    BoundService svc(inst, (hipStream_t)stream);
    // every explorer's pool at once, with about 64 parents each (up to half a
    // million children; beyond, the buffers grow when needed)
    const hipError_t pe = svc.presize((int64_t)threads * 64,
                                      std::min<int64_t>((int64_t)threads * std::max<int64_t>(pool_cap, n), 1 << 19));
    if (pe != hipSuccess) {
        svc.stop();
        return fail_status(pe);
    }
    svc.start();

    // the first levels, breadth first from the root, until there is work for
    // every explorer (the root itself is not bounded: its children are)
    std::vector<int32_t> prow(n), pdep(1, 0);  // the level's nodes: rows and depths
    int64_t nodes = 0, K = 1;
    bool ok = true;
    {
        std::vector<int32_t> lbs, nrow, ndep, row(n);
        std::vector<unsigned char> sched(n);
        for (int depth = 0; ok && K > 0 && depth < n - 1 && K < 4 * threads; ++depth) {
            int64_t nch = 0;
            ok = bound_children(n, K, prow, pdep, svc, lbs, nch);
            if (!ok) break;
            nodes += nch;
            nrow.clear();
            ndep.clear();
            for_children(n, K, prow, pdep, nch, false, sched, [&](int64_t c, int64_t k, int j) {
                const int d = pdep[k];
                if (lbs[c] >= sh.ub.load()) return;
                std::memcpy(row.data(), prow.data() + k * n, (size_t)d * 4);
                row[d] = j;
                if (d + 1 == n) {
                    sh.offer(lbs[c], row.data(), n);
                    return;
                }
                nrow.insert(nrow.end(), row.begin(), row.end());
                ndep.push_back(d + 1);
            });
            prow.swap(nrow);
            pdep.swap(ndep);
            K = (int64_t)pdep.size();
        }
    }
    sh.nodes = nodes;
    for (int64_t k = 0; k < K; ++k) {  // subtree roots: depth, then the prefix
        std::vector<int32_t> r(1 + pdep[k]);
        r[0] = pdep[k];
        std::memcpy(r.data() + 1, prow.data() + k * n, (size_t)pdep[k] * 4);
        sh.work.push_back(std::move(r));
    }
    if (ok && nodes >= node_budget && !sh.work.empty()) sh.out_of_budget = true;

    std::vector<std::thread> ts;
    for (int t = 0; ok && t < threads; ++t) ts.emplace_back(explorer, n, pool_cap, std::ref(sh), std::ref(svc));
    for (auto &t : ts) t.join();
    const hipError_t e = svc.error();
    const int64_t launches = svc.launches();
    svc.stop();
    if (!ok || sh.failed.load() || e != hipSuccess) return fail_status(e != hipSuccess ? e : hipErrorUnknown);
    res->opt = sh.ub.load();
    res->proven = sh.out_of_budget.load() ? 0 : 1;
    res->nodes_bounded = sh.nodes.load();
    res->pools = launches;
    res->threads = threads;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (perm_out) std::copy(sh.inc.begin(), sh.inc.end(), perm_out);
    return res->proven ? FSP_OK : FSP_BUDGET;
}

}  // extern "C"
