// Hybrid search: host threads explore the tree, the GPU bounds their pools
// (the host-driven scheme of Sec. III: the CPU selects and branches, the GPU
// evaluates the bounds of each pool; several host explorers share the device,
// the multi-threaded CPU exploration the paper leaves to future work).
//
// Each explorer runs its own depth-first search on a host stack: it pops
// parents while their children fit in pool_cap, writes the children's rows
// into a host pool, hands the pool to the bounding service and waits; then it
// updates the shared upper bound with complete children and pushes the others
// whose bound is below it (reverse child order).  When its stack is empty it
// takes the next subtree from a shared list: the first levels of the tree,
// expanded breadth first until there are four subtrees per explorer.
//
// The bounding service is one thread that owns every HIP call: it takes all
// pools waiting at that moment, packs them into one pinned buffer, copies it
// to the device, bounds it as one pool and copies the bounds back, so the
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
    const int32_t *rows;  // N x n, host
    const int32_t *depths;
    int64_t N;
    int32_t *lb;          // N, host (written by the service)
    bool done = false;
};

class BoundService {
public:
    BoundService(fsp_instance_s *I, hipStream_t s) : I_(I), s_(s) {}

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

    // Blocks until the pool's bounds are written; false if the device failed.
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
    int64_t launches() const { return launches_; }

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

    hipError_t reserve(int64_t N)
    {
        if (N <= cap_) return hipSuccess;
        release();
        cap_ = std::max<int64_t>(N, 4096);
        const size_t rb = (size_t)cap_ * I_->n * 4, db = (size_t)cap_ * 4;
        hipError_t e = hipHostMalloc((void **)&h_rows_, rb, 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h_dep_, db, 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h_lb_, db, 0);
        if (e == hipSuccess) e = hipMalloc((void **)&d_rows_, rb);
        if (e == hipSuccess) e = hipMalloc((void **)&d_dep_, db);
        if (e == hipSuccess) e = hipMalloc((void **)&d_lb_, db);
        if (e != hipSuccess) cap_ = 0;
        return e;
    }

    void release()
    {
        if (h_rows_) hipHostFree(h_rows_);
        if (h_dep_) hipHostFree(h_dep_);
        if (h_lb_) hipHostFree(h_lb_);
        if (d_rows_) hipFree(d_rows_);
        if (d_dep_) hipFree(d_dep_);
        if (d_lb_) hipFree(d_lb_);
        h_rows_ = h_dep_ = h_lb_ = d_rows_ = d_dep_ = d_lb_ = nullptr;
        cap_ = 0;
    }

    hipError_t run(const std::vector<PoolReq *> &batch)
    {
        const int n = I_->n;
        int64_t N = 0;
        for (PoolReq *r : batch) N += r->N;
        hipError_t e = reserve(N);
        if (e != hipSuccess) return e;
        int64_t off = 0;
        for (PoolReq *r : batch) {
            std::memcpy(h_rows_ + off * n, r->rows, (size_t)r->N * n * 4);
            std::memcpy(h_dep_ + off, r->depths, (size_t)r->N * 4);
            off += r->N;
        }
        e = hipMemcpyAsync(d_rows_, h_rows_, (size_t)N * n * 4, hipMemcpyHostToDevice, s_);
        if (e == hipSuccess) e = hipMemcpyAsync(d_dep_, h_dep_, (size_t)N * 4, hipMemcpyHostToDevice, s_);
        if (e == hipSuccess)
            e = I_->packed16 ? launch_bound_packed(I_, d_rows_, d_dep_, N, d_lb_, s_)
                             : launch_bound_lane32(I_, d_rows_, d_dep_, N, d_lb_, s_);
        if (e == hipSuccess) e = hipMemcpyAsync(h_lb_, d_lb_, (size_t)N * 4, hipMemcpyDeviceToHost, s_);
        if (e == hipSuccess) e = hipStreamSynchronize(s_);
        if (e != hipSuccess) return e;
        off = 0;
        for (PoolReq *r : batch) {
            std::memcpy(r->lb, h_lb_ + off, (size_t)r->N * 4);
            off += r->N;
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
    int64_t cap_ = 0, launches_ = 0;
    int32_t *h_rows_ = nullptr, *h_dep_ = nullptr, *h_lb_ = nullptr;
    int32_t *d_rows_ = nullptr, *d_dep_ = nullptr, *d_lb_ = nullptr;
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
    std::deque<std::vector<int32_t>> work;  // subtree roots: [depth, job_0 .. job_{n-1}]

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

void explorer(int n, int64_t pool_cap, Shared &sh, BoundService &svc)
{
    std::vector<int32_t> stack;  // nodes of n + 1 ints: depth, jobs
    std::vector<int32_t> rows, depths, lbs, parents;
    std::vector<unsigned char> sched(n);
    const int W = n + 1;
    for (;;) {
        if (stack.empty()) {
            std::lock_guard<std::mutex> lk(sh.work_mu);
            if (sh.work.empty()) return;
            stack = std::move(sh.work.front());
            sh.work.pop_front();
        }
        if (sh.failed.load() || sh.out_of_budget.load()) return;
        // pop parents while their children fit (the first always)
        int64_t nch = 0;
        parents.clear();
        while (!stack.empty()) {
            const int32_t *top = stack.data() + stack.size() - W;
            const int64_t c = n - top[0];
            if (!parents.empty() && nch + c > pool_cap) break;
            parents.insert(parents.end(), top, top + W);
            stack.resize(stack.size() - W);
            nch += c;
        }
        const int64_t K = (int64_t)parents.size() / W;
        rows.assign((size_t)nch * n, 0);
        depths.resize(nch);
        lbs.resize(nch);
        int64_t c = 0;
        for (int64_t k = 0; k < K; ++k) {
            const int32_t *par = parents.data() + k * W;
            const int d = par[0];
            std::fill(sched.begin(), sched.end(), 0);
            for (int t = 0; t < d; ++t) sched[par[1 + t]] = 1;
            for (int j = 0; j < n; ++j) {
                if (sched[j]) continue;
                int32_t *row = rows.data() + c * n;
                std::memcpy(row, par + 1, (size_t)d * 4);
                row[d] = j;
                depths[c] = d + 1;
                ++c;
            }
        }
        PoolReq r{rows.data(), depths.data(), nch, lbs.data()};
        if (!svc.bound(r)) {
            sh.failed = true;
            return;
        }
        if (sh.nodes.fetch_add(nch) + nch >= sh.budget) sh.out_of_budget = true;
        for (int64_t i = 0; i < nch; ++i)
            if (depths[i] == n && lbs[i] < sh.ub.load()) sh.offer(lbs[i], rows.data() + i * n, n);
        const int32_t ub = sh.ub.load();
        for (int64_t i = nch - 1; i >= 0; --i) {
            if (depths[i] == n || lbs[i] >= ub) continue;
            const size_t at = stack.size();
            stack.resize(at + W);
            stack[at] = depths[i];
            std::memcpy(stack.data() + at + 1, rows.data() + i * n, (size_t)n * 4);
        }
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
    svc.start();

    // root, then the first levels breadth first until there is work for every explorer
    std::vector<std::vector<int32_t>> level(1, std::vector<int32_t>(n + 1, 0));
    int64_t nodes = 0;
    bool ok = true;
    {
        std::vector<int32_t> lb(1);
        std::vector<int32_t> row(n, 0), dep(1, 0);
        PoolReq r{row.data(), dep.data(), 1, lb.data()};
        ok = svc.bound(r);
        nodes = 1;
        if (ok && lb[0] >= sh.ub.load()) level.clear();
    }
    for (int depth = 0; ok && !level.empty() && depth < n - 1 && (int64_t)level.size() < 4 * threads; ++depth) {
        std::vector<int32_t> rows, deps, lbs;
        std::vector<unsigned char> sched(n);
        for (const auto &par : level) {
            std::fill(sched.begin(), sched.end(), 0);
            for (int t = 0; t < par[0]; ++t) sched[par[1 + t]] = 1;
            for (int j = 0; j < n; ++j) {
                if (sched[j]) continue;
                const size_t at = rows.size();
                rows.resize(at + n, 0);
                std::memcpy(rows.data() + at, par.data() + 1, (size_t)par[0] * 4);
                rows[at + par[0]] = j;
                deps.push_back(par[0] + 1);
            }
        }
        lbs.resize(deps.size());
        PoolReq r{rows.data(), deps.data(), (int64_t)deps.size(), lbs.data()};
        ok = svc.bound(r);
        nodes += (int64_t)deps.size();
        std::vector<std::vector<int32_t>> next;
        for (size_t i = 0; ok && i < deps.size(); ++i) {
            if (deps[i] == n) {
                if (lbs[i] < sh.ub.load()) sh.offer(lbs[i], rows.data() + i * n, n);
                continue;
            }
            if (lbs[i] >= sh.ub.load()) continue;
            std::vector<int32_t> node(n + 1);
            node[0] = deps[i];
            std::memcpy(node.data() + 1, rows.data() + i * n, (size_t)n * 4);
            next.push_back(std::move(node));
        }
        level.swap(next);
    }
    sh.nodes = nodes;
    for (auto &nd : level) sh.work.push_back(std::move(nd));
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
