// Batched bounding of many pools (possibly of different instances and
// shapes) in one decode launch per machine-count class and one persistent
// scan launch, either captured once in a HIP graph and replayed
// (fsp_batch_*), or re-planned per call into a reusable device region (the
// merged bounding step of concurrent searches).
//
// Plan: every pool is cut into 128-node groups; a work item holds as many
// groups of one pool as its tile schedule stages in LDS at once (16 / wpg,
// wpg = waves per group, tuned per instance shape).  Items are queued longest
// first so that the persistent workgroups finish together.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "batch.h"

using namespace fspbb;

namespace fspbb {

namespace {
std::mutex g_tune_mu;
std::map<std::pair<int, int>, ScanTuning> g_tune;

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

namespace {
// Rule of thumb: about four machine pairs per wave and chain.
ScanTuning rule_tuning(int P)
{
    int w = 1;
    while (w < kBatchWaves && 4 * 2 * w <= P) w *= 2;
    return ScanTuning{w, 8, kBatchGrid};
}
}  // namespace

ScanTuning scan_tuning(int n, int m)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find({n, m});
        if (it != g_tune.end()) return it->second;
    }
    ScanTuning t = rule_tuning(m * (m - 1) / 2);
    t.waves_per_group = fit_waves_per_group(t.waves_per_group, n);
    return t;
}

ScanTuning scan_tuning_for(const fsp_instance_s *I)
{
    // the table is keyed by shape with every pair; a pair subset scans fewer pairs
    if (I->P != I->m * (I->m - 1) / 2) {
        ScanTuning t = rule_tuning(I->P);
        t.waves_per_group = fit_waves_per_group(t.waves_per_group, I->n);
        return t;
    }
    return scan_tuning(I->n, I->m);
}

void set_scan_tuning(int n, int m, ScanTuning t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{n, m}] = t;
}

bool has_scan_tuning(int n, int m)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune.count({n, m}) != 0;
}

void scan_tuning_entries(std::vector<std::pair<std::pair<int, int>, ScanTuning>> &out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    out.assign(g_tune.begin(), g_tune.end());
}

fsp_status check_pools(const fsp_pool_desc *pools, int32_t n_pools, int *dev_out)
{
    if (!pools || n_pools < 1) return FSP_E_INVAL;
    const int dev = pools[0].inst ? pools[0].inst->device : -1;
    for (int i = 0; i < n_pools; ++i) {
        const fsp_pool_desc &d = pools[i];
        if (!d.inst || d.N < 0 || d.inst->device != dev) return FSP_E_INVAL;
        if (!d.inst->packed16) return FSP_E_INVAL;
        if (d.N > 0 && (!d.prefixes || !d.depths || !d.out_lb)) return FSP_E_INVAL;
    }
    *dev_out = dev;
    return FSP_OK;
}

void plan_batch(const fsp_pool_desc *pools, int32_t n_pools, int32_t wpg_force, bool sort_depths, BatchPlan &pl,
                int32_t form_force, const Workspace16 *ready)
{
    pl = BatchPlan{};
    pl.pools.resize(n_pools);
    pl.ws_off.resize(n_pools);
    pl.decoded.assign(n_pools, 0);
    struct Cost { int64_t cost; WorkItem w; };
    std::vector<Cost> items;
    size_t ws = 0;
    pl.scan_lds = 64 * kBatchWaves * 4;  // the cross-wave reduction reuses the mask area
    for (int i = 0; i < n_pools; ++i) {
        const fsp_pool_desc &d = pools[i];
        const fsp_instance_s *I = d.inst;
        const int n = I->n, m = I->m, NW = (n + 31) >> 5;
        const int64_t G = (d.N + kGroup - 1) / kGroup, Npad = G * kGroup;
        const bool given = ready && ready[i].dec;
        pl.decoded[i] = given ? 1 : 0;
        pl.ws_off[i] = ws;
        if (!given)
            ws += al256((size_t)G * 3 * m * 64 * 4) + al256((size_t)G * NW * 128 * 4) + al256((size_t)Npad * 4);
        BatchPool &P = pl.pools[i];
        std::memset(&P, 0, sizeof(P));
        if (given) P.W = ready[i];
        if (!given && sort_depths && d.N >= kSortMinNodes) {
            P.sortB = (int32_t)std::min<int64_t>(kSortMaxBlocks, (d.N + 4095) / 4096);
            P.sort_chunk = (d.N + P.sortB - 1) / P.sortB;
            ws += al256((size_t)d.N * 4) + al256((size_t)(n + 2) * P.sortB * 4);
        }
        P.T = I->dt;
        P.prefixes = d.prefixes;
        P.depths = d.depths;
        P.out_lb = d.out_lb;
        P.N = d.N;
        P.Npad = Npad;
        P.wpg = fit_waves_per_group(wpg_force ? wpg_force : scan_tuning_for(I).waves_per_group, n);
        const int gpp = kBatchWaves / P.wpg;
        const int64_t per_wave = (I->P + P.wpg - 1) / P.wpg;
        for (int64_t g0 = 0; g0 < G; g0 += gpp) {
            const int ng = (int)std::min<int64_t>(gpp, G - g0);
            items.push_back({per_wave * I->dt.npad, WorkItem{i, (int32_t)g0, ng, 0}});
        }
        if (G > 0) pl.scan_lds = std::max(pl.scan_lds, (size_t)std::min<int64_t>(gpp, G) * (n + 1) * 256);
        pl.total_nodes += d.N;
    }
    bool all_persistent = true;
    for (int i = 0; i < n_pools; ++i)
        if (pools[i].N > 0 && scan_tuning_for(pools[i].inst).form != kBatchPersistent)
            all_persistent = false;
    pl.form = form_force >= 0 ? form_force : (all_persistent ? kBatchPersistent : kBatchGrid);
    std::stable_sort(items.begin(), items.end(), [](const Cost &x, const Cost &y) { return x.cost > y.cost; });
    for (auto &c : items) pl.items.push_back(c.w);
    pl.ws_bytes = al256(ws);

    std::map<int, std::vector<int32_t>> cls;
    for (int i = 0; i < n_pools; ++i)
        if (pools[i].N > 0 && !pl.decoded[i]) cls[(pools[i].inst->m + 3) & ~3].push_back(i);
    for (auto &kv : cls) {
        BatchPlan::Cls c;
        c.MV = kv.first;
        c.idx = kv.second;
        c.off.assign(kv.second.size() + 1, 0);
        int nmax = 0;
        for (size_t q = 0; q < kv.second.size(); ++q) {
            const BatchPool &P = pl.pools[kv.second[q]];
            c.off[q + 1] = c.off[q] + (P.Npad + 255) / 256;
            nmax = std::max(nmax, (int)P.T.n);
        }
        c.nblocks = c.off.back();
        c.lds = decode16_lds_words(nmax, c.MV) * 4;
        pl.classes.push_back(std::move(c));
    }
    pl.sort.off.assign(1, 0);
    for (int i = 0; i < n_pools; ++i) {
        const BatchPool &P = pl.pools[i];
        if (P.sortB == 0) continue;
        pl.sort.idx.push_back(i);
        pl.sort.off.push_back(pl.sort.off.back() + P.sortB);
        pl.sort.nmax = std::max(pl.sort.nmax, (int)P.T.n);
    }
    pl.sort.nblocks = pl.sort.off.back();
    size_t meta = 0;
    pl.meta_pools = meta;
    meta += al256(sizeof(BatchPool) * n_pools);
    pl.meta_items = meta;
    meta += al256(sizeof(WorkItem) * std::max<size_t>(1, pl.items.size()));
    pl.meta_counter = meta;
    meta += 256;
    for (auto &c : pl.classes) {
        c.meta_off = meta;
        meta += al256(sizeof(int64_t) * c.off.size());
        c.meta_idx = meta;
        meta += al256(sizeof(int32_t) * c.idx.size());
    }
    pl.sort.meta_off = meta;
    meta += al256(sizeof(int64_t) * pl.sort.off.size());
    pl.sort.meta_idx = meta;
    meta += al256(sizeof(int32_t) * std::max<size_t>(1, pl.sort.idx.size()));
    pl.meta_bytes = meta;
}

void layout_batch(BatchPlan &pl, char *base, std::vector<char> &host, char *dmeta)
{
    for (size_t i = 0; i < pl.pools.size(); ++i) {
        BatchPool &P = pl.pools[i];
        if (pl.decoded[i]) continue;  // the caller's workspace
        const int n = P.T.n, m = P.T.m, NW = (n + 31) >> 5;
        const int64_t G = P.Npad / kGroup;
        char *w = base + pl.ws_off[i];
        const size_t a = al256((size_t)G * 3 * m * 64 * 4), b = al256((size_t)G * NW * 128 * 4);
        P.W.dec = (uint32_t *)w;
        P.W.flg = (uint32_t *)(w + a);
        P.W.st = (uint32_t *)(w + a + b);
        P.W.order = nullptr;
        P.W.cnt = nullptr;
        if (P.sortB > 0) {
            const size_t c = al256((size_t)P.Npad * 4);
            P.W.order = (int32_t *)(w + a + b + c);
            P.W.cnt = (uint32_t *)(w + a + b + c + al256((size_t)P.N * 4));
        }
    }
    pl.dmeta = dmeta ? dmeta : base + pl.ws_bytes;
    host.assign(pl.meta_bytes, 0);
    std::memcpy(host.data() + pl.meta_pools, pl.pools.data(), sizeof(BatchPool) * pl.pools.size());
    if (!pl.items.empty())
        std::memcpy(host.data() + pl.meta_items, pl.items.data(), sizeof(WorkItem) * pl.items.size());
    for (auto &c : pl.classes) {
        std::memcpy(host.data() + c.meta_off, c.off.data(), sizeof(int64_t) * c.off.size());
        std::memcpy(host.data() + c.meta_idx, c.idx.data(), sizeof(int32_t) * c.idx.size());
    }
    std::memcpy(host.data() + pl.sort.meta_off, pl.sort.off.data(), sizeof(int64_t) * pl.sort.off.size());
    if (!pl.sort.idx.empty())
        std::memcpy(host.data() + pl.sort.meta_idx, pl.sort.idx.data(), sizeof(int32_t) * pl.sort.idx.size());
}

hipError_t enqueue_batch(const BatchPlan &pl, int grid, hipStream_t s)
{
    const BatchPool *dpools = (const BatchPool *)(pl.dmeta + pl.meta_pools);
    if (!pl.sort.idx.empty()) {
        hipError_t e = launch_batch_depth_sort(dpools, (const int64_t *)(pl.dmeta + pl.sort.meta_off),
                                               (const int32_t *)(pl.dmeta + pl.sort.meta_idx),
                                               (int)pl.sort.idx.size(), pl.sort.nblocks, pl.sort.nmax, s);
        if (e != hipSuccess) return e;
    }
    for (const auto &c : pl.classes) {
        hipError_t e = launch_batch_decode(c.MV, dpools, (const int64_t *)(pl.dmeta + c.meta_off),
                                           (const int32_t *)(pl.dmeta + c.meta_idx), (int)c.idx.size(), c.nblocks,
                                           c.lds, s);
        if (e != hipSuccess) return e;
    }
    if (pl.items.empty()) return hipSuccess;
    return launch_batch_scan(dpools, (const WorkItem *)(pl.dmeta + pl.meta_items), (int)pl.items.size(),
                             (uint32_t *)(pl.dmeta + pl.meta_counter), grid, pl.scan_lds, pl.form, s);
}

int batch_grid(int dev, size_t scan_lds)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    return prop.multiProcessorCount * batch_scan_blocks_per_cu(scan_lds);
}

hipError_t BatchArena::run(const fsp_pool_desc *pools, int32_t n_pools, hipStream_t s, const Workspace16 *ready)
{
    plan_batch(pools, n_pools, 0, false, plan, -1, ready);  // child pools of a step have few distinct depths
    const size_t need = plan.ws_bytes + plan.meta_bytes;
    if (need > dev_bytes) {
        const size_t cap = std::max(need, dev_bytes * 2);
        if (dev) stream_free(dev, s);
        dev = nullptr;
        dev_bytes = 0;
        hipError_t e = stream_alloc((void **)&dev, cap, s);
        if (e != hipSuccess) return e;
        dev_bytes = cap;
    }
    layout_batch(plan, (char *)dev, meta);
    if (meta.size() > pinned_bytes) {
        pinned_put(pinned, pinned_bytes);
        pinned = nullptr;
        pinned_bytes = 0;
        hipError_t e = pinned_get(&pinned, &pinned_bytes, meta.size() * 2);
        if (e != hipSuccess) return e;
    }
    std::memcpy(pinned, meta.data(), meta.size());
    hipError_t e = hipMemcpyAsync(plan.dmeta, pinned, meta.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    int d = 0;
    e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    return enqueue_batch(plan, plan.form == kBatchPersistent ? batch_grid(d, plan.scan_lds) : 0, s);
}

hipError_t BatchArena::plan_only(const fsp_pool_desc *pools, int32_t n_pools, hipStream_t s,
                                 const Workspace16 *ready, size_t *meta_bytes)
{
    plan_batch(pools, n_pools, 0, false, plan, -1, ready);
    if (plan.ws_bytes > dev_bytes) {
        const size_t cap = bytes_after(plan.ws_bytes);
        if (dev) stream_free(dev, s);
        dev = nullptr;
        dev_bytes = 0;
        hipError_t e = stream_alloc((void **)&dev, cap, s);
        if (e != hipSuccess) return e;
        dev_bytes = cap;
    }
    *meta_bytes = plan.meta_bytes;
    return hipSuccess;
}

void BatchArena::stage(char *dmeta, char *hdst)
{
    layout_batch(plan, (char *)dev, meta, dmeta);
    std::memcpy(hdst, meta.data(), meta.size());
}

hipError_t BatchArena::launch(hipStream_t s)
{
    int d = 0;
    if (plan.form == kBatchPersistent) {
        hipError_t e = hipGetDevice(&d);
        if (e != hipSuccess) return e;
    }
    return enqueue_batch(plan, plan.form == kBatchPersistent ? batch_grid(d, plan.scan_lds) : 0, s);
}

void BatchArena::release(hipStream_t s)
{
    if (dev) stream_free(dev, s);
    dev = nullptr;
    dev_bytes = 0;
    if (pinned) {
        hipStreamSynchronize(s);
        pinned_put(pinned, pinned_bytes);
    }
    pinned = nullptr;
    pinned_bytes = 0;
}

}  // namespace fspbb

struct fsp_batch_s {
    int device = 0;
    BatchPlan plan;
    void *dblob = nullptr;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

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

fsp_status fail(hipError_t e)
{
    set_last_error(e);
    return e == hipErrorOutOfMemory ? FSP_E_NOMEM : FSP_E_DEVICE;
}

void free_batch(fsp_batch_s *b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->dblob) hipFree(b->dblob);
    delete b;
}

}  // namespace

namespace fspbb {

// fsp_batch_create with an optional forced waves-per-group (0 = tuned).
fsp_status create_batch(const fsp_pool_desc *pools, int32_t n_pools, int32_t flags, int32_t wpg_force,
                        int32_t form_force, fsp_batch *out)
{
    if (!out) return FSP_E_INVAL;
    *out = nullptr;
    int dev = -1;
    fsp_status st = check_pools(pools, n_pools, &dev);
    if (st != FSP_OK) return st;
    DeviceGuard g(dev);
    if (!g.ok) return FSP_E_DEVICE;
    fsp_batch_s *b = new fsp_batch_s();
    b->device = dev;
    plan_batch(pools, n_pools, wpg_force, true, b->plan, form_force);
    hipError_t e = hipMalloc(&b->dblob, b->plan.ws_bytes + b->plan.meta_bytes);
    if (e != hipSuccess) { free_batch(b); return fail(e); }
    std::vector<char> meta;
    layout_batch(b->plan, (char *)b->dblob, meta);
    e = hipMemcpy(b->plan.dmeta, meta.data(), meta.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { free_batch(b); return fail(e); }
    b->grid = b->plan.form == kBatchPersistent ? batch_grid(dev, b->plan.scan_lds) : (int)b->plan.items.size();
    if (flags & FSP_BATCH_GRAPH) {
        hipStream_t cs;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) {
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e1 = enqueue_batch(b->plan, b->grid, cs);
                hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
                e = e1 != hipSuccess ? e1 : e2;
            }
            hipStreamDestroy(cs);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) { free_batch(b); return fail(e); }
    }
    *out = b;
    return FSP_OK;
}

}  // namespace fspbb

extern "C" {

fsp_status fsp_batch_create(const fsp_pool_desc *pools, int32_t n_pools, int32_t flags, fsp_batch *out)
{
    return create_batch(pools, n_pools, flags, 0, -1, out);
}

fsp_status fsp_batch_run(fsp_batch b, void *stream)
{
    if (!b) return FSP_E_INVAL;
    DeviceGuard g(b->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = b->exec ? hipGraphLaunch(b->exec, s) : enqueue_batch(b->plan, b->grid, s);
    return e == hipSuccess ? FSP_OK : fail(e);
}

fsp_status fsp_batch_destroy(fsp_batch b)
{
    if (!b) return FSP_OK;
    DeviceGuard g(b->device);
    hipDeviceSynchronize();
    free_batch(b);
    return FSP_OK;
}

fsp_status fsp_batch_info(fsp_batch b, int64_t *total_nodes, int32_t *n_items, int32_t *grid)
{
    if (!b) return FSP_E_INVAL;
    if (total_nodes) *total_nodes = b->plan.total_nodes;
    if (n_items) *n_items = (int32_t)b->plan.items.size();
    if (grid) *grid = b->grid;
    return FSP_OK;
}

fsp_status fsp_bound_pools_batched(const fsp_pool_desc *pools, int32_t n_pools, void *stream)
{
    fsp_batch b = nullptr;
    fsp_status st = fsp_batch_create(pools, n_pools, 0, &b);
    if (st != FSP_OK) return st;
    st = fsp_batch_run(b, stream);
    hipStreamSynchronize((hipStream_t)stream);
    fsp_batch_destroy(b);
    return st;
}

}  // extern "C"
