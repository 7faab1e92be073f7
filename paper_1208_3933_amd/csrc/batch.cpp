// Batched bounding of many pools (possibly of different instances and
// shapes) in one decode launch per machine-count class and one persistent
// scan launch, captured once in a HIP graph and replayed.
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
}  // namespace

ScanTuning scan_tuning(int n, int m)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find({n, m});
        if (it != g_tune.end()) return it->second;
    }
    // rule of thumb: about four machine pairs per wave and chain
    const int P = m * (m - 1) / 2;
    int w = 1;
    while (w < kBatchWaves && 4 * 2 * w <= P) w *= 2;
    return ScanTuning{w, 8};
}

void set_scan_tuning(int n, int m, ScanTuning t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[{n, m}] = t;
}

}  // namespace fspbb

struct fsp_batch_s {
    int device = 0;
    int n_pools = 0;
    int64_t total_nodes = 0;
    std::vector<BatchPool> hpools;
    std::vector<WorkItem> hitems;
    struct DecodeClass {
        int MV;
        int64_t nblocks;
        size_t lds;
        int64_t *dblk_off;
        int32_t *dcls;
        int ncls;
    };
    std::vector<DecodeClass> classes;
    BatchPool *dpools = nullptr;
    WorkItem *ditems = nullptr;
    uint32_t *dcounter = nullptr;
    void *dblob = nullptr;
    int grid = 0;
    size_t scan_lds = 0;
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

hipError_t enqueue(const fsp_batch_s *b, hipStream_t s)
{
    for (const auto &c : b->classes) {
        hipError_t e = launch_batch_decode(c.MV, b->dpools, c.dblk_off, c.dcls, c.ncls, c.nblocks, c.lds, s);
        if (e != hipSuccess) return e;
    }
    if (b->hitems.empty()) return hipSuccess;
    return launch_batch_scan(b->dpools, b->ditems, (int)b->hitems.size(), b->dcounter, b->grid, b->scan_lds, s);
}

void free_batch(fsp_batch_s *b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->dblob) hipFree(b->dblob);
    delete b;
}

}  // namespace

extern "C" {

fsp_status fsp_batch_create(const fsp_pool_desc *pools, int32_t n_pools, int32_t flags, fsp_batch *out)
{
    if (!out) return FSP_E_INVAL;
    *out = nullptr;
    if (!pools || n_pools < 1) return FSP_E_INVAL;
    const int dev = pools[0].inst ? pools[0].inst->device : -1;
    for (int i = 0; i < n_pools; ++i) {
        const fsp_pool_desc &d = pools[i];
        if (!d.inst || d.N < 0 || d.inst->device != dev) return FSP_E_INVAL;
        if (!d.inst->packed16) return FSP_E_INVAL;
        if (d.N > 0 && (!d.prefixes || !d.depths || !d.out_lb)) return FSP_E_INVAL;
    }
    DeviceGuard g(dev);
    if (!g.ok) return FSP_E_DEVICE;

    fsp_batch_s *b = new fsp_batch_s();
    b->device = dev;
    b->n_pools = n_pools;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };

    // workspace layout and pool records
    std::vector<size_t> ws_off(n_pools);
    size_t ws = 0;
    b->hpools.resize(n_pools);
    struct Cost { int64_t cost; WorkItem w; };
    std::vector<Cost> items;
    size_t scan_lds = 64 * kBatchWaves * 4;  // the cross-wave reduction reuses the mask area
    for (int i = 0; i < n_pools; ++i) {
        const fsp_pool_desc &d = pools[i];
        const fsp_instance_s *I = d.inst;
        const int n = I->n, m = I->m, NW = (n + 31) >> 5;
        const int64_t G = (d.N + kGroup - 1) / kGroup, Npad = G * kGroup;
        ws_off[i] = ws;
        ws += al((size_t)G * 3 * m * 64 * 4) + al((size_t)G * NW * 128 * 4) + al((size_t)Npad * 4);
        BatchPool &P = b->hpools[i];
        std::memset(&P, 0, sizeof(P));
        P.T = I->dt;
        P.prefixes = d.prefixes;
        P.depths = d.depths;
        P.out_lb = d.out_lb;
        P.N = d.N;
        P.Npad = Npad;
        P.wpg = scan_tuning(n, m).waves_per_group;
        const int gpp = kBatchWaves / P.wpg;
        for (int64_t g0 = 0; g0 < G; g0 += gpp) {
            const int ng = (int)std::min<int64_t>(gpp, G - g0);
            const int64_t per_wave = (I->P + P.wpg - 1) / P.wpg;
            items.push_back({per_wave * I->dt.npad, WorkItem{i, (int32_t)g0, ng, 0}});
        }
        if (G > 0) scan_lds = std::max(scan_lds, (size_t)std::min<int64_t>(gpp, G) * (n + 1) * 256);
        b->total_nodes += d.N;
    }
    std::stable_sort(items.begin(), items.end(), [](const Cost &x, const Cost &y) { return x.cost > y.cost; });
    for (auto &c : items) b->hitems.push_back(c.w);
    b->scan_lds = scan_lds;

    // decode classes by machine count rounded up to 4
    std::map<int, std::vector<int>> cls;
    for (int i = 0; i < n_pools; ++i)
        if (pools[i].N > 0) cls[(pools[i].inst->m + 3) & ~3].push_back(i);
    size_t meta = al(sizeof(BatchPool) * n_pools) + al(sizeof(WorkItem) * std::max<size_t>(1, b->hitems.size())) + 256;
    for (auto &kv : cls) meta += al(sizeof(int64_t) * (kv.second.size() + 1)) + al(sizeof(int32_t) * kv.second.size());
    hipError_t e = hipMalloc(&b->dblob, al(ws) + meta);
    if (e != hipSuccess) { free_batch(b); return fail(e); }
    char *base = (char *)b->dblob;
    for (int i = 0; i < n_pools; ++i) {
        const fsp_instance_s *I = pools[i].inst;
        const int n = I->n, m = I->m, NW = (n + 31) >> 5;
        const int64_t G = (pools[i].N + kGroup - 1) / kGroup;
        char *w = base + ws_off[i];
        BatchPool &P = b->hpools[i];
        P.W.dec = (uint32_t *)w;
        P.W.flg = (uint32_t *)(w + al((size_t)G * 3 * m * 64 * 4));
        P.W.st = (uint32_t *)(w + al((size_t)G * 3 * m * 64 * 4) + al((size_t)G * NW * 128 * 4));
        P.W.order = nullptr;
        P.W.cnt = nullptr;
    }
    char *mp = base + al(ws);
    b->dpools = (BatchPool *)mp; mp += al(sizeof(BatchPool) * n_pools);
    b->ditems = (WorkItem *)mp; mp += al(sizeof(WorkItem) * std::max<size_t>(1, b->hitems.size()));
    b->dcounter = (uint32_t *)mp; mp += 256;
    e = hipMemcpy(b->dpools, b->hpools.data(), sizeof(BatchPool) * n_pools, hipMemcpyHostToDevice);
    if (e == hipSuccess && !b->hitems.empty())
        e = hipMemcpy(b->ditems, b->hitems.data(), sizeof(WorkItem) * b->hitems.size(), hipMemcpyHostToDevice);
    for (auto &kv : cls) {
        fsp_batch_s::DecodeClass c{};
        c.MV = kv.first;
        std::vector<int64_t> off(kv.second.size() + 1, 0);
        int nmax = 0;
        for (size_t q = 0; q < kv.second.size(); ++q) {
            const BatchPool &P = b->hpools[kv.second[q]];
            off[q + 1] = off[q] + (P.Npad + 255) / 256;
            nmax = std::max(nmax, (int)P.T.n);
        }
        c.nblocks = off.back();
        c.ncls = (int)kv.second.size();
        c.lds = (size_t)16 * 256 * 4 + (size_t)(nmax + 1) * c.MV * 4;
        c.dblk_off = (int64_t *)mp; mp += al(sizeof(int64_t) * off.size());
        c.dcls = (int32_t *)mp; mp += al(sizeof(int32_t) * kv.second.size());
        if (e == hipSuccess) e = hipMemcpy(c.dblk_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(c.dcls, kv.second.data(), sizeof(int32_t) * kv.second.size(), hipMemcpyHostToDevice);
        b->classes.push_back(c);
    }
    if (e != hipSuccess) { free_batch(b); return fail(e); }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) { free_batch(b); return fail(e); }
    b->grid = prop.multiProcessorCount * batch_scan_blocks_per_cu(b->scan_lds);

    if (flags & FSP_BATCH_GRAPH) {
        hipStream_t cs;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e1 = enqueue(b, cs);
            hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
            e = e1 != hipSuccess ? e1 : e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        hipStreamDestroy(cs);
        if (e != hipSuccess) { free_batch(b); return fail(e); }
    }
    *out = b;
    return FSP_OK;
}

fsp_status fsp_batch_run(fsp_batch b, void *stream)
{
    if (!b) return FSP_E_INVAL;
    DeviceGuard g(b->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = b->exec ? hipGraphLaunch(b->exec, s) : enqueue(b, s);
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
    if (total_nodes) *total_nodes = b->total_nodes;
    if (n_items) *n_items = (int32_t)b->hitems.size();
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
