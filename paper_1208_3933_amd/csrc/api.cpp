// C ABI entry points of the bound path (include/fspbb.h).
#include <cstdint>
#include <map>
#include <unordered_map>
#include <mutex>

#include "fspbb_internal.h"
#include "bound_wide.h"

using namespace fspbb;

namespace {

// Makes the instance's device current for the duration of a call.
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

}  // namespace

namespace fspbb {

namespace {
// Blocks released by stream_free, kept for reuse by a later stream_alloc on
// the same device and stream (stream order then guarantees that the earlier
// work on a block is done before the new work starts).  Freeing a block back
// to the driver's pool costs tens of microseconds to milliseconds of host
// time per call; a search's set-up and tear-down make about twenty of them.
struct CachedBlock {
    void *ptr;
    size_t cap;
    int dev;
    hipStream_t s;
};
std::mutex g_blk_mu;
std::unordered_map<void *, std::pair<size_t, int>> g_live;  // block -> (capacity, device)
std::vector<CachedBlock> g_cached;
size_t g_cached_bytes = 0;
constexpr size_t kCacheBytes = (size_t)16 << 30, kCacheBlocks = 256;
}  // namespace

hipError_t stream_alloc(void **ptr, size_t bytes, hipStream_t s)
{
    int cdev = 0;
    hipError_t ce = hipGetDevice(&cdev);
    if (ce != hipSuccess) return ce;
    {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        size_t best = g_cached.size();
        for (size_t i = 0; i < g_cached.size(); ++i) {
            const CachedBlock &c = g_cached[i];
            if (c.dev != cdev || c.s != s || c.cap < bytes || c.cap > 2 * bytes + ((size_t)1 << 20)) continue;
            if (best == g_cached.size() || c.cap < g_cached[best].cap) best = i;
        }
        if (best < g_cached.size()) {
            const CachedBlock c = g_cached[best];
            g_cached.erase(g_cached.begin() + (std::ptrdiff_t)best);
            g_cached_bytes -= c.cap;
            g_live[c.ptr] = {c.cap, c.dev};
            *ptr = c.ptr;
            return hipSuccess;
        }
    }
    hipError_t e = pool_alloc(ptr, bytes, s);
    if (e == hipErrorOutOfMemory) {
        // kept blocks of this device go back to the pool, then one more try
        std::vector<CachedBlock> mine;
        {
            std::lock_guard<std::mutex> lk(g_blk_mu);
            for (size_t i = 0; i < g_cached.size();) {
                if (g_cached[i].dev == cdev) {
                    mine.push_back(g_cached[i]);
                    g_cached_bytes -= g_cached[i].cap;
                    g_cached.erase(g_cached.begin() + (std::ptrdiff_t)i);
                } else {
                    ++i;
                }
            }
        }
        if (!mine.empty()) {
            hipGetLastError();  // clear the failed allocation's error
            hipError_t se = hipDeviceSynchronize();  // their streams may be gone
            for (const CachedBlock &c : mine)
                if (se == hipSuccess) se = hipFreeAsync(c.ptr, nullptr);
            if (se == hipSuccess) se = hipDeviceSynchronize();
            e = se == hipSuccess ? pool_alloc(ptr, bytes, s) : se;
        }
    }
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        g_live[*ptr] = {bytes, cdev};
    }
    return e;
}

hipError_t stream_free(void *ptr, hipStream_t s)
{
    if (!ptr) return hipSuccess;
    {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        auto it = g_live.find(ptr);
        if (it != g_live.end()) {
            const size_t cap = it->second.first;
            const int dev = it->second.second;
            g_live.erase(it);
            if (g_cached_bytes + cap <= kCacheBytes && g_cached.size() < kCacheBlocks) {
                g_cached.push_back(CachedBlock{ptr, cap, dev, s});
                g_cached_bytes += cap;
                return hipSuccess;
            }
        }
    }
    return hipFreeAsync(ptr, s);
}

namespace {
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;  // per device
}  // namespace

hipError_t pool_alloc(void **ptr, size_t bytes, hipStream_t s)
{
    std::mutex &mu = g_pool_mu;
    std::map<int, hipMemPool_t> &pools = g_pools;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = pools.find(dev);
        if (it != pools.end()) {
            pool = it->second;
        } else {
            hipMemPoolProps props{};
            props.allocType = hipMemAllocationTypePinned;
            props.handleTypes = hipMemHandleTypeNone;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = dev;
            e = hipMemPoolCreate(&pool, &props);
            if (e != hipSuccess) return e;
            uint64_t keep = UINT64_MAX;
            e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            if (e != hipSuccess) {
                hipMemPoolDestroy(pool);
                return e;
            }
            pools[dev] = pool;
        }
    }
    return hipMallocFromPoolAsync(ptr, bytes, pool, s);
}

namespace {
std::mutex g_pinned_mu;
std::vector<std::pair<void *, size_t>> g_pinned;  // kept buffers and their capacities
constexpr size_t kPinnedKeep = 16;
}  // namespace

hipError_t pinned_get(void **ptr, size_t *cap, size_t bytes)
{
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        size_t best = g_pinned.size();
        for (size_t i = 0; i < g_pinned.size(); ++i)
            if (g_pinned[i].second >= bytes && (best == g_pinned.size() || g_pinned[i].second < g_pinned[best].second))
                best = i;
        if (best < g_pinned.size()) {
            *ptr = g_pinned[best].first;
            *cap = g_pinned[best].second;
            g_pinned.erase(g_pinned.begin() + (std::ptrdiff_t)best);
            return hipSuccess;
        }
    }
    *ptr = nullptr;
    *cap = 0;
    hipError_t e = hipHostMalloc(ptr, bytes, 0);
    if (e == hipSuccess) *cap = bytes;
    else *ptr = nullptr;
    return e;
}

void pinned_put(void *ptr, size_t cap)
{
    if (!ptr) return;
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        if (g_pinned.size() < kPinnedKeep) {
            g_pinned.emplace_back(ptr, cap);
            return;
        }
    }
    hipHostFree(ptr);
}

void timing_mark(fsp_instance_s *I, int which, hipStream_t s)
{
    if (!I->timing) return;
    if (!I->timing_log) I->timing_log = new std::vector<TimingRecord>();
    if (which == 0) {
        // chained timing: the launch starts where the previous one's scan
        // ended (ev[0] stays null), one event record fewer per launch
        const bool chain = I->timing == 2 && !I->timing_log->empty();
        TimingRecord r{};
        for (int k = chain ? 1 : 0; k < 3; ++k) hipEventCreate(&r.ev[k]);
        I->timing_log->push_back(r);
        if (chain) return;
    }
    if (!I->timing_log->empty()) hipEventRecord(I->timing_log->back().ev[which], s);
}
}  // namespace fspbb

namespace {

fsp_status dispatch(fsp_instance inst, const int32_t *prefixes, const int32_t *depths, int64_t N,
                    int32_t *out_lb, int variant, void *stream)
{
    if (!inst || N < 0) return FSP_E_INVAL;
    if (N == 0) return FSP_OK;
    if (!prefixes || !depths || !out_lb) return FSP_E_INVAL;
    if (variant == 0) variant = inst->packed16 ? 2 : 4;
    if (variant == 2 && !inst->packed16) return FSP_E_INVAL;
    if (variant < 1 || variant > 4) return FSP_E_INVAL;
    DeviceGuard g(inst->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    fsp_instance_s *I = const_cast<fsp_instance_s *>(inst);
    hipError_t e = variant == 1   ? launch_bound_lane32(I, prefixes, depths, N, out_lb, s)
                   : variant == 2 ? launch_bound_packed(I, prefixes, depths, N, out_lb, s)
                   : variant == 3 ? launch_bound_wavepair(I, prefixes, depths, N, out_lb, s)
                                  : launch_bound_wide(I, prefixes, depths, N, out_lb, s);
    if (e != hipSuccess) {
        set_last_error(e);
        return e == hipErrorOutOfMemory ? FSP_E_NOMEM : FSP_E_DEVICE;
    }
    return FSP_OK;
}

}  // namespace

extern "C" {

fsp_status fsp_bound_pool(fsp_instance inst, const int32_t *prefixes, const int32_t *depths, int64_t N,
                          int32_t *out_lb, void *stream)
{
    return dispatch(inst, prefixes, depths, N, out_lb, 0, stream);
}

fsp_status fsp_bound_pool_variant(fsp_instance inst, const int32_t *prefixes, const int32_t *depths,
                                  int64_t N, int32_t *out_lb, int32_t variant, void *stream)
{
    return dispatch(inst, prefixes, depths, N, out_lb, variant, stream);
}

fsp_status fsp_pool_status(fsp_instance inst, void *stream, int64_t *n_bad)
{
    if (!inst) return FSP_E_INVAL;
    DeviceGuard g(inst->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long cnt = 0;
    hipError_t e = hipMemcpyAsync(&cnt, inst->dt.bad, sizeof(cnt), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemsetAsync(inst->dt.bad, 0, sizeof(cnt), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_last_error(e); return FSP_E_DEVICE; }
    if (n_bad) *n_bad = (int64_t)cnt;
    return cnt ? FSP_E_BADNODE : FSP_OK;
}

fsp_status fsp_timing_enable(fsp_instance inst, int32_t on)
{
    if (!inst) return FSP_E_INVAL;
    inst->timing = on == 2 ? 2 : on ? 1 : 0;
    return FSP_OK;
}

fsp_status fsp_timing_read(fsp_instance inst, double *decode_ms, double *scan_ms, int64_t *launches)
{
    if (!inst) return FSP_E_INVAL;
    DeviceGuard g(inst->device);
    double dsum = 0, ssum = 0;
    int64_t cnt = 0;
    hipError_t err = hipSuccess;
    if (inst->timing_log) {
        std::vector<TimingRecord> &log = *inst->timing_log;
        for (size_t i = 0; i < log.size(); ++i) {
            const TimingRecord &r = log[i];
            // a chained record starts at the previous record's end
            hipEvent_t start = r.ev[0] ? r.ev[0] : (i > 0 ? log[i - 1].ev[2] : nullptr);
            float a = 0, b = 0;
            hipError_t e = start ? hipEventSynchronize(r.ev[2]) : hipErrorInvalidValue;
            if (e == hipSuccess) e = hipEventElapsedTime(&a, start, r.ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&b, r.ev[1], r.ev[2]);
            if (e != hipSuccess) err = e;
            dsum += a;
            ssum += b;
            ++cnt;
        }
        for (auto &r : log)
            for (auto &ev : r.ev)
                if (ev) hipEventDestroy(ev);
        inst->timing_log->clear();
    }
    if (decode_ms) *decode_ms = dsum;
    if (scan_ms) *scan_ms = ssum;
    if (launches) *launches = cnt;
    if (err != hipSuccess) { set_last_error(err); return FSP_E_DEVICE; }
    return FSP_OK;
}

fsp_status fsp_release_cached(void)
{
    std::vector<CachedBlock> blocks;
    {
        std::lock_guard<std::mutex> lk(g_blk_mu);
        blocks.swap(g_cached);
        g_cached_bytes = 0;
    }
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (blocks.empty() && g_pools.empty()) return FSP_OK;  // nothing was ever allocated
    }
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return FSP_E_DEVICE;
    hipError_t err = hipSuccess;
    std::map<int, bool> synced;
    for (const CachedBlock &c : blocks) {
        hipError_t e = hipSetDevice(c.dev);
        if (e == hipSuccess && !synced[c.dev]) e = hipDeviceSynchronize();  // the blocks' streams may be gone
        synced[c.dev] = true;
        if (e == hipSuccess) e = hipFreeAsync(c.ptr, nullptr);
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (auto &dp : g_pools) {
            hipError_t e = hipSetDevice(dp.first);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e == hipSuccess) e = hipMemPoolTrimTo(dp.second, 0);
            if (e != hipSuccess && err == hipSuccess) err = e;
        }
    }
    hipSetDevice(cur);
    if (err != hipSuccess) {
        set_last_error(err);
        return FSP_E_DEVICE;
    }
    return FSP_OK;
}

}  // extern "C"
