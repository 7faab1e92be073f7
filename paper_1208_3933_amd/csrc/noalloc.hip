// fsp_bound_pool_noalloc: pool bounding that makes no allocation at all.
//
// The decode of the 16-bit and of the 32-bit path writes a workspace
// (releases, closing sums and tails per node, unscheduled-job bits, the depth
// order and the sort counts) that the scan then reads.  fsp_bound_pool takes it from the library's
// stream-ordered pool; this entry point takes it from `scratch`, a fixed
// array in the code object, so that callers which may not allocate (work
// under graph capture, tight serving loops, harnesses that forbid it) can
// still bound pools.  Every device the library runs on holds its own copy of
// the array until the process ends.  The host may not use the array's name as
// a device address: the address of each device's copy is looked up once, with
// that device current, and only that address is passed to kernels.
#include <mutex>

#include "bound_wide.h"
#include "fspbb_internal.h"

namespace fspbb {
namespace {

static __device__ __align__(256) unsigned char scratch[FSP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of each device's copy, or null before its set-up

// Address of the current device's copy of `scratch` (looked up on the first
// call on that device), or an error.
hipError_t scratch_for(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Makes `dev` current for the life of the guard (no allocation).
struct CurrentDevice {
    int prev = -1;
    bool ok = true;
    explicit CurrentDevice(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~CurrentDevice()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

}  // namespace
}  // namespace fspbb

extern "C" {

namespace {
// Workspace bytes of the path fsp_bound_pool takes for N nodes.
size_t workspace_bytes(const fsp_instance_s *I, int64_t N)
{
    return I->packed16 ? fspbb::packed_workspace_bytes(I, N) : fspbb::wide_workspace_bytes(I, N);
}
}  // namespace

int64_t fsp_noalloc_max_nodes(fsp_instance inst)
{
    if (!inst) return -1;
    // largest N whose workspace fits (the size is monotone in N)
    int64_t lo = 0, hi = (int64_t)1 << 40;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (workspace_bytes(inst, mid) <= (size_t)FSP_NOALLOC_SCRATCH_BYTES)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

fsp_status fsp_bound_pool_noalloc(fsp_instance inst, const int32_t *prefixes, const int32_t *depths, int64_t N,
                                  int32_t *out_lb, void *stream)
{
    using namespace fspbb;
    if (!inst || N < 0) return FSP_E_INVAL;
    if (N == 0) return FSP_OK;
    if (!prefixes || !depths || !out_lb) return FSP_E_INVAL;
    fsp_instance_s *I = const_cast<fsp_instance_s *>(inst);
    if (workspace_bytes(I, N) > (size_t)FSP_NOALLOC_SCRATCH_BYTES) return FSP_E_RANGE;
    CurrentDevice g(I->device);
    if (!g.ok) return FSP_E_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    hipError_t e = scratch_for(I->device, &ws);
    if (e == hipSuccess)
        e = I->packed16 ? launch_bound_packed_ws(I, prefixes, depths, N, out_lb, s, true, ws, false)
                        : launch_bound_wide_ws(I, prefixes, depths, N, out_lb, s, true, ws, false);
    if (e != hipSuccess) {
        set_last_error(e);
        return FSP_E_DEVICE;
    }
    return FSP_OK;
}

}  // extern "C"
