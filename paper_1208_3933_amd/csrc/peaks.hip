// Peak probes: one kernel per unit that the bound kernels can saturate, timed
// with HIP events, so that a kernel's achieved rate can be set against what
// the chip delivers at its running clock as well as against the spec sheet.
//
//   valu16  chains of packed 16-bit max and add, the scan's arithmetic;
//   valu32  the same chains in 32-bit lanes (the lane-per-node mapping);
//   lds     16-byte LDS reads, conflict-free (the wave-per-node mapping);
//   hbm     a copy between two device buffers, four 16-byte non-temporal
//           loads per lane in flight.
//
// Every kernel keeps its results live with one store per lane, so nothing is
// removed by the compiler; each launch fills the chip (2,048 groups of 256).
#include "fspbb_internal.h"

namespace fspbb {

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kGroups = 2048, kThreads = 256, kChains = 8;
constexpr int kValuIters = 4096, kLdsIters = 2048;
constexpr int kLdsWords = 4096;  // uint4 entries: 64 KiB per group
constexpr int kTimed = 5;        // timed launches, averaged

__global__ __launch_bounds__(256) void probe_valu16_kernel(uint32_t e0, uint32_t c0, int iters, uint32_t *out)
{
    const u16x2 E = __builtin_bit_cast(u16x2, e0), C = __builtin_bit_cast(u16x2, c0);
    u16x2 s[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) s[k] = __builtin_bit_cast(u16x2, threadIdx.x * 0x10001u + (uint32_t)k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) s[k] = __builtin_elementwise_max(s[k], E) + C;
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) x ^= __builtin_bit_cast(uint32_t, s[k]);
    out[blockIdx.x * kThreads + threadIdx.x] = x;
}

__global__ __launch_bounds__(256) void probe_valu32_kernel(uint32_t e0, uint32_t c0, int iters, uint32_t *out)
{
    uint32_t s[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) s[k] = threadIdx.x * 7u + (uint32_t)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) s[k] = max(s[k], e0) + c0;
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) x ^= s[k];
    out[blockIdx.x * kThreads + threadIdx.x] = x;
}

// Eight 16-byte reads per iteration at fixed offsets 4 KiB apart from a
// window that moves by `step` (uniform, unknown at compile time) each time.
// The reads and their wait are one instruction block, so that the compiler
// can neither narrow them to the words consumed nor use a result before it
// has arrived; only two words of each are folded into the result, which
// keeps the vector ALU from limiting the rate.  The window start stays below
// entry 2,048, so the last read ends at byte 61,440 of the 64 KiB array.
__global__ __launch_bounds__(256) void probe_lds_kernel(int iters, int step, uint32_t *out)
{
    __shared__ uint4 buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += kThreads)
        buf[i] = make_uint4((uint32_t)i, (uint32_t)i * 3u, (uint32_t)i * 5u, (uint32_t)i * 7u);
    __syncthreads();
    const uint32_t lds0 = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint4 *)buf;
    uint32_t acc = 0;
    int base = threadIdx.x;
    for (int it = 0; it < iters; ++it) {
        const uint32_t addr = lds0 + (uint32_t)(base & 2047) * 16u;
        u32x4 v0, v1, v2, v3, v4, v5, v6, v7;
        asm volatile("ds_read_b128 %0, %8\n\t"
                     "ds_read_b128 %1, %8 offset:4096\n\t"
                     "ds_read_b128 %2, %8 offset:8192\n\t"
                     "ds_read_b128 %3, %8 offset:12288\n\t"
                     "ds_read_b128 %4, %8 offset:16384\n\t"
                     "ds_read_b128 %5, %8 offset:20480\n\t"
                     "ds_read_b128 %6, %8 offset:24576\n\t"
                     "ds_read_b128 %7, %8 offset:28672\n\t"
                     "s_waitcnt lgkmcnt(0)"
                     : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3), "=&v"(v4), "=&v"(v5), "=&v"(v6), "=&v"(v7)
                     : "v"(addr)
                     : "memory");
        acc ^= v0.x ^ v0.w ^ v1.x ^ v1.w ^ v2.x ^ v2.w ^ v3.x ^ v3.w;
        acc ^= v4.x ^ v4.w ^ v5.x ^ v5.w ^ v6.x ^ v6.w ^ v7.x ^ v7.w;
        base += step;
    }
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

// Four independent 16-byte loads in flight per lane before their stores;
// each lane's four elements are one grid stride apart.  A lane whose four
// elements are all in range takes the unchecked form, with non-temporal loads
// and stores (streamed data: 5.1 TB/s against 4.45 for plain ones); the
// others check each element.
__global__ __launch_bounds__(256) void probe_copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                          int64_t n16)
{
    const int64_t S = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += 4 * S) {
        if (i + 3 * S < n16) {
            const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src);
            u32x4 *d4 = reinterpret_cast<u32x4 *>(dst);
            const u32x4 a = __builtin_nontemporal_load(s4 + i), b = __builtin_nontemporal_load(s4 + i + S);
            const u32x4 c = __builtin_nontemporal_load(s4 + i + 2 * S), d = __builtin_nontemporal_load(s4 + i + 3 * S);
            __builtin_nontemporal_store(a, d4 + i);
            __builtin_nontemporal_store(b, d4 + i + S);
            __builtin_nontemporal_store(c, d4 + i + 2 * S);
            __builtin_nontemporal_store(d, d4 + i + 3 * S);
        } else {
            for (int64_t k = i; k < n16; k += S) dst[k] = src[k];
        }
    }
}

}  // namespace

}  // namespace fspbb

using namespace fspbb;

extern "C" fsp_status fsp_probe_peak(int32_t kind, int64_t bytes, void *stream, double *rate, double *ms)
{
    if (!rate || kind < FSP_PROBE_VALU16 || kind > FSP_PROBE_HBM) return FSP_E_INVAL;
    if (kind == FSP_PROBE_HBM && (bytes < (1 << 20) || bytes % 16 != 0)) return FSP_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *out = nullptr;
    void *src = nullptr, *dst = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    fsp_status st = FSP_OK;
    float t = 0.f;
    hipError_t e = hipMalloc((void **)&out, (size_t)kGroups * kThreads * 4);
    if (e == hipSuccess && kind == FSP_PROBE_HBM) {
        e = hipMalloc(&src, (size_t)bytes);
        if (e == hipSuccess) e = hipMalloc(&dst, (size_t)bytes);
        if (e == hipSuccess) e = hipMemsetAsync(src, 1, (size_t)bytes, s);
    }
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // three untimed launches (code load, clocks up), then kTimed timed ones
    for (int rep = 0; e == hipSuccess && rep < 3 + kTimed; ++rep) {
        if (rep == 3) e = hipEventRecord(a, s);
        if (e != hipSuccess) break;
        switch (kind) {
        case FSP_PROBE_VALU16:
            probe_valu16_kernel<<<kGroups, kThreads, 0, s>>>(0x00050005u, 0x00030003u, kValuIters, out);
            break;
        case FSP_PROBE_VALU32:
            probe_valu32_kernel<<<kGroups, kThreads, 0, s>>>(5u, 3u, kValuIters, out);
            break;
        case FSP_PROBE_LDS:
            probe_lds_kernel<<<kGroups, kThreads, 0, s>>>(kLdsIters, 8 * kThreads + 16, out);
            break;
        default:
            probe_copy_kernel<<<4 * kGroups, kThreads, 0, s>>>((const uint4 *)src, (uint4 *)dst, bytes / 16);
            break;
        }
        e = hipGetLastError();
        if (e == hipSuccess && rep == 3 + kTimed - 1) e = hipEventRecord(b, s);
    }
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e != hipSuccess) {
        set_last_error(e);
        st = e == hipErrorOutOfMemory ? FSP_E_NOMEM : FSP_E_DEVICE;
    } else {
        const double lanes = (double)kGroups * kThreads, sec = t * 1e-3 / kTimed;
        double work = 0;
        switch (kind) {
        case FSP_PROBE_VALU16: work = lanes * kValuIters * kChains * 4.0; break;  // 2 packed ops x 2 halves
        case FSP_PROBE_VALU32: work = lanes * kValuIters * kChains * 2.0; break;
        case FSP_PROBE_LDS: work = lanes * kLdsIters * 8 * 16.0; break;
        default: work = 2.0 * (double)bytes; break;
        }
        *rate = work / sec;
        if (ms) *ms = t / kTimed;
    }
    hipStreamSynchronize(s);
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    if (out) hipFree(out);
    if (src) hipFree(src);
    if (dst) hipFree(dst);
    return st;
}
