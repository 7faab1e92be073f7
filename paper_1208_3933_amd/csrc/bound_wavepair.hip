// Wave-per-node bound kernels (32-bit), the alternative mapping to the
// lane-per-node design: one wavefront per node, one lane per machine pair.
//
//   decode  one lane per node (the shared decode_node): releases, closing
//           sums, tails and the unscheduled set go to a workspace;
//   scan    one wave per node.  Lane L scans pairs L, L + 64, ... over the
//           Johnson-with-lags order of each; the records of slot i of every
//           pair are contiguous (the slot-major table), so a wave reads one
//           slot of 64 pairs with one coalesced load.  The node's unscheduled
//           set is one 16-word row of LDS per wave, read per lane at the
//           record's job word.  The bound is the wave's maximum over its
//           lanes (a shuffle reduction).
// Per slot and pair the lane does a 16-byte record load, an LDS read, and the
// same max/add/select as the other kernels, for one node, where the
// lane-per-node kernels share one scalar record load between 64 or 128 nodes.
#include "bound_common.h"

namespace fspbb {

namespace {

template <int MV>
__global__ __launch_bounds__(256) void wp_decode_kernel(DevTables T, const int32_t *__restrict__ prefixes,
                                                        const int32_t *__restrict__ depths, int64_t N,
                                                        int32_t *__restrict__ rtq, uint32_t *__restrict__ act,
                                                        int32_t *__restrict__ okf, int32_t *__restrict__ out_lb)
{
    __shared__ uint32_t bits[kMaskWords * 256];
    const int tid = threadIdx.x;
    const int64_t node = (int64_t)blockIdx.x * 256 + tid;
    const bool live = node < N;
    const int n = T.n;
    const int d = live ? depths[node] : 0;
    Decoded<MV> D;
    decode_node<MV>(T, prefixes + (live ? node : 0) * (int64_t)n, d, bits + tid, 256, D);
    if (!live) return;
    int32_t *r = rtq + node * 3 * MV;
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        r[k] = D.R[k];
        r[MV + k] = D.Tk[k];
        r[2 * MV + k] = D.Qv[k];
    }
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) act[node * kMaskWords + w] = D.act[w];
    okf[node] = D.ok ? 1 : 0;
    if (!D.ok) {
        out_lb[node] = FSP_LB_INVALID;
        atomicAdd(T.bad, 1ull);
    }
}

template <int MV>
__global__ __launch_bounds__(256) void wp_scan_kernel(DevTables T, int64_t N, const int32_t *__restrict__ rtq,
                                                      const uint32_t *__restrict__ act,
                                                      const int32_t *__restrict__ okf, int32_t *__restrict__ out_lb)
{
    __shared__ uint32_t sact[4][kMaskWords];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t node = (int64_t)blockIdx.x * 4 + wv;
    if (node >= N) return;      // whole wave
    if (!okf[node]) return;     // the same value in every lane of the wave
    if (lane < kMaskWords) sact[wv][lane] = act[node * kMaskWords + lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int n = T.n, P = T.P;
    const int32_t *R = rtq + node * 3 * MV, *TK = R + MV, *QV = R + 2 * MV;
    int32_t lb = 0;
    for (int pr = lane; pr < P; pr += 64) {
        const int k = T.pairs[2 * pr], l = T.pairs[2 * pr + 1];
        int32_t s = R[l] - R[k];
        const Rec32 *rec = T.rec32sm + pr;
        for (int i = 0; i < n; ++i) {
            const Rec32 r = rec[(size_t)i * P];
            const int32_t msk = -(int32_t)((sact[wv][r.word] >> r.bit) & 1u);
            const int32_t t = max(s, r.E) + r.C;
            s = (msk & t) | (~msk & s);
        }
        lb = max(lb, TK[k] + s + QV[l]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lb = max(lb, __shfl_xor(lb, off));
    if (lane == 0) out_lb[node] = lb;
}

template <int MV>
hipError_t launch_wp(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N, int32_t *out_lb,
                     hipStream_t s)
{
    const size_t rb = (size_t)N * 3 * MV * 4, ab = (size_t)N * kMaskWords * 4, ob = (size_t)N * 4;
    void *ws = nullptr;
    hipError_t e = stream_alloc(&ws, rb + ab + ob, s);
    if (e != hipSuccess) return e;
    int32_t *rtq = (int32_t *)ws;
    uint32_t *act = (uint32_t *)((char *)ws + rb);
    int32_t *okf = (int32_t *)((char *)ws + rb + ab);
    timing_mark(I, 0, s);
    wp_decode_kernel<MV><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(I->dt, prefixes, depths, N, rtq, act, okf,
                                                                     out_lb);
    timing_mark(I, 1, s);
    wp_scan_kernel<MV><<<(unsigned)((N + 3) / 4), 256, 0, s>>>(I->dt, N, rtq, act, okf, out_lb);
    timing_mark(I, 2, s);
    e = hipGetLastError();
    hipError_t e2 = stream_free(ws, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace

hipError_t launch_bound_wavepair(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N,
                                 int32_t *out_lb, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    if (I->m <= 8) return launch_wp<8>(I, prefixes, depths, N, out_lb, s);
    if (I->m <= 16) return launch_wp<16>(I, prefixes, depths, N, out_lb, s);
    return launch_wp<32>(I, prefixes, depths, N, out_lb, s);
}

}  // namespace fspbb
