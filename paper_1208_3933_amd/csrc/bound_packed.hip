// Fast bound path for instances whose values fit 16 bits ((n+m-1) * max p <
// 65536, true of every U[1,99] instance up to 500 jobs x 20 machines).
//
// Two kernels per pool:
//   decode  one lane per node: scheduled set, releases, closing sums and tails
//           (the per-node RM/QM work of Table I), written to a workspace in a
//           layout the scan reads with unit stride;
//   scan    one workgroup per group of 128 nodes.  Lane L of every wave holds
//           nodes L and L+64 of the group as the two 16-bit halves of each
//           register, so one packed instruction advances two nodes.  The
//           group's unscheduled masks live in LDS as one dword per (job, lane)
//           (0xffff per unscheduled half), shared by all waves; the waves split
//           the machine pairs between them and combine their maxima through
//           LDS at the end.
// The Johnson-with-lags order of a pair is the same for every node, so the
// per-slot records (mask-row offset, lag + a, b - a) are wave-uniform scalar
// loads; only the mask is per lane.  Per slot and wave: one address add, one
// LDS read, one packed max, one packed add and one bitwise select.
#include "bound_common.h"

namespace fspbb {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as16(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

// Workspace of one pool, G = ceil(N / 128) groups.
struct Workspace16 {
    uint32_t *dec;  // G x 3 x m x 64 dwords: releases R, closing sums Tk, tails Q
    uint32_t *flg;  // G x NW x 128 dwords: unscheduled-job bits per node
    uint32_t *st;   // G*128: 1 = valid node
};

template <int MV>
__global__ __launch_bounds__(256) void bound_decode16_kernel(DevTables T, const int32_t *__restrict__ prefixes,
                                                             const int32_t *__restrict__ depths, int64_t N,
                                                             int64_t Npad, Workspace16 W,
                                                             int32_t *__restrict__ out_lb)
{
    __shared__ uint32_t bits[kMaskWords * 256];
    const int tid = threadIdx.x;
    const int64_t node = (int64_t)blockIdx.x * 256 + tid;
    if (node >= Npad) return;
    const bool live = node < N;
    const int n = T.n, m = T.m, NW = (n + 31) >> 5;
    const int d = live ? depths[node] : 0;
    Decoded<MV> D;
    decode_node<MV>(T, prefixes + (live ? node : 0) * (int64_t)n, d, bits + tid, 256, D);
    const bool ok = live && D.ok;

    const int64_t G = node >> 7;
    const int g = (int)(node & 127), lane = g & 63, half = g >> 6;
    uint16_t *d16 = reinterpret_cast<uint16_t *>(W.dec);
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        if (k < m) {
            d16[((G * 3 + 0) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? D.R[k] : 0);
            d16[((G * 3 + 1) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? D.Tk[k] : 0);
            d16[((G * 3 + 2) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? D.Qv[k] : 0);
        }
    }
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w)
        if (w < NW) W.flg[(G * NW + w) * 128 + g] = ok ? D.act[w] : 0u;
    W.st[node] = ok ? 1u : 0u;
    if (live && !D.ok) {
        out_lb[node] = FSP_LB_INVALID;
        atomicAdd(T.bad, 1ull);
    }
}

__device__ __forceinline__ void scan_step(u16x2 &s, const unsigned char *lds_lane, uint32_t joff, uint32_t ce)
{
    const uint32_t msk = *reinterpret_cast<const uint32_t *>(lds_lane + joff);
    const unsigned short e = (unsigned short)(ce >> 16), c = (unsigned short)ce;
    const u16x2 E = {e, e};
    const u16x2 C = {c, c};
    const u16x2 t = __builtin_elementwise_max(s, E) + C;
    s = as16((msk & as32(t)) | (~msk & as32(s)));
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void bound_scan16_kernel(DevTables T, Workspace16 W, int64_t N,
                                                                  int32_t *__restrict__ out_lb)
{
    extern __shared__ uint32_t lds[];  // (n + 1) rows x 64 lanes; row n stays zero
    const int n = T.n, m = T.m, NW = (n + 31) >> 5;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int64_t G = blockIdx.x;

    for (int j = wave; j <= n; j += WAVES) {
        uint32_t m2 = 0;
        if (j < n) {
            const uint32_t *fw = W.flg + (G * NW + (j >> 5)) * 128;
            const uint32_t a = (fw[lane] >> (j & 31)) & 1u, b = (fw[64 + lane] >> (j & 31)) & 1u;
            m2 = (a ? 0x0000ffffu : 0u) | (b ? 0xffff0000u : 0u);
        }
        lds[j * 64 + lane] = m2;
    }
    __syncthreads();

    const unsigned char *lds_lane = reinterpret_cast<const unsigned char *>(lds) + lane * 4;
    const uint32_t *dR = W.dec + (G * 3 + 0) * m * 64 + lane;
    const uint32_t *dT = dR + m * 64;
    const uint32_t *dQ = dT + m * 64;
    u16x2 lb = {0, 0};
    for (int pr = wave; pr < T.P; pr += WAVES) {
        const int k = as_const(T.pairs)[2 * pr], l = as_const(T.pairs)[2 * pr + 1];
        u16x2 s = as16(dR[l * 64]) - as16(dR[k * 64]);
        const uint32_t tk = dT[k * 64], ql = dQ[l * 64];
        cptr<uint32_t> rec = as_const(reinterpret_cast<const uint32_t *>(T.rec16 + (size_t)pr * T.npad));
        for (int i = 0; i < 2 * T.npad; i += 8) {
            uint32_t r[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) r[c] = rec[i + c];
#pragma unroll
            for (int c = 0; c < 8; c += 2) scan_step(s, lds_lane, r[c], r[c + 1]);
        }
        const u16x2 v = as16(tk) + s + as16(ql);
        lb = __builtin_elementwise_max(lb, v);
    }
    __syncthreads();
    lds[wave * 64 + lane] = as32(lb);
    __syncthreads();
    if (wave == 0) {
        u16x2 best = as16(lds[lane]);
#pragma unroll
        for (int w = 1; w < WAVES; ++w) best = __builtin_elementwise_max(best, as16(lds[w * 64 + lane]));
        const int64_t a = G * 128 + lane, b = a + 64;
        if (a < N && W.st[a]) out_lb[a] = (int32_t)best.x;
        if (b < N && W.st[b]) out_lb[b] = (int32_t)best.y;
    }
}

static int scan_waves(int P)
{
    if (P >= 64) return 8;
    if (P >= 16) return 4;
    if (P >= 4) return 2;
    return 1;
}

hipError_t launch_bound_packed(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths,
                               int64_t N, int32_t *out_lb, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    const int n = I->n, m = I->m, NW = (n + 31) >> 5;
    const int64_t G = (N + kGroup - 1) / kGroup, Npad = G * kGroup;
    const size_t dec_b = (size_t)G * 3 * m * 64 * 4, flg_b = (size_t)G * NW * 128 * 4, st_b = (size_t)Npad * 4;
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, dec_b + flg_b + st_b, s);
    if (e != hipSuccess) return e;
    Workspace16 W;
    W.dec = (uint32_t *)ws;
    W.flg = (uint32_t *)((char *)ws + dec_b);
    W.st = (uint32_t *)((char *)ws + dec_b + flg_b);

    const dim3 dgrid((unsigned)((Npad + 255) / 256)), dblock(256);
    timing_mark(I, 0, s);
    if (m <= 8)
        bound_decode16_kernel<8><<<dgrid, dblock, 0, s>>>(I->dt, prefixes, depths, N, Npad, W, out_lb);
    else if (m <= 16)
        bound_decode16_kernel<16><<<dgrid, dblock, 0, s>>>(I->dt, prefixes, depths, N, Npad, W, out_lb);
    else
        bound_decode16_kernel<32><<<dgrid, dblock, 0, s>>>(I->dt, prefixes, depths, N, Npad, W, out_lb);
    e = hipGetLastError();
    timing_mark(I, 1, s);
    if (e == hipSuccess) {
        const int waves = scan_waves(I->P);
        const size_t lds_b = (size_t)((n + 1) > waves ? (n + 1) : waves) * 256;
        const dim3 grid((unsigned)G), block(64 * waves);
        switch (waves) {
        case 8: bound_scan16_kernel<8><<<grid, block, lds_b, s>>>(I->dt, W, N, out_lb); break;
        case 4: bound_scan16_kernel<4><<<grid, block, lds_b, s>>>(I->dt, W, N, out_lb); break;
        case 2: bound_scan16_kernel<2><<<grid, block, lds_b, s>>>(I->dt, W, N, out_lb); break;
        default: bound_scan16_kernel<1><<<grid, block, lds_b, s>>>(I->dt, W, N, out_lb); break;
        }
        e = hipGetLastError();
    }
    timing_mark(I, 2, s);
    hipError_t e2 = hipFreeAsync(ws, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace fspbb
