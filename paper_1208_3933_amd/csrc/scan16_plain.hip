// The plain 16-bit pair-scan kernel and its launch (the launch of
// fsp_bound_pool after the decode, and of steps whose children are decoded
// from their parents).
//
// One workgroup per group of 128 nodes.  Lane L of every wave holds nodes L
// and L+64 of the group as the two 16-bit halves of each register, so one
// packed instruction advances two nodes.  The group's unscheduled masks live
// in LDS as one dword per (job, lane) (0xffff per unscheduled half), shared by
// all waves; the waves split the machine pairs between them and combine their
// maxima through LDS at the end.  The Johnson-with-lags order of a pair is the
// same for every node, so the per-slot records (mask-row offset, lag + a,
// b - a) are wave-uniform scalar loads; only the mask is per lane.
#include <algorithm>
#include <cstdlib>

#include "batch.h"
#include "scan16.h"

namespace fspbb {

// Grid (groups, splits): workgroup (G, y) scans pairs [y * pps, (y+1) * pps)
// of group G.  With one split it writes each bound; with several, each split
// takes its partial maximum into out_lb with an atomic max (out_lb holds 0
// for every valid node beforehand, written by the decode).  With Ndev the
// node count is read from the device (a grid sized for a bound on it; groups
// past it leave at once).
template <int WAVES, int UNR, bool ADDTID, int NCH>
__global__ __launch_bounds__(64 * WAVES) void bound_scan16_kernel(DevTables T, Workspace16 W, int64_t N,
                                                                  int32_t *__restrict__ out_lb, int pps,
                                                                  const int64_t *__restrict__ Ndev)
{
    extern __shared__ uint32_t lds[];  // (n + 1) rows x 64 lanes; row n stays zero
    const int n = T.n, m = T.m, NW = (n + 31) >> 5;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int64_t G = blockIdx.x;
    if (Ndev) {
        N = *Ndev;
        if (G * kGroup >= N) return;  // the whole workgroup
    }

    // the mask rows from the unscheduled bits: each lane reads its two nodes'
    // bit words once per 32 jobs (all loads first), then expands them
    for (int w = wave; w < NW; w += WAVES) {
        const uint32_t *fw = W.flg + (G * NW + w) * 128;
        const uint32_t a = fw[lane], b = fw[64 + lane];
        const int jn = min(32, n - 32 * w);
        for (int t = 0; t < jn; ++t) {
            const uint32_t m2 = (((a >> t) & 1u) ? 0x0000ffffu : 0u) | (((b >> t) & 1u) ? 0xffff0000u : 0u);
            lds[(32 * w + t) * 64 + lane] = m2;
        }
    }
    if (wave == WAVES - 1) lds[n * 64 + lane] = 0u;  // the zero row of padding slots
    __syncthreads();

    const unsigned char *lds_lane = reinterpret_cast<const unsigned char *>(lds) + lane * 4;
    // LDS byte address of the mask rows (M0-relative reads add it to each row offset)
    const uint32_t lds_base = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t *)lds);
    const uint32_t *dR = W.dec + (G * 3 + 0) * m * 64 + lane;
    const uint32_t *dT = dR + m * 64;
    const uint32_t *dQ = dT + m * 64;
    cptr<int32_t> pairs = as_const(T.pairs);
    u16x2 lb = {0, 0};
    const int p0 = (int)blockIdx.y * pps, p1 = min(T.P, p0 + pps);
    int pr = p0 + wave;
    for (; pr + (NCH - 1) * WAVES < p1; pr += NCH * WAVES) {
        int prs[NCH];
        u16x2 s[NCH];
        uint32_t tk[NCH], ql[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            prs[ch] = pr + ch * WAVES;
            const int k = pairs[2 * prs[ch]], l = pairs[2 * prs[ch] + 1];
            s[ch] = as16(dR[l * 64]) - as16(dR[k * 64]);
            tk[ch] = dT[k * 64];
            ql[ch] = dQ[l * 64];
        }
        scan_pairs<UNR, NCH, ADDTID>(T, prs, s, lds_lane, lds_base);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) lb = __builtin_elementwise_max(lb, as16(tk[ch]) + s[ch] + as16(ql[ch]));
    }
    for (; pr < p1; pr += WAVES) {  // fewer than NCH pairs left for this wave
        const int prs[1] = {pr};
        const int k = pairs[2 * pr], l = pairs[2 * pr + 1];
        u16x2 s[1] = {as16(dR[l * 64]) - as16(dR[k * 64])};
        const uint32_t tk = dT[k * 64], ql = dQ[l * 64];
        scan_pairs<UNR, 1, ADDTID>(T, prs, s, lds_lane, lds_base);
        lb = __builtin_elementwise_max(lb, as16(tk) + s[0] + as16(ql));
    }
    __syncthreads();
    lds[wave * 64 + lane] = as32(lb);
    __syncthreads();
    if (wave == 0) {
        u16x2 best = as16(lds[lane]);
#pragma unroll
        for (int w = 1; w < WAVES; ++w) best = __builtin_elementwise_max(best, as16(lds[w * 64 + lane]));
        const int64_t a = G * 128 + lane, b = a + 64;
        if (gridDim.y == 1) {
            if (a < N && W.st[a]) out_lb[W.order ? W.order[a] : a] = (int32_t)best.x;
            if (b < N && W.st[b]) out_lb[W.order ? W.order[b] : b] = (int32_t)best.y;
        } else {
            if (a < N && W.st[a]) atomicMax(&out_lb[W.order ? W.order[a] : a], (int32_t)best.x);
            if (b < N && W.st[b]) atomicMax(&out_lb[W.order ? W.order[b] : b], (int32_t)best.y);
        }
    }
}

static int scan_waves(const fsp_instance_s *I)
{
    if (const char *e = getenv("FSPBB_SCAN_WAVES")) {
        const int w = atoi(e);
        if (w == 1 || w == 2 || w == 4 || w == 8 || w == 16) return w;
    }
    return scan_tuning_for(I).waves_per_group;
}

static int scan_unroll()
{
    if (const char *e = getenv("FSPBB_SCAN_UNROLL")) {
        const int u = atoi(e);
        if (u == 8 || u == 16) return u;
    }
    return 8;
}

static int scan_chains()
{
    if (const char *e = getenv("FSPBB_SCAN_CHAINS")) {
        const int c = atoi(e);
        if (c == 1 || c == 2) return c;
    }
    return 2;
}

static bool scan_addtid()
{
    if (const char *e = getenv("FSPBB_SCAN_ADDTID")) return atoi(e) != 0;
    return true;
}

template <int WAVES, bool ADDTID>
static void launch_scan_u(int unr, dim3 grid, size_t lds_b, hipStream_t s, const DevTables &dt,
                          const Workspace16 &W, int64_t N, int32_t *out_lb, int pps, const int64_t *Ndev)
{
    const dim3 block(64 * WAVES);
    const int nch = scan_chains();
    if (unr == 16 && nch == 2)
        bound_scan16_kernel<WAVES, 16, ADDTID, 2><<<grid, block, lds_b, s>>>(dt, W, N, out_lb, pps, Ndev);
    else if (unr == 16)
        bound_scan16_kernel<WAVES, 16, ADDTID, 1><<<grid, block, lds_b, s>>>(dt, W, N, out_lb, pps, Ndev);
    else if (nch == 2)
        bound_scan16_kernel<WAVES, 8, ADDTID, 2><<<grid, block, lds_b, s>>>(dt, W, N, out_lb, pps, Ndev);
    else
        bound_scan16_kernel<WAVES, 8, ADDTID, 1><<<grid, block, lds_b, s>>>(dt, W, N, out_lb, pps, Ndev);
}

template <int WAVES>
static void launch_scan(int unr, dim3 grid, size_t lds_b, hipStream_t s, const DevTables &dt, const Workspace16 &W,
                        int64_t N, int32_t *out_lb, int pps, const int64_t *Ndev)
{
    if (scan_addtid())
        launch_scan_u<WAVES, true>(unr, grid, lds_b, s, dt, W, N, out_lb, pps, Ndev);
    else
        launch_scan_u<WAVES, false>(unr, grid, lds_b, s, dt, W, N, out_lb, pps, Ndev);
}

hipError_t launch_scan16(const fsp_instance_s *I, const Workspace16 &W, int64_t N, int32_t *out_lb, hipStream_t s,
                         int splits, const int64_t *Ndev)
{
    if (N <= 0) return hipSuccess;
    const int n = I->n, P = I->P;
    if (splits < 1) splits = 1;
    if (splits > P) splits = P;
    const int pps = (P + splits - 1) / splits;
    splits = (P + pps - 1) / pps;
    // one group per workgroup: the tuned waves; a split: about one pair per
    // wave of its share (small pools are latency-bound), at most 16 waves
    int waves = scan_waves(I);
    if (splits > 1) {
        int ppw = 1;
        if (const char *e = getenv("FSPBB_SPLIT_PAIRS_PER_WAVE")) ppw = std::max(1, atoi(e));
        int w = 1;
        while (w < 16 && ppw * w < pps) w *= 2;
        waves = w;
    }
    const size_t lds_b = (size_t)((n + 1) > waves ? (n + 1) : waves) * 256;
    const dim3 grid((unsigned)((N + kGroup - 1) / kGroup), (unsigned)splits);
    const int unr = scan_unroll();
    switch (waves) {
    case 16: launch_scan<16>(unr, grid, lds_b, s, I->dt, W, N, out_lb, pps, Ndev); break;
    case 8: launch_scan<8>(unr, grid, lds_b, s, I->dt, W, N, out_lb, pps, Ndev); break;
    case 4: launch_scan<4>(unr, grid, lds_b, s, I->dt, W, N, out_lb, pps, Ndev); break;
    case 2: launch_scan<2>(unr, grid, lds_b, s, I->dt, W, N, out_lb, pps, Ndev); break;
    default: launch_scan<1>(unr, grid, lds_b, s, I->dt, W, N, out_lb, pps, Ndev); break;
    }
    return hipGetLastError();
}

}  // namespace fspbb
