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
#include <algorithm>
#include <cstdlib>

#include "bound_common.h"

namespace fspbb {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as16(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

// Workspace of one pool, G = ceil(N / 128) groups.  Nodes are decoded and
// scanned in depth order (order[i] = original index of the i-th node), so the
// lanes of a wave walk prefixes of nearly equal length.
struct Workspace16 {
    uint32_t *dec;    // G x 3 x m x 64 dwords: releases R, closing sums Tk, tails Q
    uint32_t *flg;    // G x NW x 128 dwords: unscheduled-job bits per node
    uint32_t *st;     // G*128: 1 = valid node
    int32_t *order;   // N: node index at each depth-sorted position
    uint32_t *cnt;    // (n + 2) x B: per-block depth counts, then scatter offsets
};

// ---- counting sort of node indices by depth (bucket n+1 holds invalid depths)

__device__ __forceinline__ int depth_bucket(int d, int n) { return (d >= 0 && d <= n) ? d : n + 1; }

__global__ __launch_bounds__(256) void depth_count_kernel(const int32_t *__restrict__ depths, int64_t N, int n,
                                                          int64_t chunk, int B, uint32_t *__restrict__ cnt)
{
    extern __shared__ uint32_t h[];
    for (int b = threadIdx.x; b < n + 2; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(N, lo + chunk);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&h[depth_bucket(depths[i], n)], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < n + 2; b += blockDim.x) cnt[(int64_t)b * B + blockIdx.x] = h[b];
}

// Exclusive prefix sum of cnt[0..total) in place, one block of 1024 threads.
__global__ __launch_bounds__(1024) void depth_scan_kernel(uint32_t *__restrict__ cnt, int64_t total)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (total + 1023) / 1024, lo = t * per, hi = min(total, lo + per);
    uint32_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += cnt[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t c = cnt[i];
        cnt[i] = run;
        run += c;
    }
}

__global__ __launch_bounds__(256) void depth_scatter_kernel(const int32_t *__restrict__ depths, int64_t N, int n,
                                                            int64_t chunk, int B, const uint32_t *__restrict__ cnt,
                                                            int32_t *__restrict__ order)
{
    extern __shared__ uint32_t cur[];
    for (int b = threadIdx.x; b < n + 2; b += blockDim.x) cur[b] = cnt[(int64_t)b * B + blockIdx.x];
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(N, lo + chunk);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint32_t pos = atomicAdd(&cur[depth_bucket(depths[i], n)], 1u);
        order[pos] = (int32_t)i;
    }
}

// ---- decode: one lane per node, nodes taken in depth order
//
// Computes for each node its scheduled set (rejecting out-of-range and
// repeated jobs), the completion times of its prefix on every machine (the
// releases, RM of Table I), the time of the unscheduled jobs on each machine,
// and the tails (QM of Table I: least time left after machine l over the
// unscheduled jobs).  MV = m rounded up to a multiple of 4.  The processing
// times are staged in LDS; the tails are taken two machines at a time with
// packed 16-bit minima over a scalar-loaded table.
template <int MV>
__global__ __launch_bounds__(256) void bound_decode16_kernel(DevTables T, const int32_t *__restrict__ prefixes,
                                                             const int32_t *__restrict__ depths, int64_t N,
                                                             int64_t Npad, Workspace16 W,
                                                             int32_t *__restrict__ out_lb)
{
    extern __shared__ uint32_t sm[];
    uint32_t *bits = sm;                                      // 16 words x 256 lanes
    int32_t *ptab = reinterpret_cast<int32_t *>(sm + kMaskWords * 256);  // (n+1) x MV
    const int n = T.n, m = T.m, NW = (n + 31) >> 5;
    const int tid = threadIdx.x;
    for (int e = tid; e < (n + 1) * MV; e += 256) ptab[e] = T.p32[(e / MV) * kMaxMachines + (e % MV)];
    __syncthreads();

    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    if (i >= Npad) return;
    const bool live = i < N;
    const int64_t node = live ? W.order[i] : 0;
    int d = live ? depths[node] : 0;
    bool ok = live && d >= 0 && d <= n;
    if (!ok) d = 0;

    uint32_t *mybits = bits + tid;
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) mybits[w * 256] = 0u;
    int32_t C[MV], S[MV];
#pragma unroll
    for (int k = 0; k < MV; ++k) { C[k] = 0; S[k] = 0; }
    const int32_t *row = prefixes + node * (int64_t)n;
    for (int t = 0; t < d; t += 4) {
        int32_t jj[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) jj[c] = row[min(t + c, n - 1)];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (t + c < d && ok) {
                const int j = jj[c];
                if ((unsigned)j >= (unsigned)n) { ok = false; continue; }
                const uint32_t bit = 1u << (j & 31);
                const uint32_t old = atomicOr(&mybits[(j >> 5) * 256], bit);
                if (old & bit) { ok = false; continue; }
                const int4 *pr = reinterpret_cast<const int4 *>(ptab + j * MV);
                int32_t prev = 0;
#pragma unroll
                for (int q = 0; q < MV / 4; ++q) {
                    const int4 v = pr[q];
                    const int32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) {
                        const int k = 4 * q + cc;
                        const int32_t ck = max(C[k], prev) + x[cc];
                        C[k] = ck;
                        prev = ck;
                        S[k] += x[cc];
                    }
                }
            }
        }
    }

    u32v<kMaskWords> act;
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) {
        const int lo = w * 32;
        const uint32_t valid = n >= lo + 32 ? 0xffffffffu : (n <= lo ? 0u : ((1u << (n - lo)) - 1u));
        act[w] = ok ? (~mybits[w * 256] & valid) : 0u;
    }
    // tails, two machines per register: q = min over jobs of (Q | inactive mask)
    uint32_t q2[MV / 2];
#pragma unroll
    for (int c = 0; c < MV / 2; ++c) q2[c] = 0xffffffffu;
    for (int j = 0; j < n; ++j) {
        const uint32_t off = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)act[j >> 5], j & 31, 1);
        cptr<uint32_t> qr = as_const(T.tails16 + (size_t)j * (kMaxMachines / 2));
#pragma unroll
        for (int c = 0; c < MV / 2; ++c)
            q2[c] = as32(__builtin_elementwise_min(as16(q2[c]), as16(qr[c] | off)));
    }

    const bool empty = d == n;  // no unscheduled job: every tail is 0
    const int64_t G = i >> 7;
    const int g = (int)(i & 127), lane = g & 63, half = g >> 6;
    uint16_t *d16 = reinterpret_cast<uint16_t *>(W.dec);
    cptr<int32_t> cs = as_const(T.colsum32);
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        if (k < m) {
            const uint32_t qk = (q2[k >> 1] >> (16 * (k & 1))) & 0xffffu;
            d16[((G * 3 + 0) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? C[k] : 0);
            d16[((G * 3 + 1) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? C[k] + (cs[k] - S[k]) : 0);
            d16[((G * 3 + 2) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok && !empty ? qk : 0u);
        }
    }
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w)
        if (w < NW) W.flg[(G * NW + w) * 128 + g] = act[w];
    W.st[i] = ok ? 1u : 0u;
    if (live && !ok) {
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

// Mask rows of UNR slots through the LDS "add thread id" read: for each slot
// M0 = row offset, and every lane reads the dword at M0 + 4 * lane, so no
// vector instruction is spent on addresses.  M0 is saved and restored; the
// block waits for its own reads (scalar loads are then complete as well).
// A write of M0 by a scalar instruction needs one wait state before the read.
// The scalar adds write SCC, which the block declares clobbered.
template <int UNR>
__device__ __forceinline__ void gather_rows_addtid(uint32_t (&x)[UNR], const uint32_t (&joff)[UNR], uint32_t base);

#define FSP_ADDTID_1(i) "s_add_u32 m0, %[j" #i "], %[base]\n\ts_nop 0\n\tds_read_addtid_b32 %[x" #i "]\n\t"

template <>
__device__ __forceinline__ void gather_rows_addtid<8>(uint32_t (&x)[8], const uint32_t (&joff)[8], uint32_t base)
{
    uint32_t save;
    asm volatile("s_mov_b32 %[sv], m0\n\t"
                 FSP_ADDTID_1(0) FSP_ADDTID_1(1) FSP_ADDTID_1(2) FSP_ADDTID_1(3)
                 FSP_ADDTID_1(4) FSP_ADDTID_1(5) FSP_ADDTID_1(6) FSP_ADDTID_1(7)
                 "s_waitcnt lgkmcnt(0)\n\t"
                 "s_mov_b32 m0, %[sv]"
                 : [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [x3] "=&v"(x[3]),
                   [x4] "=&v"(x[4]), [x5] "=&v"(x[5]), [x6] "=&v"(x[6]), [x7] "=&v"(x[7]), [sv] "=&s"(save)
                 : [j0] "s"(joff[0]), [j1] "s"(joff[1]), [j2] "s"(joff[2]), [j3] "s"(joff[3]),
                   [j4] "s"(joff[4]), [j5] "s"(joff[5]), [j6] "s"(joff[6]), [j7] "s"(joff[7]),
                   [base] "s"(base)
                 : "scc");
}

template <>
__device__ __forceinline__ void gather_rows_addtid<4>(uint32_t (&x)[4], const uint32_t (&joff)[4], uint32_t base)
{
    uint32_t save;
    asm volatile("s_mov_b32 %[sv], m0\n\t"
                 FSP_ADDTID_1(0) FSP_ADDTID_1(1) FSP_ADDTID_1(2) FSP_ADDTID_1(3)
                 "s_waitcnt lgkmcnt(0)\n\t"
                 "s_mov_b32 m0, %[sv]"
                 : [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [x3] "=&v"(x[3]), [sv] "=&s"(save)
                 : [j0] "s"(joff[0]), [j1] "s"(joff[1]), [j2] "s"(joff[2]), [j3] "s"(joff[3]),
                   [base] "s"(base)
                 : "scc");
}

template <>
__device__ __forceinline__ void gather_rows_addtid<16>(uint32_t (&x)[16], const uint32_t (&joff)[16], uint32_t base)
{
    uint32_t save;
    asm volatile("s_mov_b32 %[sv], m0\n\t"
                 FSP_ADDTID_1(0) FSP_ADDTID_1(1) FSP_ADDTID_1(2) FSP_ADDTID_1(3)
                 FSP_ADDTID_1(4) FSP_ADDTID_1(5) FSP_ADDTID_1(6) FSP_ADDTID_1(7)
                 FSP_ADDTID_1(8) FSP_ADDTID_1(9) FSP_ADDTID_1(10) FSP_ADDTID_1(11)
                 FSP_ADDTID_1(12) FSP_ADDTID_1(13) FSP_ADDTID_1(14) FSP_ADDTID_1(15)
                 "s_waitcnt lgkmcnt(0)\n\t"
                 "s_mov_b32 m0, %[sv]"
                 : [x0] "=&v"(x[0]), [x1] "=&v"(x[1]), [x2] "=&v"(x[2]), [x3] "=&v"(x[3]),
                   [x4] "=&v"(x[4]), [x5] "=&v"(x[5]), [x6] "=&v"(x[6]), [x7] "=&v"(x[7]),
                   [x8] "=&v"(x[8]), [x9] "=&v"(x[9]), [x10] "=&v"(x[10]), [x11] "=&v"(x[11]),
                   [x12] "=&v"(x[12]), [x13] "=&v"(x[13]), [x14] "=&v"(x[14]), [x15] "=&v"(x[15]),
                   [sv] "=&s"(save)
                 : [j0] "s"(joff[0]), [j1] "s"(joff[1]), [j2] "s"(joff[2]), [j3] "s"(joff[3]),
                   [j4] "s"(joff[4]), [j5] "s"(joff[5]), [j6] "s"(joff[6]), [j7] "s"(joff[7]),
                   [j8] "s"(joff[8]), [j9] "s"(joff[9]), [j10] "s"(joff[10]), [j11] "s"(joff[11]),
                   [j12] "s"(joff[12]), [j13] "s"(joff[13]), [j14] "s"(joff[14]), [j15] "s"(joff[15]),
                   [base] "s"(base)
                 : "scc");
}

template <>
__device__ __forceinline__ void gather_rows_addtid<32>(uint32_t (&x)[32], const uint32_t (&joff)[32], uint32_t base)
{
    uint32_t lo[16], hi[16], jl[16], jh[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) { jl[c] = joff[c]; jh[c] = joff[16 + c]; }
    gather_rows_addtid<16>(lo, jl, base);
    gather_rows_addtid<16>(hi, jh, base);
#pragma unroll
    for (int c = 0; c < 16; ++c) { x[c] = lo[c]; x[16 + c] = hi[c]; }
}
#undef FSP_ADDTID_1

__device__ __forceinline__ void scan_update(u16x2 &s, uint32_t msk, uint32_t ce)
{
    const unsigned short e = (unsigned short)(ce >> 16), c = (unsigned short)ce;
    const u16x2 E = {e, e};
    const u16x2 C = {c, c};
    const u16x2 t = __builtin_elementwise_max(s, E) + C;
    s = as16((msk & as32(t)) | (~msk & as32(s)));
}

// Scans NCH machine pairs in lockstep over their Johnson-order slots.  The
// chains are independent, so their dependent packed operations interleave.
template <int UNR, int NCH, bool ADDTID>
__device__ __forceinline__ void scan_pairs(const DevTables &T, const int (&prs)[NCH], u16x2 (&s)[NCH],
                                           const unsigned char *lds_lane, uint32_t lds_base)
{
    const int npad = T.npad;  // multiple of 4; padding slots read the zero row
    cptr<uint32_t> rec[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
        rec[ch] = as_const(reinterpret_cast<const uint32_t *>(T.rec16 + (size_t)prs[ch] * npad));
    int i = 0;
    for (; i + UNR <= npad; i += UNR) {
        uint32_t r[NCH][2 * UNR];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int c = 0; c < 2 * UNR; ++c) r[ch][c] = rec[ch][2 * i + c];
        if constexpr (ADDTID) {
            uint32_t jo[NCH * UNR], x[NCH * UNR];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int c = 0; c < UNR; ++c) jo[ch * UNR + c] = r[ch][2 * c];
            gather_rows_addtid<NCH * UNR>(x, jo, lds_base);
#pragma unroll
            for (int c = 0; c < UNR; ++c)
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) scan_update(s[ch], x[ch * UNR + c], r[ch][2 * c + 1]);
        } else {
#pragma unroll
            for (int c = 0; c < UNR; ++c)
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) scan_step(s[ch], lds_lane, r[ch][2 * c], r[ch][2 * c + 1]);
        }
    }
    for (; i < npad; i += 4) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            uint32_t r[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) r[c] = rec[ch][2 * i + c];
#pragma unroll
            for (int c = 0; c < 8; c += 2) scan_step(s[ch], lds_lane, r[c], r[c + 1]);
        }
    }
}

template <int WAVES, int UNR, bool ADDTID, int NCH>
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
    // LDS byte address of the mask rows (M0-relative reads add it to each row offset)
    const uint32_t lds_base = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t *)lds);
    const uint32_t *dR = W.dec + (G * 3 + 0) * m * 64 + lane;
    const uint32_t *dT = dR + m * 64;
    const uint32_t *dQ = dT + m * 64;
    cptr<int32_t> pairs = as_const(T.pairs);
    u16x2 lb = {0, 0};
    int pr = wave;
    for (; pr + (NCH - 1) * WAVES < T.P; pr += NCH * WAVES) {
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
    for (; pr < T.P; pr += WAVES) {  // fewer than NCH pairs left for this wave
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
        if (a < N && W.st[a]) out_lb[W.order[a]] = (int32_t)best.x;
        if (b < N && W.st[b]) out_lb[W.order[b]] = (int32_t)best.y;
    }
}

static int scan_waves(int P)
{
    if (const char *e = getenv("FSPBB_SCAN_WAVES")) {
        const int w = atoi(e);
        if (w == 1 || w == 2 || w == 4 || w == 8 || w == 16) return w;
    }
    if (P >= 128) return 16;
    if (P >= 64) return 8;
    if (P >= 16) return 4;
    if (P >= 4) return 2;
    return 1;
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
                          const Workspace16 &W, int64_t N, int32_t *out_lb)
{
    const dim3 block(64 * WAVES);
    const int nch = scan_chains();
    if (unr == 16 && nch == 2)
        bound_scan16_kernel<WAVES, 16, ADDTID, 2><<<grid, block, lds_b, s>>>(dt, W, N, out_lb);
    else if (unr == 16)
        bound_scan16_kernel<WAVES, 16, ADDTID, 1><<<grid, block, lds_b, s>>>(dt, W, N, out_lb);
    else if (nch == 2)
        bound_scan16_kernel<WAVES, 8, ADDTID, 2><<<grid, block, lds_b, s>>>(dt, W, N, out_lb);
    else
        bound_scan16_kernel<WAVES, 8, ADDTID, 1><<<grid, block, lds_b, s>>>(dt, W, N, out_lb);
}

template <int WAVES>
static void launch_scan(int unr, dim3 grid, size_t lds_b, hipStream_t s, const DevTables &dt, const Workspace16 &W,
                        int64_t N, int32_t *out_lb)
{
    if (scan_addtid())
        launch_scan_u<WAVES, true>(unr, grid, lds_b, s, dt, W, N, out_lb);
    else
        launch_scan_u<WAVES, false>(unr, grid, lds_b, s, dt, W, N, out_lb);
}

hipError_t launch_bound_packed(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths,
                               int64_t N, int32_t *out_lb, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    const int n = I->n, m = I->m, NW = (n + 31) >> 5;
    const int64_t G = (N + kGroup - 1) / kGroup, Npad = G * kGroup;
    const int B = (int)std::min<int64_t>(1024, (N + 4095) / 4096);
    const int64_t chunk = (N + B - 1) / B;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t dec_b = al((size_t)G * 3 * m * 64 * 4), flg_b = al((size_t)G * NW * 128 * 4),
                 st_b = al((size_t)Npad * 4), ord_b = al((size_t)N * 4), cnt_b = al((size_t)(n + 2) * B * 4);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, dec_b + flg_b + st_b + ord_b + cnt_b, s);
    if (e != hipSuccess) return e;
    char *w = (char *)ws;
    Workspace16 W;
    W.dec = (uint32_t *)w;
    W.flg = (uint32_t *)(w + dec_b);
    W.st = (uint32_t *)(w + dec_b + flg_b);
    W.order = (int32_t *)(w + dec_b + flg_b + st_b);
    W.cnt = (uint32_t *)(w + dec_b + flg_b + st_b + ord_b);

    timing_mark(I, 0, s);
    const size_t hb = (size_t)(n + 2) * 4;
    depth_count_kernel<<<B, 256, hb, s>>>(depths, N, n, chunk, B, W.cnt);
    depth_scan_kernel<<<1, 1024, 0, s>>>(W.cnt, (int64_t)(n + 2) * B);
    depth_scatter_kernel<<<B, 256, hb, s>>>(depths, N, n, chunk, B, W.cnt, W.order);

    const dim3 dgrid((unsigned)((Npad + 255) / 256)), dblock(256);
    const int MV = (m + 3) & ~3;
    const size_t dlds = (size_t)kMaskWords * 256 * 4 + (size_t)(n + 1) * MV * 4;
#define FSP_DECODE(MVV) \
    case MVV: bound_decode16_kernel<MVV><<<dgrid, dblock, dlds, s>>>(I->dt, prefixes, depths, N, Npad, W, out_lb); break;
    switch (MV) {
        FSP_DECODE(4) FSP_DECODE(8) FSP_DECODE(12) FSP_DECODE(16)
        FSP_DECODE(20) FSP_DECODE(24) FSP_DECODE(28) FSP_DECODE(32)
    }
#undef FSP_DECODE
    e = hipGetLastError();
    timing_mark(I, 1, s);
    if (e == hipSuccess) {
        const int waves = scan_waves(I->P);
        const size_t lds_b = (size_t)((n + 1) > waves ? (n + 1) : waves) * 256;
        const dim3 grid((unsigned)G);
        const int unr = scan_unroll();
        switch (waves) {
        case 16: launch_scan<16>(unr, grid, lds_b, s, I->dt, W, N, out_lb); break;
        case 8: launch_scan<8>(unr, grid, lds_b, s, I->dt, W, N, out_lb); break;
        case 4: launch_scan<4>(unr, grid, lds_b, s, I->dt, W, N, out_lb); break;
        case 2: launch_scan<2>(unr, grid, lds_b, s, I->dt, W, N, out_lb); break;
        default: launch_scan<1>(unr, grid, lds_b, s, I->dt, W, N, out_lb); break;
        }
        e = hipGetLastError();
    }
    timing_mark(I, 2, s);
    hipError_t e2 = hipFreeAsync(ws, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace fspbb
