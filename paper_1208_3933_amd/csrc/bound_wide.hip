// 32-bit bound path with the 16-bit path's structure, for instances whose
// values reach 16 bits ((n+m-1) * max p >= 65536, e.g. processing times of a
// few hundred at 200 x 20).
//
// Three steps per pool:
//   depth sort  node indices by depth (the 16-bit path's counting sort), so a
//               decode wave's prefix loops have equal length;
//   decode      one lane per node: scheduled set, releases (RM of Table I),
//               closing sums and tails (QM), written to a workspace in the
//               layout the scan reads with unit stride (the 16-bit decode's
//               structure with 32-bit values);
//   scan        one workgroup per group of 64 nodes, one node per lane.  The
//               group's unscheduled masks sit in LDS as one dword per (job,
//               lane), all ones for an unscheduled job; the Johnson-with-lags
//               records of a pair are wave-uniform scalar loads; each slot is
//               one max, one add and one bitwise select (Fig. 2's update in
//               gap form, s <- max(s, lag + a) + (b - a)).  The waves split
//               the machine pairs and combine their maxima through LDS.
#include <algorithm>

#include "batch.h"
#include "bound_wide.h"
#include "lds_stage.h"
#include "scan16.h"

namespace fspbb {

// ---- decode: one lane per node, depth order; block `blockIdx.x` of 256 nodes
//
// The structure of the 16-bit decode with 32-bit values: the processing
// times are staged in LDS (int32 rows of MV machines, row n zero), the prefix
// loop is branch-free (a slot past the depth or an out-of-range job takes the
// zero row, which leaves the completion times unchanged) with two 16-byte row
// loads in flight, the scheduled bits are set by LDS ORs that return nothing
// and repeats are found at the end by a popcount.  Tails are packed 16-bit
// minima when every tail fits 16 bits, else 32-bit minima.
inline size_t decodew_lds_words(int n, int MV) { return (size_t)((n + 31) >> 5) * 256 + (size_t)(n + 1) * MV; }

template <int MV>
__global__ __launch_bounds__(256) void bound_decodew_kernel(DevTables T, const int32_t *__restrict__ prefixes,
                                                            const int32_t *__restrict__ depths, int64_t N,
                                                            int64_t Npad, WorkspaceW W,
                                                            int32_t *__restrict__ out_lb)
{
    extern __shared__ uint32_t sm[];
    const int n = T.n, m = T.m, NW = (n + 31) >> 5;
    uint32_t *bits = sm;                                         // NW words x 256 lanes
    int32_t *pl = reinterpret_cast<int32_t *>(sm + NW * 256);   // (n + 1) x MV; row n is zero
    const int tid = threadIdx.x;
    stage_lds<16>(pl, (n + 1) * MV, [&](int e) {  // row n of p32 is zero
        const int j = e / MV, k = e - j * MV;
        return T.p32[(size_t)j * kMaxMachines + k];
    });
    __syncthreads();

    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    if (i >= Npad) return;
    const bool live = i < N;
    const int64_t node = live ? (W.order ? W.order[i] : i) : 0;
    int d = live ? depths[node] : 0;
    bool ok = live && d >= 0 && d <= n;
    if (!ok) d = 0;

    uint32_t *mybits = bits + tid;
    for (int w = 0; w < NW; ++w) mybits[w * 256] = 0u;
    int32_t C[MV], S[MV];
#pragma unroll
    for (int k = 0; k < MV; ++k) { C[k] = 0; S[k] = 0; }
    auto step4 = [&](int32_t j0, int32_t j1, int32_t j2, int32_t j3, int t) {
        const int32_t jj[4] = {j0, j1, j2, j3};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bool in = t + c < d, good = (unsigned)jj[c] < (unsigned)n;
            ok = ok && (good || !in);
            const int j = in && good ? jj[c] : n;
            const bool real = j < n;
            atomicOr(&mybits[(real ? j >> 5 : 0) * 256], real ? 1u << (j & 31) : 0u);
            const int4 *pr = reinterpret_cast<const int4 *>(pl + j * MV);
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
    };
    const int32_t *row = prefixes + node * (int64_t)n;
    if ((n & 3) == 0 && ((uintptr_t)prefixes & 15) == 0) {
        const int4 *r4 = reinterpret_cast<const int4 *>(row);
        const int last = (n >> 2) - 1;
        int4 a = r4[0];
        for (int t = 0; t < d; t += 8) {
            const int4 b = r4[min((t >> 2) + 1, last)];
            step4(a.x, a.y, a.z, a.w, t);
            a = r4[min((t >> 2) + 2, last)];
            step4(b.x, b.y, b.z, b.w, t + 4);
        }
    } else {
        for (int t = 0; t < d; t += 4)
            step4(row[min(t, n - 1)], row[min(t + 1, n - 1)], row[min(t + 2, n - 1)], row[min(t + 3, n - 1)], t);
    }

    u32v<kMaskWords> act;
    int nset = 0;
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) {
        const int lo = w * 32;
        const uint32_t valid = n >= lo + 32 ? 0xffffffffu : (n <= lo ? 0u : ((1u << (n - lo)) - 1u));
        const uint32_t b = w < NW ? mybits[w * 256] : 0u;
        nset += __popc(b);
        act[w] = ~b & valid;
    }
    ok = ok && nset == d;
    if (!ok) {
#pragma unroll
        for (int w = 0; w < kMaskWords; ++w) act[w] = 0u;
    }
    // heads: each machine's release becomes the earliest start on it of an
    // unscheduled job scheduled next (uniform job loop: LDS broadcasts)
    if (T.heads && ok && d < n) {
        int32_t h[MV];
#pragma unroll
        for (int k = 0; k < MV; ++k) h[k] = 0x7fffffff;
        for (int j = 0; j < n; ++j) {
            const bool a = (act[j >> 5] >> (j & 31)) & 1u;
            const int4 *pr = reinterpret_cast<const int4 *>(pl + j * MV);
            int32_t prev = 0;
#pragma unroll
            for (int q = 0; q < MV / 4; ++q) {
                const int4 v = pr[q];
                const int32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const int k = 4 * q + cc;
                    const int32_t start = max(C[k], prev);
                    h[k] = a ? min(h[k], start) : h[k];
                    prev = start + x[cc];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < MV; ++k) C[k] = h[k];
    }
    // tails: the least over unscheduled jobs of the time after machine l
    uint32_t qv[MV];
    if (T.tails16ok) {
        constexpr int H = MV / 2;
        uint32_t q2[H];
#pragma unroll
        for (int c = 0; c < H; ++c) q2[c] = 0xffffffffu;
        for (int w = 0; w < NW; ++w) {
            const uint32_t aw = act[w];
            const int jn = min(32, n - 32 * w);
            cptr<uint32_t> qw = as_const(T.tails16 + (size_t)(32 * w) * (kMaxMachines / 2));
            for (int b = 0; b < jn; ++b) {
                const uint32_t off = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)aw, b, 1);
                cptr<uint32_t> qr = qw + (size_t)b * (kMaxMachines / 2);
#pragma unroll
                for (int c = 0; c < H; ++c)
                    q2[c] = as32(__builtin_elementwise_min(as16(q2[c]), as16(qr[c] | off)));
            }
        }
#pragma unroll
        for (int k = 0; k < MV; ++k) qv[k] = (q2[k >> 1] >> (16 * (k & 1))) & 0xffffu;
    } else {
#pragma unroll
        for (int k = 0; k < MV; ++k) qv[k] = 0xffffffffu;
        for (int w = 0; w < NW; ++w) {
            const uint32_t aw = act[w];
            const int jn = min(32, n - 32 * w);
            cptr<uint32_t> qw = as_const(reinterpret_cast<const uint32_t *>(T.tails32) + (size_t)(32 * w) * kMaxMachines);
            for (int b = 0; b < jn; ++b) {
                const uint32_t off = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)aw, b, 1);
                cptr<uint32_t> qr = qw + (size_t)b * kMaxMachines;
#pragma unroll
                for (int k = 0; k < MV; ++k) qv[k] = min(qv[k], qr[k] | off);
            }
        }
    }

    const bool empty = d == n;  // no unscheduled job: every tail is 0
    const int64_t G = i >> 6;
    const int lane = (int)(i & 63);
    cptr<int32_t> cs = as_const(T.colsum32);
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        if (k < m) {
            W.dec[((G * 3 + 0) * m + k) * 64 + lane] = ok ? C[k] : 0;
            W.dec[((G * 3 + 1) * m + k) * 64 + lane] = ok ? C[k] + (cs[k] - S[k]) : 0;
            W.dec[((G * 3 + 2) * m + k) * 64 + lane] = ok && !empty ? (int32_t)qv[k] : 0;
        }
    }
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w)
        if (w < NW) W.flg[(G * NW + w) * 64 + lane] = act[w];
    W.st[i] = ok ? 1u : 0u;
    if (live && !ok) {
        out_lb[node] = FSP_LB_INVALID;
        atomicAdd(T.bad, 1ull);
    }
}

// NCH pair chains over their Johnson-order slots in lockstep; UNR slots per
// chain per batch of LDS row reads (M0-relative, no address arithmetic).
template <int UNR, int NCH>
__device__ __forceinline__ void scanw_pairs(const DevTables &T, const int (&prs)[NCH], int32_t (&s)[NCH],
                                            uint32_t lds_base)
{
    const int npad = T.npad;  // multiple of 4; padding slots read the zero row
    cptr<uint32_t> rec[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
        rec[ch] = as_const(reinterpret_cast<const uint32_t *>(T.recw + (size_t)prs[ch] * npad));
    int i = 0;
    for (; i + UNR <= npad; i += UNR) {
        uint32_t r[NCH][3 * UNR];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int c = 0; c < 3 * UNR; ++c) r[ch][c] = rec[ch][3 * i + c];
        uint32_t jo[NCH * UNR], x[NCH * UNR];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int c = 0; c < UNR; ++c) jo[ch * UNR + c] = r[ch][3 * c];
        gather_rows_addtid<NCH * UNR>(x, jo, lds_base);
#pragma unroll
        for (int c = 0; c < UNR; ++c)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int32_t t = max(s[ch], (int32_t)r[ch][3 * c + 1]) + (int32_t)r[ch][3 * c + 2];
                s[ch] = (int32_t)((x[ch * UNR + c] & (uint32_t)t) | (~x[ch * UNR + c] & (uint32_t)s[ch]));
            }
    }
    for (; i < npad; i += 4) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            uint32_t r[12], jo[4], x[4];
#pragma unroll
            for (int c = 0; c < 12; ++c) r[c] = rec[ch][3 * i + c];
#pragma unroll
            for (int c = 0; c < 4; ++c) jo[c] = r[3 * c];
            gather_rows_addtid<4>(x, jo, lds_base);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int32_t t = max(s[ch], (int32_t)r[3 * c + 1]) + (int32_t)r[3 * c + 2];
                s[ch] = (int32_t)((x[c] & (uint32_t)t) | (~x[c] & (uint32_t)s[ch]));
            }
        }
    }
}

template <int WAVES, int UNR, int NCH>
__global__ __launch_bounds__(64 * WAVES) void bound_scanw_kernel(DevTables T, WorkspaceW W, int64_t N,
                                                                 int32_t *__restrict__ out_lb)
{
    extern __shared__ uint32_t lds[];  // (n + 1) rows x 64 lanes; row n stays zero
    const int n = T.n, m = T.m, NW = (n + 31) >> 5;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t G = blockIdx.x;

    // mask rows from the unscheduled bits: one word load per 32 jobs
    for (int w = wave; w < NW; w += WAVES) {
        const uint32_t a = W.flg[(G * NW + w) * 64 + lane];
        const int jn = min(32, n - 32 * w);
        for (int t = 0; t < jn; ++t) lds[(32 * w + t) * 64 + lane] = 0u - ((a >> t) & 1u);
    }
    if (wave == WAVES - 1) lds[n * 64 + lane] = 0u;  // the zero row of padding slots
    __syncthreads();

    const uint32_t lds_base = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t *)lds);
    const int32_t *dR = W.dec + (G * 3 + 0) * m * 64 + lane;
    const int32_t *dT = dR + m * 64;
    const int32_t *dQ = dT + m * 64;
    cptr<int32_t> pairs = as_const(T.pairs);
    int32_t lb = 0;
    int pr = wave;
    for (; pr + (NCH - 1) * WAVES < T.P; pr += NCH * WAVES) {
        int prs[NCH];
        int32_t s[NCH], tk[NCH], ql[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            prs[ch] = pr + ch * WAVES;
            const int k = pairs[2 * prs[ch]], l = pairs[2 * prs[ch] + 1];
            s[ch] = dR[l * 64] - dR[k * 64];
            tk[ch] = dT[k * 64];
            ql[ch] = dQ[l * 64];
        }
        scanw_pairs<UNR, NCH>(T, prs, s, lds_base);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) lb = max(lb, tk[ch] + s[ch] + ql[ch]);
    }
    for (; pr < T.P; pr += WAVES) {  // fewer than NCH pairs left for this wave
        const int prs[1] = {pr};
        const int k = pairs[2 * pr], l = pairs[2 * pr + 1];
        int32_t s[1] = {dR[l * 64] - dR[k * 64]};
        const int32_t tk = dT[k * 64], ql = dQ[l * 64];
        scanw_pairs<UNR, 1>(T, prs, s, lds_base);
        lb = max(lb, tk + s[0] + ql);
    }
    __syncthreads();
    lds[wave * 64 + lane] = (uint32_t)lb;
    __syncthreads();
    if (wave == 0) {
        int32_t best = (int32_t)lds[lane];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) best = max(best, (int32_t)lds[w * 64 + lane]);
        const int64_t a = G * 64 + lane;
        if (a < N && W.st[a]) out_lb[W.order ? W.order[a] : a] = best;
    }
}

namespace {

struct WideLayout {
    size_t dec, flg, st, ord, cnt;
    size_t total() const { return dec + flg + st + ord + cnt; }
};

WideLayout wide_layout(const fsp_instance_s *I, int64_t N)
{
    const int n = I->n, m = I->m, NW = (n + 31) >> 5;
    const int64_t G = (N + kGroupW - 1) / kGroupW, Npad = G * kGroupW;
    const int B = (int)std::min<int64_t>(kSortMaxBlocks, (N + 4095) / 4096);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return WideLayout{al((size_t)G * 3 * m * 64 * 4), al((size_t)G * NW * 64 * 4), al((size_t)Npad * 4),
                      al((size_t)N * 4), al((size_t)(n + 2) * B * 4)};
}

// Waves per 64-node group: about four pairs per wave and chain (the 16-bit
// path's rule), at most 16.
int wide_waves(int P)
{
    int w = 1;
    while (w < 16 && 4 * 2 * w <= P) w *= 2;
    return w;
}

template <int WAVES>
void launch_scanw(dim3 grid, size_t lds_b, hipStream_t s, const DevTables &dt, const WorkspaceW &W, int64_t N,
                  int32_t *out_lb)
{
    bound_scanw_kernel<WAVES, 8, 2><<<grid, 64 * WAVES, lds_b, s>>>(dt, W, N, out_lb);
}

}  // namespace

size_t wide_workspace_bytes(const fsp_instance_s *I, int64_t N) { return N > 0 ? wide_layout(I, N).total() : 0; }

hipError_t launch_bound_wide_ws(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N,
                                int32_t *out_lb, hipStream_t s, bool sort_depths, void *ws, bool marks)
{
    if (N <= 0) return hipSuccess;
    const int n = I->n, m = I->m;
    const int64_t G = (N + kGroupW - 1) / kGroupW, Npad = G * kGroupW;
    const int B = (int)std::min<int64_t>(kSortMaxBlocks, (N + 4095) / 4096);
    const int64_t chunk = (N + B - 1) / B;
    const WideLayout L = wide_layout(I, N);
    // every section is written in full before it is read: no clearing
    char *w = (char *)ws;
    WorkspaceW W;
    W.dec = (int32_t *)w;
    W.flg = (uint32_t *)(w + L.dec);
    W.st = (uint32_t *)(w + L.dec + L.flg);
    W.order = sort_depths ? (int32_t *)(w + L.dec + L.flg + L.st) : nullptr;
    W.cnt = (uint32_t *)(w + L.dec + L.flg + L.st + L.ord);

    if (marks) timing_mark(I, 0, s);
    if (sort_depths) launch_depth_sort(depths, N, n, B, chunk, W.cnt, W.order, s);
    const dim3 dgrid((unsigned)((Npad + 255) / 256));
    const int MV = (m + 3) & ~3;
    const size_t dlds = decodew_lds_words(n, MV) * 4;
#define FSP_DECODEW(MVV) \
    case MVV: bound_decodew_kernel<MVV><<<dgrid, 256, dlds, s>>>(I->dt, prefixes, depths, N, Npad, W, out_lb); break;
    switch (MV) {
        FSP_DECODEW(4) FSP_DECODEW(8) FSP_DECODEW(12) FSP_DECODEW(16)
        FSP_DECODEW(20) FSP_DECODEW(24) FSP_DECODEW(28) FSP_DECODEW(32)
    }
#undef FSP_DECODEW
    hipError_t e = hipGetLastError();
    if (marks) timing_mark(I, 1, s);
    if (e == hipSuccess) {
        const int waves = wide_waves(I->P);
        const size_t lds_b = (size_t)std::max(n + 1, waves) * 256;
        const dim3 grid((unsigned)G);
        switch (waves) {
        case 16: launch_scanw<16>(grid, lds_b, s, I->dt, W, N, out_lb); break;
        case 8: launch_scanw<8>(grid, lds_b, s, I->dt, W, N, out_lb); break;
        case 4: launch_scanw<4>(grid, lds_b, s, I->dt, W, N, out_lb); break;
        case 2: launch_scanw<2>(grid, lds_b, s, I->dt, W, N, out_lb); break;
        default: launch_scanw<1>(grid, lds_b, s, I->dt, W, N, out_lb); break;
        }
        e = hipGetLastError();
    }
    if (marks) timing_mark(I, 2, s);
    return e;
}

hipError_t launch_bound_wide(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N,
                             int32_t *out_lb, hipStream_t s, bool sort_depths)
{
    if (N <= 0) return hipSuccess;
    void *ws = nullptr;
    hipError_t e = stream_alloc(&ws, wide_workspace_bytes(I, N), s);
    if (e != hipSuccess) return e;
    e = launch_bound_wide_ws(I, prefixes, depths, N, out_lb, s, sort_depths, ws, true);
    hipError_t e2 = stream_free(ws, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace fspbb
