// Bounding a step's children from their parents (16-bit instances, plain
// releases).  A child appends one job j to its parent's prefix, so
//   - its releases extend the parent's completion times by j (one pass over
//     the machines),
//   - its unscheduled time on machine k is the parent's minus p[j][k],
//   - its tail on k is the least tail among the parent's unscheduled jobs
//     other than j: the parent's least one, or the second least when j is
//     the job holding the least,
//   - its unscheduled set is the parent's without j.
// Each parent is decoded once (order n m work) and each child in order m,
// where decoding a child from its row costs order n m.  The children's scan
// inputs go straight to the scan workspace and the pair scans are the plain
// kernel's, so every bound equals the one computed from the child's row.
// Child rows are never written: survivors are built from the parent copy.
#include <algorithm>

#include "kids16.h"
#include "lds_stage.h"
#include "scan16.h"
#include "step_dev.h"

namespace fspbb {

namespace {

// Stages the processing times as 16-bit pairs: row j holds machines (2c, 2c+1)
// in word c; row n is zero.  Every thread of the block calls it.
template <int H>
__device__ inline void stage_p16(int n, const int32_t *p32, uint32_t *p16)
{
    stage_lds<8>(p16, (n + 1) * H, [&](int e) {
        const int2 r = *reinterpret_cast<const int2 *>(p32 + (size_t)(e / H) * kMaxMachines + 2 * (e % H));
        return ((uint32_t)r.x & 0xffffu) | ((uint32_t)r.y << 16);
    });
    __syncthreads();
}

// Chain part, one lane per parent: completion times of the prefix and the
// time of the unscheduled jobs per machine.  With COUNT the parents are not
// validated yet (the tails part of the same launch does it): the depth is
// clamped to 0..n and a job outside 0..n-1 takes the zero row, so every read
// stays in bounds and an invalid parent's record, never used, is harmless.
// Otherwise parents with no children (invalid, or complete) are skipped.
// Block blk of the chain part; p16: LDS for the staged rows.
template <int MV, bool COUNT>
__device__ inline void kid_chain(ReqP q, int64_t blk, uint32_t *p16)
{
    constexpr int H = MV / 2;
    if (!q->w.prow || blk * 256 >= q->a.K) return;  // whole block
    const int n = q->T.n;
    stage_p16<H>(n, q->T.p32, p16);
    int32_t *__restrict__ rec = q->w.krec;
    const int64_t p = blk * 256 + threadIdx.x;
    if (p >= q->a.K) return;
    if (!COUNT && q->w.cnt[p] == 0) return;
    const int d = COUNT ? min(max(parent_depth(q, p), 0), n) : parent_depth(q, p);
    const int32_t *row = parent_row(q, p);
    int32_t C[MV];
    u16x2 S2[H];
#pragma unroll
    for (int k = 0; k < MV; ++k) C[k] = 0;
#pragma unroll
    for (int c = 0; c < H; ++c) S2[c] = u16x2{0, 0};
    // four prefix slots at a time; a slot past the depth takes the zero row,
    // which leaves the completion times unchanged
    auto step4 = [&](int32_t j0, int32_t j1, int32_t j2, int32_t j3, int t) {
        const int32_t jj[4] = {j0, j1, j2, j3};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = t + c < d && (unsigned)jj[c] < (unsigned)n ? jj[c] : n;
            const uint2 *pr = reinterpret_cast<const uint2 *>(p16 + __mul24(j, H));
            int32_t prev = 0;
#pragma unroll
            for (int q4 = 0; q4 < MV / 4; ++q4) {
                const uint2 v = pr[q4];
                S2[2 * q4] += as16(v.x);
                S2[2 * q4 + 1] += as16(v.y);
                const int32_t x[4] = {(int32_t)(v.x & 0xffffu), (int32_t)(v.x >> 16), (int32_t)(v.y & 0xffffu),
                                      (int32_t)(v.y >> 16)};
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const int k = 4 * q4 + cc;
                    C[k] = max(C[k], prev) + x[cc];
                    prev = C[k];
                }
            }
        }
    };
    if ((n & 3) == 0 && ((uintptr_t)row & 15) == 0) {
        // 16-byte row loads, two in flight (indices clamped into the prefix)
        const int4 *r4 = reinterpret_cast<const int4 *>(row);
        const int last = max(0, (d - 1) >> 2);
        int4 a = d > 0 ? r4[0] : int4{0, 0, 0, 0};
        for (int t = 0; t < d; t += 8) {
            const int4 b = r4[min((t >> 2) + 1, last)];
            step4(a.x, a.y, a.z, a.w, t);
            a = r4[min((t >> 2) + 2, last)];
            step4(b.x, b.y, b.z, b.w, t + 4);
        }
    } else {
        for (int t = 0; t < d; t += 4)
            step4(row[t], row[min(t + 1, d - 1)], row[min(t + 2, d - 1)], row[min(t + 3, d - 1)], t);
    }
    int32_t *r = rec + p * kKidRec;
    cptr<int32_t> cs = as_const(q->T.colsum32);
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        r[kKidC + k] = C[k];
        r[kKidU + k] = cs[k] - (int32_t)((k & 1) ? S2[k >> 1].y : S2[k >> 1].x);
    }
}

// Tails part, one wave per parent: copies the parent row, builds its
// unscheduled set, and lane k (< m) finds the least and second least tails on machine k over the
// unscheduled jobs, taken in increasing id.  With COUNT it also validates the
// parent and writes its child count (the count kernel's work); otherwise the
// count kernel has done so.
// Block blk of the tails part (four parents); mask: 4 x kMaskWords words of LDS.
template <bool COUNT>
__device__ inline void kid_tails(ReqP q, int64_t blk, uint32_t (*mask)[kMaskWords])
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = blk * 4 + wv;
    if (!q->w.prow) return;        // whole block: the request bounds children from rows
    if (p >= q->a.K) return;       // whole wave
    if (!COUNT && q->w.cnt[p] == 0) return;  // whole wave
    int32_t *__restrict__ rec = q->w.krec;
    int32_t *__restrict__ prow = q->w.prow;
    const int32_t *__restrict__ tails32 = q->T.tails32;
    const int n = q->T.n, m = q->T.m, NW = (n + 31) >> 5;
    const int d = parent_depth(q, p);
    const int32_t *row = parent_row(q, p);
    const bool ok = wave_prefix_set(row, d, n, mask[wv], lane);  // reads the row only for a depth in 0..n
    if (COUNT) {
        if (lane == 0) {
            q->w.cnt[p] = (ok && d < n) ? (uint32_t)(n - d) : 0u;
            if (!ok) atomicAdd(q->w.bad, 1ull);
        }
        if (!ok || d == n) return;  // whole wave: no children
    }
    int32_t *pr = prow + p * (int64_t)n;
    for (int t = lane; t < d; t += 64) pr[t] = row[t];
    int32_t *r = rec + p * kKidRec;
    if (lane < NW) {
        const int lo = lane * 32;
        const uint32_t valid = n >= lo + 32 ? 0xffffffffu : ((1u << (n - lo)) - 1u);
        r[kKidM + lane] = (int32_t)(~mask[wv][lane] & valid);
    }
    int32_t q1 = 0x7fffffff, j1 = 0, q2 = 0x7fffffff;
    const int k = lane < m ? lane : 0;
    for (int w = 0; w < NW; ++w) {
        const uint32_t sched = __builtin_amdgcn_readfirstlane(mask[wv][w]);
        const int jn = min(32, n - 32 * w);
        const int32_t *tw = tails32 + (size_t)(32 * w) * kMaxMachines + k;
#pragma unroll 8
        for (int b = 0; b < jn; ++b) {
            const int32_t t = tw[(size_t)b * kMaxMachines];
            const int32_t v = ((sched >> b) & 1u) ? 0x7fffffff : t;
            const bool lt1 = v < q1;
            q2 = lt1 ? q1 : min(q2, v);
            j1 = lt1 ? 32 * w + b : j1;
            q1 = lt1 ? v : q1;
        }
    }
    if (lane < m) {
        r[kKidQ1 + lane] = q1;
        r[kKidJ1 + lane] = j1;
        r[kKidQ2 + lane] = q2;
    }
}

// Both per-parent parts in one launch: blocks [0, bc) the chain part, the
// rest the tails part (block-uniform branch).
template <int MV, bool COUNT>
__global__ __launch_bounds__(256) void kid_parents_kernel(const StepReq *__restrict__ reqs, int bc)
{
    extern __shared__ uint32_t p16[];
    __shared__ uint32_t mask[4][kMaskWords];
    ReqP q = req_of(reqs);
    if ((int)blockIdx.x < bc) kid_chain<MV, COUNT>(q, blockIdx.x, p16);
    else kid_tails<COUNT>(q, (int64_t)blockIdx.x - bc, mask);
}

// Position of the k-th set bit (from 0) of x, which has more than k set bits.
__device__ __forceinline__ int select_bit(uint32_t x, int k)
{
    int pos = 0;
#pragma unroll
    for (int sh = 16; sh > 0; sh >>= 1) {
        const uint32_t lo = x & ((1u << sh) - 1u);
        const int c = __popc(lo);
        if (k >= c) {
            k -= c;
            x >>= sh;
            pos += sh;
        } else {
            x = lo;
        }
    }
    return pos;
}

// One lane per child (and per padding slot up to the group boundary): writes
// the scan inputs of child i in the decode kernel's layout, and its depth.
// With LIST it also finds the child's parent (the last one whose offset is
// at most i) and appended job (the (i - offset)-th unscheduled job of the
// parent, in increasing id) and writes them, the list kernel's work, and
// takes the leaf step for complete children (the leaf kernel's work).
template <int MV, bool LIST>
__global__ __launch_bounds__(256) void kid_decode_kernel(const StepReq *__restrict__ reqs)
{
    constexpr int H = MV / 2;
    extern __shared__ uint32_t p16[];
    ReqP q = req_of(reqs);
    const int64_t N = q->nchild, Npad = (N + kGroup - 1) / kGroup * kGroup;
    if (!q->w.prow || (int64_t)blockIdx.x * 256 >= Npad) return;  // whole block
    const int n = q->T.n, m = q->T.m, NW = (n + 31) >> 5;
    stage_p16<H>(n, q->T.p32, p16);
    const int32_t *__restrict__ rec = q->w.krec;
    uint32_t *const Wdec = q->w.kw.dec, *const Wflg = q->w.kw.flg, *const Wst = q->w.kw.st;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= Npad) return;
    const bool live = i < N;
    int32_t j = n;  // the zero row for padding slots
    int64_t p = 0;
    int d = 0;
    if (live) {
        if (LIST) {
            const uint32_t *off = q->w.off;
            int64_t lo = 0, hi = q->a.K - 1;  // off[0] = 0 <= i
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if ((int64_t)off[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            p = lo;
            int k = (int)(i - (int64_t)off[p]);
            const int32_t *rp = rec + p * kKidRec;
            j = n;
            for (int w = 0; w < NW; ++w) {
                const uint32_t bits = (uint32_t)rp[kKidM + w];
                const int c = __popc(bits);
                if (k < c) {
                    j = 32 * w + select_bit(bits, k);
                    break;
                }
                k -= c;
            }
            // (a step with an invalid parent has fewer children than listed;
            // it is reported, and the zero row keeps the reads in bounds)
            j = min(j, n);
            q->w.ujob[i] = j;
            q->w.upar[i] = (int32_t)p;
        } else {
            j = q->w.ujob[i];
            p = q->w.upar[i];
        }
        d = parent_depth(q, p) + 1;
        q->w.cdepth[i] = d;
    }
    const int32_t *r = rec + p * kKidRec;
    const uint2 *pj = reinterpret_cast<const uint2 *>(p16 + __mul24(j, H));
    const bool empty = d == n;  // a complete child: no tail
    const int64_t G = i >> 7;
    const int g = (int)(i & 127), lane = g & 63, half = g >> 6;
    uint16_t *d16 = reinterpret_cast<uint16_t *>(Wdec);
    int32_t prev = 0, mk = 0;
#pragma unroll
    for (int q4 = 0; q4 < MV / 4; ++q4) {
        const uint2 v = pj[q4];
        const int32_t x[4] = {(int32_t)(v.x & 0xffffu), (int32_t)(v.x >> 16), (int32_t)(v.y & 0xffffu),
                              (int32_t)(v.y >> 16)};
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int k = 4 * q4 + cc;
            const int32_t ck = max(r[kKidC + k], prev) + x[cc];
            prev = ck;
            if (k == m - 1) mk = ck;
            if (k < m) {
                const int32_t tk = ck + (r[kKidU + k] - x[cc]);
                const int32_t qk = r[kKidJ1 + k] == j ? r[kKidQ2 + k] : r[kKidQ1 + k];
                d16[((G * 3 + 0) * m + k) * 128 + lane * 2 + half] = (uint16_t)(live ? ck : 0);
                d16[((G * 3 + 1) * m + k) * 128 + lane * 2 + half] = (uint16_t)(live ? tk : 0);
                d16[((G * 3 + 2) * m + k) * 128 + lane * 2 + half] = (uint16_t)(live && !empty ? qk : 0);
            }
        }
    }
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) {
        if (w < NW) {
            const uint32_t drop = (j >> 5) == w ? 1u << (j & 31) : 0u;
            Wflg[(G * NW + w) * 128 + g] = live ? ((uint32_t)r[kKidM + w] & ~drop) : 0u;
        }
    }
    // With LIST the leaf step is done here too: a complete child's bound is
    // its makespan (its releases on every pair, no job left, and a pair
    // ending on the last machine), the last completion time just computed.
    if (LIST && live && empty && mk < q->a.ub_in)
        atomicMin(q->w.best, ((unsigned long long)(uint32_t)mk << 32) | (unsigned long long)i);
    Wst[i] = live ? 1u : 0u;
    // a scan split over several workgroups takes its bounds by atomic max
    if (live && q->w.clb) q->w.clb[i] = 0;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// segs: null for the plain form (counts, offsets and the child lists done
// by the step kernels); else the offset scan segments, and the parents'
// launch counts and the decode lists (the form without the count and list
// launches).
template <int MV>
hipError_t launch_kids(const StepReq *dreqs, int R, int64_t maxK, int64_t maxC, int nmax, const ScanSeg *segs,
                       hipStream_t s)
{
    const size_t lds = (size_t)(nmax + 1) * (MV / 2) * 4;
    const int64_t Npad = (maxC + kGroup - 1) / kGroup * kGroup;
    const int bc = (int)((maxK + 255) / 256), bt = (int)((maxK + 3) / 4);
    const dim3 gp((unsigned)(bc + bt), R), gd((unsigned)((Npad + 255) / 256), R);
    if (!segs) {
        kid_parents_kernel<MV, false><<<gp, 256, lds, s>>>(dreqs, bc);
        kid_decode_kernel<MV, false><<<gd, 256, lds, s>>>(dreqs);
        return hipGetLastError();
    }
    kid_parents_kernel<MV, true><<<gp, 256, lds, s>>>(dreqs, bc);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = exclusive_scan_segments(segs, R, maxK, s);
    if (e != hipSuccess) return e;
    kid_decode_kernel<MV, true><<<gd, 256, lds, s>>>(dreqs);
    return hipGetLastError();
}

}  // namespace

bool kids16_eligible(const fsp_instance_s *I) { return I->packed16 && !I->dt.heads; }

hipError_t kids16_ensure(Kids16 &k, const fsp_instance_s *I, int64_t K, int64_t nch, hipStream_t s)
{
    k.K = K;
    k.nch = nch;
    if (k.blob && K <= k.capK && nch <= k.capC && I->n == k.n && I->m == k.m) return hipSuccess;
    if (k.blob) stream_free(k.blob, s);
    k.blob = nullptr;
    const int n = I->n, m = I->m, NW = (n + 31) >> 5;
    // both grow by doubling: a search's steps vary by a few children
    const int64_t capK = std::max<int64_t>({K, 2 * k.capK, 1}), capC = std::max<int64_t>({nch, 2 * k.capC, kGroup});
    const int64_t G = (capC + kGroup - 1) / kGroup;
    const size_t rows_b = al256((size_t)capK * n * 4), rec_b = al256((size_t)capK * kKidRec * 4),
                 dec_b = al256((size_t)G * 3 * m * 64 * 4), flg_b = al256((size_t)G * NW * 128 * 4),
                 st_b = al256((size_t)G * kGroup * 4);
    hipError_t e = stream_alloc(&k.blob, rows_b + rec_b + dec_b + flg_b + st_b, s);
    if (e != hipSuccess) {
        k = Kids16{};
        return e;
    }
    k.capK = capK;
    k.capC = capC;
    k.bytes = rows_b + rec_b + dec_b + flg_b + st_b;
    k.n = n;
    k.m = m;
    char *b = (char *)k.blob;
    k.prow = (int32_t *)b;
    k.rec = (int32_t *)(b + rows_b);
    k.W.dec = (uint32_t *)(b + rows_b + rec_b);
    k.W.flg = (uint32_t *)(b + rows_b + rec_b + dec_b);
    k.W.st = (uint32_t *)(b + rows_b + rec_b + dec_b + flg_b);
    k.W.order = nullptr;
    k.W.cnt = nullptr;
    return hipSuccess;
}

namespace {
// Byte sizes of one search's scratch: parent rows, parent records, decode,
// bits, valid flags (each 256-byte aligned).
struct KidsSizes {
    size_t rows, rec, dec, flg, st;
    KidsSizes(int n, int m, int64_t K, int64_t C)
    {
        const int NW = (n + 31) >> 5;
        const int64_t G = std::max<int64_t>((C + kGroup - 1) / kGroup, 1);
        rows = al256((size_t)std::max<int64_t>(K, 1) * n * 4);
        rec = al256((size_t)std::max<int64_t>(K, 1) * kKidRec * 4);
        dec = al256((size_t)G * 3 * m * 64 * 4);
        flg = al256((size_t)G * NW * 128 * 4);
        st = al256((size_t)G * kGroup * 4);
    }
    size_t total() const { return rows + rec + dec + flg + st; }
    void point(char *b, Kids16 &k) const
    {
        k.prow = (int32_t *)b;
        k.rec = (int32_t *)(b + rows);
        k.W.dec = (uint32_t *)(b + rows + rec);
        k.W.flg = (uint32_t *)(b + rows + rec + dec);
        k.W.st = (uint32_t *)(b + rows + rec + dec + flg);
        k.W.order = nullptr;
        k.W.cnt = nullptr;
    }
};
}  // namespace

size_t KidsArena::step_bytes(const fsp_instance_s *I, int64_t K, int64_t nch)
{
    return KidsSizes(I->n, I->m, K, nch).total();
}

hipError_t KidsArena::layout(const std::vector<const fsp_instance_s *> &I, const std::vector<int64_t> &K,
                             const std::vector<int64_t> &nch, std::vector<Kids16> &out, hipStream_t s)
{
    size_t need = 0;
    for (size_t i = 0; i < I.size(); ++i) need += step_bytes(I[i], K[i], nch[i]);
    if (need > cap) {
        const size_t c = cap_after(need);
        if (blob) stream_free(blob, s);
        blob = nullptr;
        cap = 0;
        hipError_t e = stream_alloc(&blob, c, s);
        if (e != hipSuccess) return e;
        cap = c;
    }
    out.assign(I.size(), Kids16{});
    char *b = (char *)blob;
    for (size_t i = 0; i < I.size(); ++i) {
        const KidsSizes z(I[i]->n, I[i]->m, K[i], nch[i]);
        z.point(b, out[i]);
        out[i].K = K[i];
        out[i].nch = nch[i];
        b += z.total();
    }
    return hipSuccess;
}

void KidsArena::release(hipStream_t s)
{
    if (blob) stream_free(blob, s);
    blob = nullptr;
    cap = 0;
}

void kids16_release(Kids16 &k, hipStream_t s)
{
    if (k.blob) stream_free(k.blob, s);
    k = Kids16{};
}

void kids16_point(StepScratch &w, const Kids16 &k)
{
    w.prow = k.prow;
    w.krec = k.rec;
    w.kw = k.W;
}

hipError_t kids16_decode(const StepReq *dreqs, int R, int64_t maxK, int64_t maxC, int nmax, int mmax, hipStream_t s,
                         const ScanSeg *segs)
{
    if (R <= 0 || maxK <= 0 || maxC <= 0) return hipSuccess;
    switch ((mmax + 3) & ~3) {
    case 4: return launch_kids<4>(dreqs, R, maxK, maxC, nmax, segs, s);
    case 8: return launch_kids<8>(dreqs, R, maxK, maxC, nmax, segs, s);
    case 12: return launch_kids<12>(dreqs, R, maxK, maxC, nmax, segs, s);
    case 16: return launch_kids<16>(dreqs, R, maxK, maxC, nmax, segs, s);
    case 20: return launch_kids<20>(dreqs, R, maxK, maxC, nmax, segs, s);
    case 24: return launch_kids<24>(dreqs, R, maxK, maxC, nmax, segs, s);
    case 28: return launch_kids<28>(dreqs, R, maxK, maxC, nmax, segs, s);
    default: return launch_kids<32>(dreqs, R, maxK, maxC, nmax, segs, s);
    }
}

hipError_t kids16_bound(const StepReq *dreq, fsp_instance_s *I, Kids16 &k, int32_t *clb, hipStream_t s)
{
    if (k.nch <= 0 || k.K <= 0) return hipSuccess;
    hipError_t e = kids16_decode(dreq, 1, k.K, k.nch, I->n, I->m, s);
    if (e != hipSuccess) return e;
    return launch_scan16(I, k.W, k.nch, clb, s);
}

}  // namespace fspbb
