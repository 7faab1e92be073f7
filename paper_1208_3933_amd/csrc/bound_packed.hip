// Fast bound path for instances whose values fit 16 bits ((n+m-1) * max p <
// 65536, true of every U[1,99] instance up to 500 jobs x 20 machines): the
// depth sort and the decode of a pool, its launch, and the batched forms of
// decode and scan.  The plain scan kernel is in scan16_plain.hip.
//
// Two kernels per pool:
//   decode  one lane per node: scheduled set, releases, closing sums and tails
//           (the per-node RM/QM work of Table I), written to a workspace in a
//           layout the scan reads with unit stride;
//   scan    one workgroup per group of 128 nodes, two nodes per lane as 16-bit
//           halves, records as wave-uniform scalar loads, masks in LDS.
#include <algorithm>
#include <cstdlib>

#include "batch.h"
#include "lds_stage.h"
#include "scan16.h"

namespace fspbb {

// Packed halves for tail minima (instances whose tails are at most
// kTailsHalfMax): two tails as the bits of two half-precision numbers, which
// order as the integers do.  kHalfNone (0x7bff twice) stands for a scheduled
// job: above every tail.
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h16x2 as_h16(uint32_t x) { return __builtin_bit_cast(h16x2, x); }
constexpr uint32_t kHalfNone = 0x7bff7bffu;

// ---- counting sort of node indices by depth (bucket n+1 holds invalid depths)

__device__ __forceinline__ int depth_bucket(int d, int n) { return (d >= 0 && d <= n) ? d : n + 1; }

constexpr int kSortPer = 16;  // depths in flight per thread

// Block `blk` of B: histogram of the depths of nodes [blk*chunk, (blk+1)*chunk)
// into cnt[bucket * B + blk].  h: n + 2 words of LDS.
__device__ inline void depth_count_block(const int32_t *__restrict__ depths, int64_t N, int n, int64_t chunk, int B,
                                         uint32_t *__restrict__ cnt, int64_t blk, uint32_t *h)
{
    for (int b = threadIdx.x; b < n + 2; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int64_t lo = blk * chunk, hi = min(N, lo + chunk);
    // each thread's depths are loaded kSortPer at a time before their counts
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (int64_t)kSortPer * blockDim.x) {
        int32_t dv[kSortPer];
#pragma unroll
        for (int k = 0; k < kSortPer; ++k) dv[k] = depths[min(i0 + (int64_t)k * blockDim.x, hi - 1)];
#pragma unroll
        for (int k = 0; k < kSortPer; ++k)
            if (i0 + (int64_t)k * blockDim.x < hi) atomicAdd(&h[depth_bucket(dv[k], n)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n + 2; b += blockDim.x) cnt[(int64_t)b * B + blk] = h[b];
}

// Block `blk` of B: each node goes to the next free position of its depth
// bucket.  The first position of bucket b in this block is the number of
// nodes in smaller buckets (over all blocks) plus those of bucket b in the
// blocks before it; the block sums the per-block counts itself (B is at most
// kSortMaxBlocks, so this is a few thousand cached reads).
// sh: 2 (n + 2) + 256 words of LDS.
__device__ inline void depth_scatter_block(const int32_t *__restrict__ depths, int64_t N, int n, int64_t chunk, int B,
                                           const uint32_t *__restrict__ cnt, int32_t *__restrict__ order, int64_t blk,
                                           uint32_t *sh)
{
    const int t = threadIdx.x, nb = n + 2;
    uint32_t *cur = sh, *tot = sh + nb, *part = sh + 2 * nb;
    for (int b = t; b < nb; b += blockDim.x) {
        const uint32_t *c = cnt + (int64_t)b * B;
        uint32_t all = 0, before = 0;
        if ((B & 3) == 0) {  // rows of 16-byte multiples (cnt is 256-byte aligned): 16-byte loads
            const uint4 *c4 = reinterpret_cast<const uint4 *>(c);
#pragma unroll 4
            for (int k4 = 0; k4 < (B >> 2); ++k4) {
                const uint4 v = c4[k4];
                const int k = 4 * k4;
                all += v.x + v.y + v.z + v.w;
                before += (k < blk ? v.x : 0u) + (k + 1 < blk ? v.y : 0u) + (k + 2 < blk ? v.z : 0u) +
                          (k + 3 < blk ? v.w : 0u);
            }
        } else {
            for (int k = 0; k < B; ++k) {
                const uint32_t v = c[k];
                all += v;
                before += k < blk ? v : 0u;
            }
        }
        tot[b] = all;
        cur[b] = before;
    }
    __syncthreads();
    // exclusive scan of tot over the buckets: each thread sums a run of
    // buckets, the runs are scanned across the block, then walked again
    const int per = (nb + blockDim.x - 1) / blockDim.x, lo = t * per, hi = min(nb, lo + per);
    uint32_t run = 0;
    for (int b = lo; b < hi; ++b) run += tot[b];
    part[t] = run;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t base = part[t] - run;
    for (int b = lo; b < hi; ++b) {
        cur[b] += base;
        base += tot[b];
    }
    __syncthreads();
    const int64_t lo_i = blk * chunk, hi_i = min(N, lo_i + chunk);
    for (int64_t i0 = lo_i + t; i0 < hi_i; i0 += (int64_t)kSortPer * blockDim.x) {
        int32_t dv[kSortPer];
#pragma unroll
        for (int k = 0; k < kSortPer; ++k) dv[k] = depths[min(i0 + (int64_t)k * blockDim.x, hi_i - 1)];
#pragma unroll
        for (int k = 0; k < kSortPer; ++k) {
            const int64_t i = i0 + (int64_t)k * blockDim.x;
            if (i < hi_i) {
                const uint32_t pos = atomicAdd(&cur[depth_bucket(dv[k], n)], 1u);
                order[pos] = (int32_t)i;
            }
        }
    }
}

__global__ __launch_bounds__(256) void depth_count_kernel(const int32_t *__restrict__ depths, int64_t N, int n,
                                                          int64_t chunk, int B, uint32_t *__restrict__ cnt)
{
    extern __shared__ uint32_t h[];
    depth_count_block(depths, N, n, chunk, B, cnt, blockIdx.x, h);
}

__global__ __launch_bounds__(256) void depth_scatter_kernel(const int32_t *__restrict__ depths, int64_t N, int n,
                                                            int64_t chunk, int B, const uint32_t *__restrict__ cnt,
                                                            int32_t *__restrict__ order)
{
    extern __shared__ uint32_t sh[];
    depth_scatter_block(depths, N, n, chunk, B, cnt, order, blockIdx.x, sh);
}

void launch_depth_sort(const int32_t *depths, int64_t N, int n, int B, int64_t chunk, uint32_t *cnt, int32_t *order,
                       hipStream_t s)
{
    const size_t hb = (size_t)(n + 2) * 4, sb = ((size_t)(n + 2) * 2 + 256) * 4;
    depth_count_kernel<<<B, 256, hb, s>>>(depths, N, n, chunk, B, cnt);
    depth_scatter_kernel<<<B, 256, sb, s>>>(depths, N, n, chunk, B, cnt, order);
}

// ---- decode: one lane per node, nodes taken in depth order
//
// Computes for each node its scheduled set (rejecting out-of-range and
// repeated jobs), the completion times of its prefix on every machine (the
// releases, RM of Table I), the time of the unscheduled jobs on each machine,
// and the tails (QM of Table I: least time left after machine l over the
// unscheduled jobs).  MV = m rounded up to a multiple of 4.
//   - The processing times are staged in LDS as 16-bit pairs (machines 2c and
//     2c+1 of a job in one dword): the sums of the scheduled jobs' times are
//     packed adds, and the completion-time recurrence takes each time as a
//     16-bit half of a dword.
//   - Each lane keeps its scheduled set as bits in LDS, set by OR writes that
//     return nothing; a repeated job shows at the end as fewer set bits than
//     the depth.
//   - The tails are taken two machines at a time with packed minima over a
//     scalar-loaded table, four jobs per batch of scalar loads: packed
//     half-precision three-operand minima when every tail is at most
//     kTailsHalfMax, packed 16-bit integer minima otherwise.
// Decodes block `blk` (256 nodes) of one pool; every thread of the block calls it.
// sm: dynamic LDS of decode16_lds_words(n, MV) words.
template <int MV>
__device__ inline void decode16_block(const DevTables &T, const int32_t *__restrict__ prefixes,
                                      const int32_t *__restrict__ depths, int64_t N, int64_t Npad,
                                      const Workspace16 &W, int32_t *__restrict__ out_lb, int64_t blk,
                                      uint32_t *sm, bool zero_lb = false)
{
    constexpr int H = MV / 2;  // packed pairs per job row
    const int n = T.n, m = T.m, NW = (n + 31) >> 5;
    uint32_t *bits = sm;                       // (n / 32 + 1) words x 256 lanes: job bits, job n's bit included
    uint32_t *p16 = sm + ((n >> 5) + 1) * 256;  // (n + 1) x H; row n is zero
    const int tid = threadIdx.x;
    stage_lds<8>(p16, (n + 1) * H, [&](int e) {
        const int2 r = *reinterpret_cast<const int2 *>(T.p32 + (size_t)(e / H) * kMaxMachines + 2 * (e % H));
        return ((uint32_t)r.x & 0xffffu) | ((uint32_t)r.y << 16);
    });
    __syncthreads();

    const int64_t i = blk * 256 + tid;
    if (i >= Npad) return;
    const bool live = i < N;
    const int64_t node = live ? (W.order ? W.order[i] : i) : 0;
    int d = live ? depths[node] : 0;
    bool ok = live && d >= 0 && d <= n;
    if (!ok) d = 0;

    uint32_t *mybits = bits + tid;
    for (int w = 0; w < NW; ++w) mybits[w * 256] = 0u;
    int32_t C[MV];
    u16x2 S2[H];
#pragma unroll
    for (int k = 0; k < MV; ++k) C[k] = 0;
#pragma unroll
    for (int c = 0; c < H; ++c) S2[c] = u16x2{0, 0};
    // Slots t..t+3 of the prefix, branch-free.  An out-of-range job becomes
    // job n: the zero row, which leaves the completion times unchanged (they
    // never decrease along the machines), and a bit outside the job mask, so
    // that the node's count of scheduled jobs falls short of its depth.  With
    // `tail`, slots past the depth take job n too.
    auto step4 = [&](int32_t j0, int32_t j1, int32_t j2, int32_t j3, int t, bool tail) {
        const int32_t jj[4] = {j0, j1, j2, j3};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int j = (int)min((uint32_t)jj[c], (uint32_t)n);
            if (tail && t + c >= d) j = n;
            atomicOr(&mybits[(j >> 5) * 256], 1u << (j & 31));
            const uint2 *pr = reinterpret_cast<const uint2 *>(p16 + __mul24(j, H));
            int32_t prev = 0;
#pragma unroll
            for (int q = 0; q < MV / 4; ++q) {
                const uint2 v = pr[q];
                S2[2 * q] += as16(v.x);
                S2[2 * q + 1] += as16(v.y);
                const int32_t x[4] = {(int32_t)(v.x & 0xffffu), (int32_t)(v.x >> 16),
                                      (int32_t)(v.y & 0xffffu), (int32_t)(v.y >> 16)};
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const int k = 4 * q + cc;
                    const int32_t ck = max(C[k], prev) + x[cc];
                    C[k] = ck;
                    prev = ck;
                }
            }
        }
    };
    const int32_t *row = prefixes + node * (int64_t)n;
    if ((n & 3) == 0 && ((uintptr_t)prefixes & 15) == 0) {
        // rows of a multiple of 4 jobs are 16-byte aligned: one vector load
        // per 4 jobs, two loads in flight (indices clamped into the prefix,
        // so no line past the depth is fetched)
        const int4 *r4 = reinterpret_cast<const int4 *>(row);
        const int last = max(0, (d - 1) >> 2);
        int4 a = d > 0 ? r4[0] : int4{0, 0, 0, 0};
        int t = 0;
        for (; t + 8 <= d; t += 8) {
            const int4 b = r4[min((t >> 2) + 1, last)];
            step4(a.x, a.y, a.z, a.w, t, false);
            a = r4[min((t >> 2) + 2, last)];
            step4(b.x, b.y, b.z, b.w, t + 4, false);
        }
        if (t < d) {  // the last 1 to 7 slots
            const int4 b = r4[min((t >> 2) + 1, last)];
            step4(a.x, a.y, a.z, a.w, t, true);
            if (t + 4 < d) step4(b.x, b.y, b.z, b.w, t + 4, true);
        }
    } else {
        for (int t = 0; t < d; t += 4)
            step4(row[t], row[min(t + 1, d - 1)], row[min(t + 2, d - 1)], row[min(t + 3, d - 1)], t, true);
    }

    u32v<kMaskWords> act;
    int nset = 0;
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) {
        const int lo = w * 32;
        const uint32_t valid = n >= lo + 32 ? 0xffffffffu : (n <= lo ? 0u : ((1u << (n - lo)) - 1u));
        const uint32_t b = (w < NW ? mybits[w * 256] : 0u) & valid;
        nset += __popc(b);
        act[w] = ~b & valid;
    }
    ok = ok && nset == d;  // fewer bits than slots: a job out of range or repeated
    if (!ok) {
#pragma unroll
        for (int w = 0; w < kMaskWords; ++w) act[w] = 0u;
    }
    // heads: with T.heads, each machine's release becomes the earliest start
    // on it of an unscheduled job scheduled next (uniform job loop: the time
    // rows are LDS broadcasts)
    if (T.heads && ok && d < n) {
        int32_t h[MV];
#pragma unroll
        for (int k = 0; k < MV; ++k) h[k] = 0x7fffffff;
        for (int j = 0; j < n; ++j) {
            const bool a = (act[j >> 5] >> (j & 31)) & 1u;
            const uint2 *pr = reinterpret_cast<const uint2 *>(p16 + j * H);
            int32_t prev = 0;
#pragma unroll
            for (int q = 0; q < MV / 4; ++q) {
                const uint2 v = pr[q];
                const int32_t x[4] = {(int32_t)(v.x & 0xffffu), (int32_t)(v.x >> 16),
                                      (int32_t)(v.y & 0xffffu), (int32_t)(v.y >> 16)};
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
    // tails, two machines per register: q = min over jobs of (Q | inactive mask)
    uint32_t q2[H];
    if (__all(2 * d <= n)) {
        // a wave of nodes at most half deep: each machine's tail is that of
        // the first job, in increasing tail order on the machine, that the
        // node has not scheduled; a few ranks usually reach it for every
        // lane and machine, against a minimum over all n jobs
        uint32_t qv[MV], need = 0;  // need: machines still without a tail
#pragma unroll
        for (int k = 0; k < MV; ++k) {
            qv[k] = 0;
            if (k < m) need |= 1u << k;
        }
        for (int r = 0; r < n; ++r) {
            cptr<uint32_t> row = as_const(T.tord + (size_t)r * kMaxMachines);
#pragma unroll
            for (int k = 0; k < MV; ++k) {
                if (k < m) {
                    const uint32_t e = row[k], j = e >> 16;
                    const bool take = ((need >> k) & 1u) && !((mybits[(j >> 5) * 256] >> (j & 31)) & 1u);
                    qv[k] = take ? (e & 0xffffu) : qv[k];
                    need = take ? need & ~(1u << k) : need;
                }
            }
            if (__all(need == 0)) break;
        }
#pragma unroll
        for (int c = 0; c < H; ++c) q2[c] = qv[2 * c] | (qv[2 * c + 1] << 16);
    } else if (T.tails16ok == 2) {
        // every tail is at most kTailsHalfMax: minima as packed halves, two
        // jobs per three-operand minimum; a scheduled job contributes 0x7bff
        h16x2 qh[H];
#pragma unroll
        for (int c = 0; c < H; ++c) qh[c] = as_h16(kHalfNone);
        // the constant in a vector register, so that each select reads its
        // scalar-loaded tail directly (one scalar operand per instruction)
        uint32_t none;
        asm volatile("v_mov_b32 %0, %1" : "=v"(none) : "i"(kHalfNone));
        for (int w = 0; w < NW; ++w) {
            const uint32_t aw = act[w];
            const int jn = min(32, n - 32 * w);
            cptr<uint32_t> qw = as_const(T.tails16 + (size_t)(32 * w) * (kMaxMachines / 2));
            int b = 0;
            for (; b + 4 <= jn; b += 4) {
#pragma unroll
                for (int u = 0; u < 4; u += 2) {
                    const uint32_t offa = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)aw, b + u, 1);
                    const uint32_t offb = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)aw, b + u + 1, 1);
                    cptr<uint32_t> qa = qw + (size_t)(b + u) * (kMaxMachines / 2);
                    cptr<uint32_t> qb = qa + kMaxMachines / 2;
#pragma unroll
                    for (int c = 0; c < H; ++c)
                        qh[c] = __builtin_elementwise_minimum(
                            __builtin_elementwise_minimum(qh[c], as_h16((qa[c] & ~offa) | (none & offa))),
                            as_h16((qb[c] & ~offb) | (none & offb)));
                }
            }
            for (; b < jn; ++b) {
                const uint32_t off = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)aw, b, 1);
                cptr<uint32_t> qr = qw + (size_t)b * (kMaxMachines / 2);
#pragma unroll
                for (int c = 0; c < H; ++c)
                    qh[c] = __builtin_elementwise_minimum(qh[c], as_h16((qr[c] & ~off) | (none & off)));
            }
        }
#pragma unroll
        for (int c = 0; c < H; ++c) q2[c] = __builtin_bit_cast(uint32_t, qh[c]);
    } else {
#pragma unroll
        for (int c = 0; c < H; ++c) q2[c] = 0xffffffffu;
        for (int w = 0; w < NW; ++w) {
            const uint32_t aw = act[w];
            const int jn = min(32, n - 32 * w);
            cptr<uint32_t> qw = as_const(T.tails16 + (size_t)(32 * w) * (kMaxMachines / 2));
            int b = 0;
            for (; b + 4 <= jn; b += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t off = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)aw, b + u, 1);
                    cptr<uint32_t> qr = qw + (size_t)(b + u) * (kMaxMachines / 2);
#pragma unroll
                    for (int c = 0; c < H; ++c)
                        q2[c] = as32(__builtin_elementwise_min(as16(q2[c]), as16(qr[c] | off)));
                }
            }
            for (; b < jn; ++b) {
                const uint32_t off = ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)aw, b, 1);
                cptr<uint32_t> qr = qw + (size_t)b * (kMaxMachines / 2);
#pragma unroll
                for (int c = 0; c < H; ++c)
                    q2[c] = as32(__builtin_elementwise_min(as16(q2[c]), as16(qr[c] | off)));
            }
        }
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
            const int32_t sk = (k & 1) ? S2[k >> 1].y : S2[k >> 1].x;
            d16[((G * 3 + 0) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? C[k] : 0);
            d16[((G * 3 + 1) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? C[k] + (cs[k] - sk) : 0);
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
    } else if (live && zero_lb) {
        out_lb[node] = 0;  // the split scan takes the maximum over its workgroups into it
    }
}

// zero_lb: write 0 to each valid node's bound, for a scan split over
// several workgroups per group.  Up to 20 machines, five waves per SIMD (at
// most 96 registers; at 20 machines one 8-byte spill outside the prefix
// loop): the decode is latency-bound, and the fifth wave takes 1.7% off it
// at 200x20.
template <int MV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MV <= 20 ? 5 : 1))) void bound_decode16_kernel(DevTables T, const int32_t *__restrict__ prefixes,
                                                             const int32_t *__restrict__ depths, int64_t N,
                                                             int64_t Npad, Workspace16 W,
                                                             int32_t *__restrict__ out_lb, int zero_lb)
{
    extern __shared__ uint32_t sm[];
    decode16_block<MV>(T, prefixes, depths, N, Npad, W, out_lb, blockIdx.x, sm, zero_lb != 0);
}

// ---- decode with four or eight lanes per node, for pools too small to fill the chip
//
// The one-lane decode above is latency-bound on a small pool: each lane walks
// its whole prefix through all m machines one job at a time.  Here the L
// lanes of a node (L = 4 or 8, aligned) split the machines, lane q holding
// machines [q*MQ, (q+1)*MQ), and the completion-time recurrence of the prefix
// runs as a pipeline across them: at step s lane q takes job s - q, with the
// completion time on the machine before its first one handed over by lane
// q - 1 (a one-lane DPP shift), the only value that crosses lanes.
//
// The block's 256 / L prefix rows are staged in LDS, each in a slot row with
// L words of padding before it and room after it for the pipeline's reads
// past the deepest prefix.  A first pass, with the prefix split over the
// node's lanes, checks every job's range, sets the scheduled bits (LDS ORs; a
// repeated job shows at the end as fewer set bits than the depth) and
// replaces each entry by the offset of the job's time row, or of the zero
// row for an invalid job or an entry past the depth; the padding holds the
// zero row too.  A step before a lane's first job or past the prefix thus
// reads the zero row, which leaves the completion times unchanged, because
// they never decrease along the machines.  Step s of lane q reads entry
// s - q at a fixed distance from its own base: the offsets are read four
// steps ahead, the time rows two steps ahead, and a step spends one address
// add on them.  The tails split the jobs over the node's lanes (job j to
// lane j mod L), with packed 16-bit minima combined across them.
//
// Writes the scan workspace in the layout of the one-lane decode (nodes in
// pool order), and out_lb = 0 for every valid node so that a scan split over
// several workgroups can combine by atomic max; FSP_LB_INVALID otherwise.
// One block of 256 threads per 256 / L nodes; Npad is a multiple of 128;
// n <= 256 (the slot rows' LDS); MV is a multiple of L (machines past m have
// zero times).

// LDS bytes of decode16_lanes_kernel outside the slot rows (L lanes per node,
// 256 / L nodes per block).
__host__ __device__ inline int lanes_lds_rest(int n, int MV, int L)
{
    return ((n + 1) * MV + n * (MV / 2) + (256 / L) * (((n + 31) >> 5) + 2)) * 4;
}

// Words per slot row: L words of padding before the prefix, the n entries,
// and room for the pipeline's reads past the deepest prefix (L + 6 words),
// rounded up to 4; one more 16-byte unit when that makes the row an odd
// number of them, which puts the nodes of a half-wave (read by their lanes at
// consecutive words) on different LDS banks, but only while two blocks still
// fit a compute unit.
__host__ __device__ inline int lanes_slot_row(int n, int MV, int L)
{
    const int r = (L + n + L + 6 + 3) & ~3;
    const int rc = ((r >> 2) & 1) ? r : r + 4;
    return (256 / L) * rc * 4 + lanes_lds_rest(n, MV, L) <= 80 * 1024 ? rc : r;
}

template <int MV, int L>
__global__ __launch_bounds__(256) void decode16_lanes_kernel(DevTables T, const int32_t *__restrict__ prefixes,
                                                             const int32_t *__restrict__ depths, int64_t N,
                                                             Workspace16 W, int32_t *__restrict__ out_lb)
{
    static_assert(L == 4 || L == 8, "four or eight lanes per node");
    static_assert(MV % L == 0, "whole machines per lane");
    constexpr int NB = 256 / L;  // nodes per block
    constexpr int MQ = MV / L;   // machines per lane
    constexpr int H = MV / 2;    // packed tail pairs per job
    constexpr int PADB = L;      // slot words before the prefix
    extern __shared__ uint32_t sm[];
    const int n = T.n, m = T.m, NW = (n + 31) >> 5, RS = lanes_slot_row(n, MV, L);
    int32_t *slots = reinterpret_cast<int32_t *>(sm);  // NB nodes x RS: padding, prefix entries, padding
    int32_t *pl = slots + NB * RS;                     // (n + 1) x MV times; row n is zero
    uint32_t *tq = reinterpret_cast<uint32_t *>(pl + (n + 1) * MV);  // n x H packed tails
    uint32_t *bits = tq + n * H;                       // NB nodes x NW scheduled-job words
    int32_t *sdep = reinterpret_cast<int32_t *>(bits + NB * NW);  // NB depths (0 for an invalid node)
    int32_t *sbad = sdep + NB;                                    // NB flags: a job out of range
    const int tid = threadIdx.x, q = tid & (L - 1), nl = tid / L;
    const int zrow = n * MV;  // offset of the zero row in pl
    // Workgroups go to the chip's eight XCDs in turn (linear id mod 8), and
    // the split scan's workgroups of group G land on XCD G mod 8 when the
    // group count is a multiple of 8.  The blocks that decode group G are
    // placed on that XCD too: block b is the (b / 8)-th of XCD b mod 8, so
    // the scan finds the group's workspace in the same L2.
    constexpr int BPG = kGroup / NB;  // blocks per 128-node group
    const int64_t xb = blockIdx.x & 7, kb = blockIdx.x >> 3;
    const int64_t grp = xb + 8 * (kb / BPG);
    const int64_t node0 = grp * kGroup + (kb % BPG) * NB;
    if (grp * kGroup >= N) return;  // a group past the pool (whole block)
    const int64_t node = node0 + nl;
    const bool live = node < N;
    int d;
    bool fused = false;  // rows checked and converted during the staging
    {
        // Every global load of the staging is issued before the first store:
        // the time rows (row n of p32 is zero), the packed tails, the depth
        // and the block's NB prefix rows, which are contiguous in the pool
        // (entry e of the copy is job e mod n of node e / n; the grid never
        // starts a block past the pool's end, so lim >= n).
        constexpr int PP = MV + 1, TP = H;  // (n + 1) * MV <= 256 * PP, n * H <= 256 * TP
        const int cp = (n + 1) * MV, ct = n * H;
        int32_t pv[PP];
        uint32_t tv[TP];
#pragma unroll
        for (int k = 0; k < PP; ++k) {
            const int e = min(k * 256 + tid, cp - 1), j = e / MV;
            pv[k] = T.p32[(size_t)j * kMaxMachines + (e - j * MV)];
        }
#pragma unroll
        for (int k = 0; k < TP; ++k) {
            const int e = min(k * 256 + tid, ct - 1), j = e / H;
            tv[k] = T.tails16[(size_t)j * (kMaxMachines / 2) + (e - j * H)];
        }
        d = live ? depths[node] : 0;
        const int lim = (int)max<int64_t>(0, min<int64_t>(NB, N - node0)) * n;
        const int32_t *src = prefixes + node0 * (int64_t)n;
        fused = lim > 0 && (n & 3) == 0 && ((uintptr_t)src & 15) == 0;
        if (fused) {
            // 16-byte loads (NB n / 4 of them, at most 16 per thread) never
            // cross a row.  The loaded jobs are checked and turned into
            // time-row offsets right here, once every node's depth is in LDS.
            const int4 *s4 = reinterpret_cast<const int4 *>(src);
            const int lim4 = lim >> 2, c4 = NB * n / 4;
            int4 rv[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) rv[k] = s4[min(k * 256 + tid, lim4 - 1)];
#pragma unroll
            for (int k = 0; k < PP; ++k)
                if (k * 256 + tid < cp) pl[k * 256 + tid] = pv[k];
#pragma unroll
            for (int k = 0; k < TP; ++k)
                if (k * 256 + tid < ct) tq[k * 256 + tid] = tv[k];
            for (int e = tid; e < NB * NW; e += 256) bits[e] = 0u;
            if (q == 0) {
                const bool dok = live && d >= 0 && d <= n;
                sdep[nl] = dok ? d : 0;
                sbad[nl] = dok ? 0 : 1;
            }
            __syncthreads();
            // entry w of the block's rows is job w mod n of node w / n
            // (w < 2^16, so the reciprocal product is exact)
            const uint32_t magic = 0xffffffffu / (uint32_t)n + 1u;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int e = k * 256 + tid;
                if (e < c4) {
                    const uint32_t w = 4u * (uint32_t)e;
                    const int r = (int)__umulhi(w, magic), t = (int)w - r * n;
                    const int dr = sdep[r];
                    const int32_t jj[4] = {rv[k].x, rv[k].y, rv[k].z, rv[k].w};
                    int32_t off[4];
                    bool bad = false;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool in = e < lim4 && t + u < dr, good = (unsigned)jj[u] < (unsigned)n;
                        if (in && good) atomicOr(&bits[r * NW + (jj[u] >> 5)], 1u << (jj[u] & 31));
                        bad |= in && !good;
                        off[u] = in && good ? jj[u] * MV : zrow;
                    }
                    if (bad) sbad[r] = 1;
                    *reinterpret_cast<int4 *>(slots + r * RS + PADB + t) = int4{off[0], off[1], off[2], off[3]};
                }
            }
        } else if (lim > 0) {
            stage_lds_with<16, int32_t>(
                NB * n,
                [&](int e) {
                    const int32_t v = src[min(e, lim - 1)];
                    return e < lim ? v : 0;
                },
                [&](int e, int32_t v) {
                    const int r = e / n;
                    slots[r * RS + PADB + (e - r * n)] = v;
                });
        }
        if (!fused) {
#pragma unroll
            for (int k = 0; k < PP; ++k)
                if (k * 256 + tid < cp) pl[k * 256 + tid] = pv[k];
#pragma unroll
            for (int k = 0; k < TP; ++k)
                if (k * 256 + tid < ct) tq[k * 256 + tid] = tv[k];
            for (int e = tid; e < NB * NW; e += 256) bits[e] = 0u;
        }
    }
    __syncthreads();

    bool ok = live && d >= 0 && d <= n;
    if (!ok) d = 0;
    int32_t *myslot = slots + nl * RS;
    uint32_t *mybits = bits + nl * NW;

    // the padding takes the zero row
    if (q == 0) {
#pragma unroll
        for (int t = 0; t < PADB; ++t) myslot[t] = zrow;
    }
    for (int t = PADB + n + q; t < RS; t += L) myslot[t] = zrow;
    if (fused) {
        ok = ok && !sbad[nl];
    } else {
        // range checks, scheduled bits and time-row offsets, the prefix
        // split over the node's lanes
        for (int t = q; t < n; t += 4 * L) {
            int32_t raw[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) raw[u] = myslot[PADB + min(t + L * u, n - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tt = t + L * u;
                if (tt < n) {
                    const bool in = tt < d, good = (unsigned)raw[u] < (unsigned)n;
                    if (in && good) atomicOr(&mybits[raw[u] >> 5], 1u << (raw[u] & 31));
                    if (in && !good) ok = false;
                    myslot[PADB + tt] = in && good ? raw[u] * MV : zrow;
                }
            }
        }
    }
    __syncthreads();

    int32_t C[MQ], S[MQ];
#pragma unroll
    for (int kk = 0; kk < MQ; ++kk) { C[kk] = 0; S[kk] = 0; }
    // wave-uniform step count: the deepest prefix of the wave plus the pipeline fill
    int smax = d + L - 1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) smax = max(smax, __shfl_xor(smax, off));

    // step s of lane q takes entry s - q: base[s] (base[0] is padding for
    // q > 0).  Rings of four registers, indexed by the step modulo 4 in a loop
    // unrolled four times: offsets read four steps ahead, rows two steps ahead.
    const int32_t *base = myslot + PADB - q;
    const int lq = q * MQ;  // this lane's first machine in a time row
    int32_t xr[4][MQ], o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = base[k];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int kk = 0; kk < MQ; ++kk) xr[k][kk] = pl[o[k] + lq + kk];
    int32_t last = 0;  // completion on this lane's last machine of its previous job
    // a multiple of four steps: a step past the prefix reads the zero row
    for (int s4 = 0; s4 < smax; s4 += 4) {
        const int32_t *b4 = base + s4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int a2 = o[(c + 2) & 3] + lq;  // step s + 2, read two steps ago
            o[c] = b4[c + 4];                    // step s + 4
#pragma unroll
            for (int kk = 0; kk < MQ; ++kk) xr[(c + 2) & 3][kk] = pl[a2 + kk];
            // completion on the machine before this lane's first, for this job
            const int32_t fromleft = __builtin_amdgcn_mov_dpp(last, 0x111, 0xf, 0xf, true);  // row_shr:1
            int32_t prev = q == 0 ? 0 : fromleft;
#pragma unroll
            for (int kk = 0; kk < MQ; ++kk) {
                const int32_t ck = max(C[kk], prev) + xr[c][kk];
                C[kk] = ck;
                prev = ck;
                S[kk] += xr[c][kk];
            }
            last = prev;
        }
    }
    __syncthreads();

    // a repeated job shows as fewer scheduled bits than the depth; every lane
    // of the quad sees the same bits, and the range checks are combined
    int nset = 0;
    for (int w = 0; w < NW; ++w) nset += __popc(mybits[w]);
    int bad = !ok;
    bad |= __builtin_amdgcn_mov_dpp(bad, 0xb1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
    bad |= __builtin_amdgcn_mov_dpp(bad, 0x4e, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
    if constexpr (L == 8) bad |= __shfl_xor(bad, 4);
    ok = !bad && live && nset == d;

    // tails: lane q takes jobs j = 32w + q + L i, minima over (Q | off) as
    // packed halves (three-operand, two jobs each) when every tail is at most
    // kTailsHalfMax, else as packed 16-bit integers; the partial minima of a
    // node's lanes are below 0x8000 in the first case, so the 16-bit
    // reduction across lanes serves both
    const bool halves = T.tails16ok == 2;
    uint32_t q2[H];
    h16x2 qh[H];
#pragma unroll
    for (int c = 0; c < H; ++c) {
        q2[c] = 0xffffffffu;
        qh[c] = as_h16(kHalfNone);
    }
    for (int w = 0; w < NW; ++w) {
        const int lo = w * 32;
        const uint32_t valid = n >= lo + 32 ? 0xffffffffu : ((1u << (n - lo)) - 1u);
        const uint32_t un = ~mybits[w] & valid;
        // four jobs per pass, their rows read before their minima; a job past
        // n reads row n - 1 with every half masked off
        for (int b = q; b < 32 && lo + b < n; b += 4 * L) {
            uint32_t off[4], r[4][H];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int bb = b + L * u;
                const bool in = bb < 32 && lo + bb < n;
                off[u] = in ? ~(uint32_t)__builtin_amdgcn_sbfe((int32_t)un, bb, 1) : 0xffffffffu;
                const uint32_t *tr = tq + min(lo + bb, n - 1) * H;
#pragma unroll
                for (int c = 0; c < H; ++c) r[u][c] = tr[c];
            }
            if (halves) {
#pragma unroll
                for (int u = 0; u < 4; u += 2)
#pragma unroll
                    for (int c = 0; c < H; ++c)
                        qh[c] = __builtin_elementwise_minimum(
                            __builtin_elementwise_minimum(qh[c], as_h16((r[u][c] & ~off[u]) | (kHalfNone & off[u]))),
                            as_h16((r[u + 1][c] & ~off[u + 1]) | (kHalfNone & off[u + 1])));
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < H; ++c)
                        q2[c] = as32(__builtin_elementwise_min(as16(q2[c]), as16(r[u][c] | off[u])));
            }
        }
    }
    if (halves) {
#pragma unroll
        for (int c = 0; c < H; ++c) q2[c] = __builtin_bit_cast(uint32_t, qh[c]);
    }
#pragma unroll
    for (int c = 0; c < H; ++c) {
        q2[c] = as32(__builtin_elementwise_min(as16(q2[c]),
                                               as16((uint32_t)__builtin_amdgcn_mov_dpp((int)q2[c], 0xb1, 0xf, 0xf,
                                                                                      false))));  // [1,0,3,2]
        q2[c] = as32(__builtin_elementwise_min(as16(q2[c]),
                                               as16((uint32_t)__builtin_amdgcn_mov_dpp((int)q2[c], 0x4e, 0xf, 0xf,
                                                                                      false))));  // [2,3,0,1]
        if constexpr (L == 8)
            q2[c] = as32(__builtin_elementwise_min(as16(q2[c]), as16((uint32_t)__shfl_xor((int)q2[c], 4))));
    }

    const bool empty = d == n;  // no unscheduled job: every tail is 0
    const int64_t G = node >> 7;
    const int g = (int)(node & 127), lane = g & 63, half = g >> 6;
    uint16_t *d16 = reinterpret_cast<uint16_t *>(W.dec);
    cptr<int32_t> cs = as_const(T.colsum32);
#pragma unroll
    for (int kk = 0; kk < MQ; ++kk) {
        const int k = q * MQ + kk;
        if (k < m) {
            const uint32_t qk = (q2[k >> 1] >> (16 * (k & 1))) & 0xffffu;
            d16[((G * 3 + 0) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? C[kk] : 0);
            d16[((G * 3 + 1) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok ? C[kk] + (cs[k] - S[kk]) : 0);
            d16[((G * 3 + 2) * m + k) * 128 + lane * 2 + half] = (uint16_t)(ok && !empty ? qk : 0u);
        }
    }
    for (int w = q; w < NW; w += L) {
        const int lo = w * 32;
        const uint32_t valid = n >= lo + 32 ? 0xffffffffu : ((1u << (n - lo)) - 1u);
        W.flg[(G * NW + w) * 128 + g] = ok ? (~mybits[w] & valid) : 0u;
    }
    if (q == 0) {
        W.st[node] = ok ? 1u : 0u;
        if (live) {
            out_lb[node] = ok ? 0 : FSP_LB_INVALID;
            if (!ok) atomicAdd(T.bad, 1ull);
        }
    }
}

// LDS bytes of decode16_lanes_kernel for n jobs and MV machine slots.
inline size_t decode16_lanes_lds(int n, int MV, int L)
{
    return (size_t)lanes_lds_rest(n, MV, L) + (size_t)(256 / L) * lanes_slot_row(n, MV, L) * 4;
}

// How a pool is decoded and scanned.  Below one serial-decode wave per SIMD
// the one-lane decode is latency-bound, so smaller pools take the four-lane
// decode (nodes in pool order, no depth sort); a pool of fewer
// groups than two per compute unit also splits each group's machine pairs
// over several workgroups (at least four pairs per split, about one per
// wave), which needs zeroed bounds from the decode.  Pools on the one-lane
// decode split too, up to the workgroups that fit the LDS at once.
struct PoolPlan {
    bool lanes;          // several lanes per node in the decode
    int splits;          // pair splits of the scan
    int lanes_per_node;  // 4 or 8
};


constexpr int kLanesMaxJobs = 256;  // the four-lane decode stages 64 prefix rows in LDS

static int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
            cus = c;
        else
            cus = 256;
    }
    return cus;
}

static int64_t device_lds_per_cu()
{
    static int64_t bytes = 0;
    if (bytes == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
            v > 0)
            bytes = v;
        else
            bytes = 160 * 1024;
    }
    return bytes;
}

// Pair splits of the scan for G groups: doubled while the workgroups stay
// under `fill` per compute unit (default two) and each split keeps at least
// four pairs.
static int split_count(const fsp_instance_s *I, int64_t G, int fill = 0)
{
    const int cus = device_cus();
    int cap = 16;
    if (const char *e = getenv("FSPBB_SMALL_SPLITS")) cap = atoi(e);  // 0 or 1: no splits
    int minp = 4;  // least pairs per split
    if (fill <= 0) {
        fill = 2;
        if (const char *e = getenv("FSPBB_SPLIT_FILL")) fill = std::max(1, atoi(e));
    }
    if (const char *e = getenv("FSPBB_SPLIT_MIN_PAIRS")) minp = std::max(1, atoi(e));
    int sp = 1;
    while (sp < cap && G * sp < (int64_t)fill * cus && minp * 2 * sp <= I->P) sp *= 2;
    return sp;
}

int scan_splits_for(const fsp_instance_s *I, int64_t N)
{
    if (N <= 0) return 1;
    return split_count(I, (N + kGroup - 1) / kGroup);
}

static PoolPlan pool_plan(const fsp_instance_s *I, int64_t N, int64_t G)
{
    const int cus = device_cus();
    int cap = 16;
    if (const char *e = getenv("FSPBB_SMALL_SPLITS")) cap = atoi(e);  // 0 or 1: the regular path only
    int64_t lanes_below = (int64_t)cus * 4 * 64;                      // one one-lane wave per SIMD
    if (const char *e = getenv("FSPBB_LANES_BELOW")) lanes_below = atoll(e);
    if (I->dt.heads || cap <= 1) return PoolPlan{false, 1, 4};
    if (N >= lanes_below || I->n > kLanesMaxJobs) {
        // the one-lane decode.  When a group's scan is long (n·P of at
        // least 9,000 job-pair slots), its pairs split while the workgroups
        // stay under as many per compute unit as fit its LDS (one group's
        // mask rows, (n + 1) x 256 bytes), at most three.  Measured:
        //   - 500x20, 8,192 nodes: 187 us at four splits, about 295 unsplit;
        //   - 200x20 and 200x10, 65,536 nodes: 3-6% faster at two;
        //   - shorter scans (50x10, 100x10, 20x20, 20x5) are 2-9% slower
        //     split, and so are more workgroups than fit at once (500x20,
        //     32,768 nodes: 385 us at four splits against 334 unsplit).
        const int64_t fit = device_lds_per_cu() / ((int64_t)(I->n + 1) * 256);
        int fill1 = (int)std::min<int64_t>(3, std::max<int64_t>(1, fit));
        bool split = (int64_t)I->n * I->P >= 9000;
        if (const char *e = getenv("FSPBB_ONE_LANE_FILL")) {
            fill1 = std::max(1, atoi(e));
            split = true;
        }
        return PoolPlan{false, split ? split_count(I, G, fill1) : 1, 4};
    }
    const int sp = split_count(I, G);
    // eight lanes per node while their blocks (32 nodes each) do not
    // outnumber the compute units; four above (measured at 200x20: 24 against
    // 30 us at 4,096 nodes, equal at 16,384, slower at 32,768)
    int lpn = N <= (int64_t)32 * cus ? 8 : 4;
    if (const char *e = getenv("FSPBB_LANES_PER_NODE")) lpn = atoi(e) == 8 ? 8 : 4;
    return PoolPlan{true, sp, lpn};
}

// ---- batched bounding: many pools in one decode launch per machine-count
// class and one persistent scan launch fed by a device work queue.

// Copies a struct from a wave-uniform address with scalar loads.
template <class S>
__device__ __forceinline__ S load_uniform(const S *p)
{
    static_assert(sizeof(S) % 4 == 0, "dword-sized struct");
    S out;
    uint32_t *o = reinterpret_cast<uint32_t *>(&out);
    cptr<uint32_t> q = as_const(reinterpret_cast<const uint32_t *>(p));
#pragma unroll
    for (int w = 0; w < (int)(sizeof(S) / 4); ++w) o[w] = q[w];
    return out;
}

// Index of the last pool whose first block is <= blockIdx.x (off has npools + 1 entries).
__device__ __forceinline__ int pool_of_block(const int64_t *blk_off, int npools)
{
    cptr<int64_t> off = as_const(blk_off);
    int lo = 0, hi = npools - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void batch_depth_count_kernel(const BatchPool *__restrict__ pools,
                                                                const int64_t *__restrict__ blk_off,
                                                                const int32_t *__restrict__ sort_pools, int nsort)
{
    extern __shared__ uint32_t h[];
    const int q = pool_of_block(blk_off, nsort);
    const BatchPool P = load_uniform(pools + as_const(sort_pools)[q]);
    depth_count_block(P.depths, P.N, P.T.n, P.sort_chunk, P.sortB, P.W.cnt,
                      (int64_t)blockIdx.x - as_const(blk_off)[q], h);
}

__global__ __launch_bounds__(256) void batch_depth_scatter_kernel(const BatchPool *__restrict__ pools,
                                                                  const int64_t *__restrict__ blk_off,
                                                                  const int32_t *__restrict__ sort_pools, int nsort)
{
    extern __shared__ uint32_t sh[];
    const int q = pool_of_block(blk_off, nsort);
    const BatchPool P = load_uniform(pools + as_const(sort_pools)[q]);
    depth_scatter_block(P.depths, P.N, P.T.n, P.sort_chunk, P.sortB, P.W.cnt, P.W.order,
                        (int64_t)blockIdx.x - as_const(blk_off)[q], sh);
}

hipError_t launch_batch_depth_sort(const BatchPool *pools, const int64_t *blk_off, const int32_t *sort_pools,
                                   int nsort, int64_t nblocks, int nmax, hipStream_t s)
{
    if (nsort <= 0 || nblocks <= 0) return hipSuccess;
    const size_t hb = (size_t)(nmax + 2) * 4, sb = ((size_t)(nmax + 2) * 2 + 256) * 4;
    batch_depth_count_kernel<<<(unsigned)nblocks, 256, hb, s>>>(pools, blk_off, sort_pools, nsort);
    batch_depth_scatter_kernel<<<(unsigned)nblocks, 256, sb, s>>>(pools, blk_off, sort_pools, nsort);
    return hipGetLastError();
}

template <int MV>
__global__ __launch_bounds__(256) void batch_decode16_kernel(const BatchPool *__restrict__ pools,
                                                             const int64_t *__restrict__ blk_off,
                                                             const int32_t *__restrict__ cls_pools, int ncls)
{
    extern __shared__ uint32_t sm[];
    const int q = pool_of_block(blk_off, ncls);
    const BatchPool P = load_uniform(pools + as_const(cls_pools)[q]);
    decode16_block<MV>(P.T, P.prefixes, P.depths, P.N, P.Npad, P.W, P.out_lb,
                       (int64_t)blockIdx.x - as_const(blk_off)[q], sm);
}

// One work item of a batched scan: the masks of up to 16 / wpg groups of one
// pool are staged in LDS; wpg waves scan the machine pairs of each group (two
// chains per wave), then one wave per group takes the maximum over its waves.
// Every thread of the workgroup calls it; it ends with the workgroup past the
// reduction, LDS free for the next item.  before_reduce runs on thread 0 just
// before the final reduction (it may start a memory operation whose result is
// read after the item).
template <int UNR, class F>
__device__ inline void batch_scan_item(const BatchPool *__restrict__ pools, const WorkItem *__restrict__ items,
                                       int it, uint32_t *lds, uint32_t lds0, int lane, int wave, F before_reduce)
{
    const WorkItem wi = load_uniform(items + it);
    const BatchPool P = load_uniform(pools + wi.pool);
    const int n = P.T.n, m = P.T.m, NW = (n + 31) >> 5, np1 = n + 1;
    const int wpg = P.wpg;
    for (int r = wave; r < wi.ngroups * np1; r += kBatchWaves) {
        const int gi = r / np1, j = r - gi * np1;
        uint32_t m2 = 0;
        if (j < n) {
            const uint32_t *fw = P.W.flg + ((int64_t)(wi.group0 + gi) * NW + (j >> 5)) * 128;
            const uint32_t a = (fw[lane] >> (j & 31)) & 1u, b = (fw[64 + lane] >> (j & 31)) & 1u;
            m2 = (a ? 0x0000ffffu : 0u) | (b ? 0xffff0000u : 0u);
        }
        lds[(gi * np1 + j) * 64 + lane] = m2;
    }
    __syncthreads();
    const int gi = wave / wpg, sw = wave - gi * wpg;
    u16x2 lb = {0, 0};
    if (gi < wi.ngroups) {
        const int64_t G = wi.group0 + gi;
        const uint32_t gbase = lds0 + (uint32_t)(gi * np1) * 256u;
        const unsigned char *lds_lane =
            reinterpret_cast<const unsigned char *>(lds) + (size_t)gi * np1 * 256 + lane * 4;
        const uint32_t *dR = P.W.dec + (G * 3 + 0) * m * 64 + lane;
        const uint32_t *dT = dR + m * 64;
        const uint32_t *dQ = dT + m * 64;
        cptr<int32_t> pairs = as_const(P.T.pairs);
        int pr = sw;
        for (; pr + wpg < P.T.P; pr += 2 * wpg) {
            int prs[2] = {pr, pr + wpg};
            u16x2 sv[2];
            uint32_t tk[2], ql[2];
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                const int k = pairs[2 * prs[ch]], l = pairs[2 * prs[ch] + 1];
                sv[ch] = as16(dR[l * 64]) - as16(dR[k * 64]);
                tk[ch] = dT[k * 64];
                ql[ch] = dQ[l * 64];
            }
            scan_pairs<UNR, 2, true>(P.T, prs, sv, lds_lane, gbase);
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) lb = __builtin_elementwise_max(lb, as16(tk[ch]) + sv[ch] + as16(ql[ch]));
        }
        for (; pr < P.T.P; pr += wpg) {
            const int prs[1] = {pr};
            const int k = pairs[2 * pr], l = pairs[2 * pr + 1];
            u16x2 sv[1] = {as16(dR[l * 64]) - as16(dR[k * 64])};
            const uint32_t tk = dT[k * 64], ql = dQ[l * 64];
            scan_pairs<UNR, 1, true>(P.T, prs, sv, lds_lane, gbase);
            lb = __builtin_elementwise_max(lb, as16(tk) + sv[0] + as16(ql));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) before_reduce();
    lds[wave * 64 + lane] = as32(lb);
    __syncthreads();
    if (wave < wi.ngroups) {
        const int64_t G = wi.group0 + wave;
        u16x2 best = as16(lds[(wave * wpg) * 64 + lane]);
        for (int w = 1; w < wpg; ++w) best = __builtin_elementwise_max(best, as16(lds[(wave * wpg + w) * 64 + lane]));
        const int64_t a = G * 128 + lane, b = a + 64;
        if (a < P.N && P.W.st[a]) P.out_lb[P.W.order ? P.W.order[a] : a] = (int32_t)best.x;
        if (b < P.N && P.W.st[b]) P.out_lb[P.W.order ? P.W.order[b] : b] = (int32_t)best.y;
    }
    __syncthreads();
}

// Persistent scan: gridDim.x workgroups; workgroup b takes item b, then items
// from a device counter (offset by the grid) until none is left.  The next
// index is fetched during the current item's reduction.
template <int UNR>
__global__ __launch_bounds__(64 * kBatchWaves) void batch_scan16_kernel(const BatchPool *__restrict__ pools,
                                                                       const WorkItem *__restrict__ items,
                                                                       int n_items, uint32_t *__restrict__ counter)
{
    extern __shared__ uint32_t lds[];
    __shared__ int s_next;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lds0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t *)lds);
    int it = blockIdx.x;
    while (it < n_items) {  // uniform: every wave leaves together (the counter only grows)
        batch_scan_item<UNR>(pools, items, it, lds, lds0, lane, wave,
                             [&]() { s_next = (int)gridDim.x + (int)atomicAdd(counter, 1u); });
        it = __builtin_amdgcn_readfirstlane(s_next);
    }
}

// One workgroup per work item (the hardware dispatches them in item order,
// longest first).
template <int UNR>
__global__ __launch_bounds__(64 * kBatchWaves) void batch_scan16_grid_kernel(const BatchPool *__restrict__ pools,
                                                                            const WorkItem *__restrict__ items)
{
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lds0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint32_t *)lds);
    batch_scan_item<UNR>(pools, items, (int)blockIdx.x, lds, lds0, lane, wave, []() {});
}

hipError_t launch_batch_decode(int MV, const BatchPool *pools, const int64_t *blk_off, const int32_t *cls_pools,
                               int ncls, int64_t nblocks, size_t lds_bytes, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks), block(256);
#define FSP_BDECODE(MVV) \
    case MVV: batch_decode16_kernel<MVV><<<grid, block, lds_bytes, s>>>(pools, blk_off, cls_pools, ncls); break;
    switch (MV) {
        FSP_BDECODE(4) FSP_BDECODE(8) FSP_BDECODE(12) FSP_BDECODE(16)
        FSP_BDECODE(20) FSP_BDECODE(24) FSP_BDECODE(28) FSP_BDECODE(32)
    default: return hipErrorInvalidValue;
    }
#undef FSP_BDECODE
    return hipGetLastError();
}

__global__ void batch_reset_kernel(uint32_t *counter) { *counter = 0u; }

hipError_t launch_batch_scan(const BatchPool *pools, const WorkItem *items, int n_items, uint32_t *counter,
                             int grid, size_t lds_bytes, int form, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (form == kBatchGrid) {
        batch_scan16_grid_kernel<8><<<n_items, 64 * kBatchWaves, lds_bytes, s>>>(pools, items);
    } else {
        batch_reset_kernel<<<1, 1, 0, s>>>(counter);
        batch_scan16_kernel<8><<<grid, 64 * kBatchWaves, lds_bytes, s>>>(pools, items, n_items, counter);
    }
    return hipGetLastError();
}


int batch_scan_blocks_per_cu(size_t lds_bytes)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_scan16_kernel<8>, 64 * kBatchWaves, lds_bytes) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

namespace {
// Section sizes of the 16-bit workspace for N nodes, each rounded up to 256 bytes.
struct PackedWsLayout {
    size_t dec, flg, st, ord, cnt;
    size_t total() const { return dec + flg + st + ord + cnt; }
};

PackedWsLayout packed_ws_layout(const fsp_instance_s *I, int64_t N)
{
    const int n = I->n, m = I->m, NW = (n + 31) >> 5;
    const int64_t G = (N + kGroup - 1) / kGroup, Npad = G * kGroup;
    const int B = (int)std::min<int64_t>(kSortMaxBlocks, (N + 4095) / 4096);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return PackedWsLayout{al((size_t)G * 3 * m * 64 * 4), al((size_t)G * NW * 128 * 4), al((size_t)Npad * 4),
                          al((size_t)N * 4), al((size_t)(n + 2) * B * 4)};
}
}  // namespace

size_t packed_workspace_bytes(const fsp_instance_s *I, int64_t N)
{
    return N > 0 ? packed_ws_layout(I, N).total() : 0;
}

hipError_t launch_bound_packed_ws(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths, int64_t N,
                                  int32_t *out_lb, hipStream_t s, bool sort_depths, void *ws, bool marks)
{
    if (N <= 0) return hipSuccess;
    const int n = I->n, m = I->m;
    const int64_t G = (N + kGroup - 1) / kGroup, Npad = G * kGroup;
    const int B = (int)std::min<int64_t>(kSortMaxBlocks, (N + 4095) / 4096);
    const int64_t chunk = (N + B - 1) / B;
    const PackedWsLayout L = packed_ws_layout(I, N);
    // every section is written in full before it is read (the count kernel
    // writes all n + 2 buckets of its block, the decode every node slot of
    // the padded pool), so the workspace needs no clearing
    char *w = (char *)ws;
    Workspace16 W;
    W.dec = (uint32_t *)w;
    W.flg = (uint32_t *)(w + L.dec);
    W.st = (uint32_t *)(w + L.dec + L.flg);
    W.order = sort_depths ? (int32_t *)(w + L.dec + L.flg + L.st) : nullptr;
    W.cnt = (uint32_t *)(w + L.dec + L.flg + L.st + L.ord);

    const int MV = (m + 3) & ~3;
    const PoolPlan plan = pool_plan(I, N, G);
    if (plan.lanes) {
        // L lanes per node in pool order, then the pairs of each group, split
        // over several workgroups when the groups are few
        W.order = nullptr;
        if (marks) timing_mark(I, 0, s);
        const int L = plan.lanes_per_node, MVL = (m + L - 1) / L * L;
        // blocks for every group, rounded up to whole rounds of 8 XCDs
        const int64_t bpg = kGroup / (256 / L), nblk = (G + 7) / 8 * 8 * bpg;
        const dim3 lgrid((unsigned)nblk);
        const size_t llds = decode16_lanes_lds(n, MVL, L);
#define FSP_LDECODE(MVV, LL) \
    case MVV: decode16_lanes_kernel<MVV, LL><<<lgrid, 256, llds, s>>>(I->dt, prefixes, depths, N, W, out_lb); break;
        if (L == 8) {
            switch (MVL) { FSP_LDECODE(8, 8) FSP_LDECODE(16, 8) FSP_LDECODE(24, 8) FSP_LDECODE(32, 8) }
        } else {
            switch (MVL) {
                FSP_LDECODE(4, 4) FSP_LDECODE(8, 4) FSP_LDECODE(12, 4) FSP_LDECODE(16, 4)
                FSP_LDECODE(20, 4) FSP_LDECODE(24, 4) FSP_LDECODE(28, 4) FSP_LDECODE(32, 4)
            }
        }
#undef FSP_LDECODE
        hipError_t e = hipGetLastError();
        if (marks) timing_mark(I, 1, s);
        if (e == hipSuccess) e = launch_scan16(I, W, N, out_lb, s, plan.splits);
        if (marks) timing_mark(I, 2, s);
        return e;
    }

    if (marks) timing_mark(I, 0, s);
    if (sort_depths) launch_depth_sort(depths, N, n, B, chunk, W.cnt, W.order, s);

    const size_t dlds = decode16_lds_words(n, MV) * 4;
    const int zero_lb = plan.splits > 1 ? 1 : 0;
    // decode of sorted positions [0, Np) of a part whose workspace starts at W
    auto decode = [&](const Workspace16 &Wp, int64_t Np, int64_t Nppad, hipStream_t st) {
        const dim3 dgrid((unsigned)((Nppad + 255) / 256)), dblock(256);
#define FSP_DECODE(MVV) \
    case MVV: \
        bound_decode16_kernel<MVV><<<dgrid, dblock, dlds, st>>>(I->dt, prefixes, depths, Np, Nppad, Wp, out_lb, zero_lb); \
        break;
        switch (MV) {
            FSP_DECODE(4) FSP_DECODE(8) FSP_DECODE(12) FSP_DECODE(16)
            FSP_DECODE(20) FSP_DECODE(24) FSP_DECODE(28) FSP_DECODE(32)
        }
#undef FSP_DECODE
        return hipGetLastError();
    };
    hipError_t e = decode(W, N, Npad, s);
    if (marks) timing_mark(I, 1, s);
    if (e == hipSuccess) e = launch_scan16(I, W, N, out_lb, s, plan.splits);
    if (marks) timing_mark(I, 2, s);
    return e;
}

hipError_t launch_bound_packed(fsp_instance_s *I, const int32_t *prefixes, const int32_t *depths,
                               int64_t N, int32_t *out_lb, hipStream_t s, bool sort_depths)
{
    if (N <= 0) return hipSuccess;
    void *ws = nullptr;
    hipError_t e = stream_alloc(&ws, packed_workspace_bytes(I, N), s);
    if (e != hipSuccess) return e;
    e = launch_bound_packed_ws(I, prefixes, depths, N, out_lb, s, sort_depths, ws, true);
    hipError_t e2 = stream_free(ws, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace fspbb
