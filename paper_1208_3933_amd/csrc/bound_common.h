// Per-node decode shared by the bound kernels: the scheduled set, the machine
// releases (RM of Table I), the sums that close each pair scan, and the tails
// (QM of Table I).
#pragma once

#include "fspbb_internal.h"

namespace fspbb {

template <int W> using u32v = uint32_t __attribute__((ext_vector_type(W)));
template <int W> using i32v = int32_t __attribute__((ext_vector_type(W)));

// Wave-uniform reads of instance tables go through the constant address space
// so the compiler emits scalar loads (the tables are never written by a kernel).
template <class T>
using cptr = const __attribute__((address_space(4))) T *;
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T *p)
{
    return (cptr<T>)p;
}

constexpr int kMaskWords = kMaxJobs / 32;  // 16 words: a register vector the
                                           // compiler indexes with one move

// Result of decoding one node.  For machine k: R[k] is the completion time of
// the scheduled prefix on k (its release; 0 at the root), Tk[k] = R[k] plus
// the time of all unscheduled jobs on k (the value timeOnM1 reaches at the end
// of any pair scan of Fig. 2 that starts on k), Qv[k] the tail of k: the least,
// over unscheduled jobs, of their total time on the machines after k (0 when
// no job is left).  act holds one bit per unscheduled job.
template <int MV>
struct Decoded {
    int32_t R[MV], Tk[MV], Qv[MV];
    u32v<kMaskWords> act;
    bool ok;
};

// Decodes the node whose prefix is row[0..d-1] (one lane, one node).  MV is a
// compile-time bound on m (multiple of 4).  bits is this lane's column of a
// 16-word LDS scratch mask, word w at bits[w * stride]; it is used to build the
// scheduled set with LDS atomics and to detect repeated jobs.
template <int MV>
__device__ inline void decode_node(const DevTables &T, const int32_t *__restrict__ row, int d,
                                   uint32_t *bits, int stride, Decoded<MV> &out)
{
    const int n = T.n, m = T.m;
    bool ok = (d >= 0 && d <= n);
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) bits[w * stride] = 0u;
    int32_t C[MV], S[MV];
#pragma unroll
    for (int k = 0; k < MV; ++k) { C[k] = 0; S[k] = 0; }
    if (ok) {
        for (int t = 0; t < d; ++t) {
            const int j = row[t];
            if ((unsigned)j >= (unsigned)n) { ok = false; break; }
            const uint32_t bit = 1u << (j & 31);
            const uint32_t old = atomicOr(&bits[(j >> 5) * stride], bit);
            if (old & bit) { ok = false; break; }
            // one step of the completion-time recurrence (Sec. II-C); the
            // padded columns k >= m only repeat the last value and are unused
            const int4 *pr = reinterpret_cast<const int4 *>(T.p32 + (size_t)j * kMaxMachines);
            int32_t prev = 0;
#pragma unroll
            for (int q = 0; q < MV / 4; ++q) {
                const int4 v = pr[q];
                const int32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int k = 4 * q + c;
                    const int32_t ck = max(C[k], prev) + x[c];
                    C[k] = ck;
                    prev = ck;
                    S[k] += x[c];
                }
            }
        }
    }
    u32v<kMaskWords> act;
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) {
        const int lo = w * 32;
        const uint32_t valid = n >= lo + 32 ? 0xffffffffu : (n <= lo ? 0u : ((1u << (n - lo)) - 1u));
        act[w] = ok ? (~bits[w * stride] & valid) : 0u;
    }
    // heads: with T.heads, each machine's release becomes the earliest start
    // on it of an unscheduled job scheduled next (the job loop is uniform
    // across lanes, so the time rows are scalar loads)
    if (T.heads && ok && d < n) {
        int32_t h[MV];
#pragma unroll
        for (int k = 0; k < MV; ++k) h[k] = 0x7fffffff;
        for (int j = 0; j < n; ++j) {
            const bool a = (act[j >> 5] >> (j & 31)) & 1u;
            cptr<int32_t> pr = as_const(T.p32 + (size_t)j * kMaxMachines);
            int32_t prev = 0;
#pragma unroll
            for (int k = 0; k < MV; ++k) {
                const int32_t start = max(C[k], prev);
                h[k] = a ? min(h[k], start) : h[k];
                prev = start + pr[k];
            }
        }
#pragma unroll
        for (int k = 0; k < MV; ++k) C[k] = h[k];
    }
    // tails: least remaining time after machine l over the unscheduled jobs
    int32_t q[MV];
#pragma unroll
    for (int k = 0; k < MV; ++k) q[k] = 0x7fffffff;
    for (int j = 0; j < n; ++j) {
        const bool a = (act[j >> 5] >> (j & 31)) & 1u;
        cptr<int32_t> qr = as_const(T.tails32 + (size_t)j * kMaxMachines);
#pragma unroll
        for (int k = 0; k < MV; ++k) q[k] = a ? min(q[k], qr[k]) : q[k];
    }
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        const int32_t cs = as_const(T.colsum32)[k];
        out.R[k] = ok ? C[k] : 0;
        out.Tk[k] = ok ? C[k] + (cs - S[k]) : 0;
        out.Qv[k] = (ok && q[k] != 0x7fffffff) ? q[k] : 0;
    }
    (void)m;
    out.act = act;
    out.ok = ok;
}

}  // namespace fspbb
