// Best-first frontier kernels (see best_first.h).  The frontier is kept as
// records sorted by (bound, insertion order), so that
//   - the nodes the upper bound eliminates are a tail (one binary search),
//   - the parents of a step are a prefix (one block scans the children
//     counts until pool_cap is reached),
//   - inserting a step's survivors is a merge of two sorted sequences: each
//     record finds its output position by a binary search in the other one
//     (earlier insertion first on equal bounds).
// Only 12-byte records move; rows stay in their slab slots.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "best_first.h"
#include "fspbb_internal.h"

namespace fspbb {

namespace {

constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(kSelThreads) void bf_select_kernel(const int32_t *__restrict__ lb,
                                                                const int32_t *__restrict__ depth, int64_t M,
                                                                int32_t ub, int n, int64_t pool_cap,
                                                                int64_t *__restrict__ sel)
{
    __shared__ int64_t sh[kSelThreads];
    __shared__ int64_t s_mp;
    const int t = threadIdx.x;
    if (t == 0) {
        int64_t lo = 0, hi = M;  // first record with bound >= ub
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (lb[mid] < ub) lo = mid + 1;
            else hi = mid;
        }
        s_mp = lo;
    }
    __syncthreads();
    const int64_t Mp = s_mp;
    int64_t base = 0, sum = 0, K = 0, nch = 0;
    while (base < Mp) {  // uniform over the block
        const int64_t i = base + t;
        const int64_t c = i < Mp ? (int64_t)(n - depth[i]) : 0;
        sh[t] = c;
        __syncthreads();
        for (int off = 1; off < kSelThreads; off <<= 1) {
            const int64_t a = t >= off ? sh[t - off] : 0;
            __syncthreads();
            sh[t] += a;
            __syncthreads();
        }
        // every record has at least one child, so the running sum grows and
        // the records taken form a prefix
        const bool ok = i < Mp && (i == 0 || sum + sh[t] <= pool_cap);
        const int cnt = __syncthreads_count(ok);
        if (cnt < kSelThreads || base + kSelThreads >= Mp) {
            K = base + cnt;
            nch = cnt > 0 ? sum + sh[cnt - 1] : sum;
            break;
        }
        sum += sh[kSelThreads - 1];
        base += kSelThreads;
        __syncthreads();
    }
    if (t == 0) {
        sel[0] = Mp;
        sel[1] = K;
        sel[2] = nch;
    }
}

__global__ void bf_fill_kernel(int32_t *__restrict__ fl, int64_t count, int32_t first)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) fl[i] = first + (int32_t)i;
}

__global__ void bf_keys_kernel(const int32_t *__restrict__ lb, const uint32_t *__restrict__ nsurv, int64_t cap,
                               int32_t pad, int32_t *__restrict__ keys, int32_t *__restrict__ ranks)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    keys[i] = i < (int64_t)*nsurv ? lb[i] : pad;
    ranks[i] = (int32_t)i;
}

// Number of v[0, len) below x (strict = true) or at most x.
__device__ __forceinline__ int64_t count_before(const int32_t *v, int64_t len, int32_t x, bool strict)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const bool before = strict ? v[mid] < x : v[mid] <= x;
        if (before) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void bf_merge_a_kernel(Frontier F, int64_t a0, int64_t nA, const int32_t *__restrict__ kb,
                                  const uint32_t *__restrict__ nsurv, Frontier G)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nA) return;
    const int32_t v = F.lb[a0 + i];
    const int64_t pos = i + count_before(kb, (int64_t)*nsurv, v, true);
    G.lb[pos] = v;
    G.depth[pos] = F.depth[a0 + i];
    G.slot[pos] = F.slot[a0 + i];
}

__global__ void bf_merge_b_kernel(Frontier F, int64_t a0, int64_t nA, const int32_t *__restrict__ kb,
                                  const int32_t *__restrict__ rk, const int32_t *__restrict__ sdep,
                                  const uint32_t *__restrict__ nsurv, const int32_t *__restrict__ freelist,
                                  int64_t top, Frontier G)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)*nsurv) return;
    const int32_t v = kb[j];
    const int64_t pos = j + count_before(F.lb + a0, nA, v, false);
    const int32_t r = rk[j];
    G.lb[pos] = v;
    G.depth[pos] = sdep[r];
    G.slot[pos] = freelist[top - 1 - r];
}

__global__ void bf_free_kernel(Frontier F, int64_t K, int64_t Mp, int64_t M, int32_t *__restrict__ freelist,
                               int64_t top, const uint32_t *__restrict__ nsurv)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K + (M - Mp)) return;
    const int32_t slot = t < K ? F.slot[t] : F.slot[Mp + (t - K)];
    freelist[top - (int64_t)*nsurv + t] = slot;
}

unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

hipError_t bf_select(const Frontier &F, int64_t M, int32_t ub, int n, int64_t pool_cap, int64_t *sel,
                     hipStream_t s)
{
    bf_select_kernel<<<1, kSelThreads, 0, s>>>(F.lb, F.depth, M, ub, n, pool_cap, sel);
    return hipGetLastError();
}

hipError_t bf_fill_slots(int32_t *freelist, int64_t count, int32_t first, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    bf_fill_kernel<<<blocks256(count), 256, 0, s>>>(freelist, count, first);
    return hipGetLastError();
}

hipError_t bf_sort_survivors(const int32_t *lb, const uint32_t *nsurv, int64_t cap, int32_t ub, int32_t *keys,
                             int32_t *ranks, int32_t *keys_out, int32_t *rank_out, void **tmp, size_t *tmp_bytes,
                             hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    // survivors have bounds below ub: sort on the bits of ub only, with the
    // padding past the survivors at the largest key of that width (>= ub)
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) - 1 < (int64_t)ub) ++bits;
    const int32_t pad = (int32_t)(((int64_t)1 << bits) - 1);
    bf_keys_kernel<<<blocks256(cap), 256, 0, s>>>(lb, nsurv, cap, pad, keys, ranks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // a stable LSD radix sort (onesweep) at every size: the library default
    // below a million items is a merge sort, whose log2(cap / 2048) passes
    // cost about 80 us at 262,144 items against a few passes of 8 bits
    using Cfg = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                           rocprim::default_config, 0>;
    size_t need = 0;
    e = rocprim::radix_sort_pairs<Cfg>(nullptr, need, reinterpret_cast<const uint32_t *>(keys),
                                       reinterpret_cast<uint32_t *>(keys_out), ranks, rank_out, (int64_t)cap, 0u,
                                       (unsigned)bits, s);
    if (e != hipSuccess) return e;
    if (need > *tmp_bytes) {
        if (*tmp) stream_free(*tmp, s);
        *tmp = nullptr;
        *tmp_bytes = 0;
        e = stream_alloc(tmp, need, s);
        if (e != hipSuccess) return e;
        *tmp_bytes = need;
    }
    return rocprim::radix_sort_pairs<Cfg>(*tmp, need, reinterpret_cast<const uint32_t *>(keys),
                                          reinterpret_cast<uint32_t *>(keys_out), ranks, rank_out, (int64_t)cap, 0u,
                                          (unsigned)bits, s);
}

hipError_t bf_merge(const Frontier &F, int64_t a0, int64_t nA, const int32_t *kb, const int32_t *rk,
                    const int32_t *sdep, const uint32_t *nsurv, int64_t cap, const int32_t *freelist, int64_t top,
                    const Frontier &G, hipStream_t s)
{
    if (nA > 0) bf_merge_a_kernel<<<blocks256(nA), 256, 0, s>>>(F, a0, nA, kb, nsurv, G);
    if (cap > 0) bf_merge_b_kernel<<<blocks256(cap), 256, 0, s>>>(F, a0, nA, kb, rk, sdep, nsurv, freelist, top, G);
    return hipGetLastError();
}

hipError_t bf_free_slots(const Frontier &F, int64_t K, int64_t Mp, int64_t M, int32_t *freelist, int64_t top,
                         const uint32_t *nsurv, hipStream_t s)
{
    const int64_t cnt = K + (M - Mp);
    if (cnt <= 0) return hipSuccess;
    bf_free_kernel<<<blocks256(cnt), 256, 0, s>>>(F, K, Mp, M, freelist, top, nsurv);
    return hipGetLastError();
}

}  // namespace fspbb
