// Instance creation: validation, the per-instance tables of Table I and their
// upload to the device (Sec. II-D: lags and Johnson orders are computed once
// per instance, then shared by every bound).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "fspbb_internal.h"

namespace fspbb {

static thread_local char g_last_error[256] = "";

void set_last_error(hipError_t e)
{
    snprintf(g_last_error, sizeof(g_last_error), "%s (%d)", hipGetErrorString(e), (int)e);
}

// Johnson's rule with lags for one pair (Johnson 1954; Mitten 1959): with
// a = p[j][k], b = p[j][l] and lag L, jobs with a <= b first by increasing
// a + L, then jobs with a > b by decreasing b + L.  Ties by job id.  Any
// tie-break gives the same bound; a fixed one keeps the tables reproducible.
static void johnson_with_lags(const int32_t *p, int n, int m, int k, int l, std::vector<int> &order,
                              std::vector<int32_t> &lagv)
{
    lagv.assign(n, 0);
    for (int j = 0; j < n; ++j)
        for (int h = k + 1; h < l; ++h) lagv[j] += p[j * m + h];
    order.resize(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        int32_t ax = p[x * m + k], bx = p[x * m + l], ay = p[y * m + k], by = p[y * m + l];
        bool gx = ax <= bx, gy = ay <= by;
        if (gx != gy) return gx;  // the a <= b group first
        if (gx) {
            int32_t kx = ax + lagv[x], ky = ay + lagv[y];
            if (kx != ky) return kx < ky;
        } else {
            int32_t kx = bx + lagv[x], ky = by + lagv[y];
            if (kx != ky) return kx > ky;
        }
        return x < y;
    });
}

}  // namespace fspbb

using namespace fspbb;

extern "C" {

const char *fsp_status_string(fsp_status s)
{
    switch (s) {
    case FSP_OK: return "FSP_OK";
    case FSP_E_INVAL: return "FSP_E_INVAL: invalid argument";
    case FSP_E_RANGE: return "FSP_E_RANGE: value or size out of range";
    case FSP_E_NOMEM: return "FSP_E_NOMEM: allocation failed";
    case FSP_E_DEVICE: return "FSP_E_DEVICE: HIP runtime error";
    case FSP_E_BADNODE: return "FSP_E_BADNODE: pool held invalid nodes";
    case FSP_E_NODEVICE: return "FSP_E_NODEVICE: no gfx950 device";
    case FSP_BUDGET: return "FSP_BUDGET: node budget reached";
    case FSP_PENDING: return "FSP_PENDING: search not finished";
    default: return "unknown status";
    }
}

const char *fsp_last_error_string(void) { return g_last_error; }

fsp_status fsp_create_instance(const int32_t *p, int32_t n, int32_t m, fsp_instance *out)
{
    return fsp_create_instance_ex(p, n, m, 0, out);
}

namespace {

// Builds an instance whose bound takes the maximum over `prs` (pairs (k,l),
// k < l, lexicographic, no repeats; checked by the callers).
fsp_status create_instance(const int32_t *p, int32_t n, int32_t m, int32_t flags,
                           const std::vector<std::pair<int, int>> &prs, fsp_instance *out)
{
    int64_t pmax = 0;
    for (int64_t i = 0; i < (int64_t)n * m; ++i) {
        if (p[i] < 0) return FSP_E_INVAL;
        pmax = std::max<int64_t>(pmax, p[i]);
    }
    int64_t maxv = (int64_t)(n + m - 1) * pmax;
    if (maxv >= (int64_t)1 << 31) return FSP_E_RANGE;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return FSP_E_NODEVICE;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_last_error(e); return FSP_E_DEVICE; }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) { set_last_error(e); return FSP_E_DEVICE; }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FSP_E_NODEVICE;

    const int P = (int)prs.size();
    const int npad = (n + 3) & ~3;

    // host tables
    constexpr int S = kMaxMachines;  // row stride of the padded device tables
    std::vector<int32_t> hp((size_t)(n + 1) * S, 0), colsum(S, 0), tails((size_t)n * S, 0), pairs(2 * P);
    std::vector<Rec32> rec32((size_t)P * n), rec32sm((size_t)n * P);
    std::vector<Rec16> rec16((size_t)P * npad);
    std::vector<RecW> recw((size_t)P * npad);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < m; ++k) hp[(size_t)j * S + k] = p[j * m + k];
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < m; ++k) colsum[k] += p[j * m + k];
    for (int j = 0; j < n; ++j)
        for (int l = 0; l < m; ++l)
            for (int h = l + 1; h < m; ++h) tails[(size_t)j * S + l] += p[j * m + h];
    std::vector<uint32_t> tails16((size_t)n * (S / 2), 0);
    for (int j = 0; j < n; ++j)
        for (int c = 0; c < S / 2; ++c)
            tails16[(size_t)j * (S / 2) + c] = ((uint32_t)tails[(size_t)j * S + 2 * c] & 0xffffu) |
                                               ((uint32_t)tails[(size_t)j * S + 2 * c + 1] << 16);
    // tord: for rank r and machine l < m, the r-th job by increasing tail on
    // machine l (ties by job) as (job << 16) | tail, the tail's low 16 bits
    std::vector<uint32_t> tord((size_t)n * S, 0);
    {
        std::vector<int> idx(n);
        for (int l = 0; l < m; ++l) {
            for (int j = 0; j < n; ++j) idx[j] = j;
            std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) {
                return tails[(size_t)a * S + l] < tails[(size_t)c * S + l];
            });
            for (int r = 0; r < n; ++r)
                tord[(size_t)r * S + l] = ((uint32_t)idx[r] << 16) | ((uint32_t)tails[(size_t)idx[r] * S + l] & 0xffffu);
        }
    }
    std::vector<int> order;
    std::vector<int32_t> lagv;
    for (int pr = 0; pr < P; ++pr) {
        {
            const int k = prs[pr].first, l = prs[pr].second;
            pairs[2 * pr] = k;
            pairs[2 * pr + 1] = l;
            johnson_with_lags(p, n, m, k, l, order, lagv);
            for (int i = 0; i < npad; ++i) {
                Rec16 r16{(uint32_t)n * 256u, 0u};  // padding: the all-zero mask row
                RecW rw{(uint32_t)n * 256u, 0, 0};
                if (i < n) {
                    int j = order[i];
                    int32_t a = p[j * m + k], b = p[j * m + l];
                    int32_t E = lagv[j] + a, C = b - a;
                    rec32[(size_t)pr * n + i] = Rec32{(uint32_t)(j >> 5), (uint32_t)(j & 31), E, C};
                    rec32sm[(size_t)i * P + pr] = rec32[(size_t)pr * n + i];
                    r16 = Rec16{(uint32_t)j * 256u, ((uint32_t)E << 16) | ((uint32_t)C & 0xffffu)};
                    rw = RecW{(uint32_t)j * 256u, E, C};
                }
                rec16[(size_t)pr * npad + i] = r16;
                recw[(size_t)pr * npad + i] = rw;
            }
        }
    }

    // one device blob
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off_p = 0;
    size_t off_cs = align(off_p + hp.size() * 4);
    size_t off_t = align(off_cs + colsum.size() * 4);
    size_t off_t16 = align(off_t + tails.size() * 4);
    size_t off_pr = align(off_t16 + tails16.size() * 4);
    size_t off_r32 = align(off_pr + pairs.size() * 4);
    size_t off_rsm = align(off_r32 + rec32.size() * sizeof(Rec32));
    size_t off_r16 = align(off_rsm + rec32sm.size() * sizeof(Rec32));
    size_t off_rw = align(off_r16 + rec16.size() * sizeof(Rec16));
    size_t off_to = align(off_rw + recw.size() * sizeof(RecW));
    size_t off_bad = align(off_to + tord.size() * 4);
    size_t total = align(off_bad + sizeof(unsigned long long));
    std::vector<unsigned char> blob(total, 0);
    std::memcpy(blob.data() + off_p, hp.data(), hp.size() * 4);
    std::memcpy(blob.data() + off_cs, colsum.data(), colsum.size() * 4);
    std::memcpy(blob.data() + off_t, tails.data(), tails.size() * 4);
    std::memcpy(blob.data() + off_t16, tails16.data(), tails16.size() * 4);
    std::memcpy(blob.data() + off_pr, pairs.data(), pairs.size() * 4);
    std::memcpy(blob.data() + off_r32, rec32.data(), rec32.size() * sizeof(Rec32));
    std::memcpy(blob.data() + off_rsm, rec32sm.data(), rec32sm.size() * sizeof(Rec32));
    std::memcpy(blob.data() + off_r16, rec16.data(), rec16.size() * sizeof(Rec16));
    std::memcpy(blob.data() + off_rw, recw.data(), recw.size() * sizeof(RecW));
    std::memcpy(blob.data() + off_to, tord.data(), tord.size() * 4);

    void *d = nullptr;
    e = hipMalloc(&d, total);
    if (e != hipSuccess) { set_last_error(e); return FSP_E_NOMEM; }
    e = hipMemcpy(d, blob.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) { set_last_error(e); hipFree(d); return FSP_E_DEVICE; }

    fsp_instance_s *I = new (std::nothrow) fsp_instance_s();
    if (!I) { hipFree(d); return FSP_E_NOMEM; }
    I->n = n; I->m = m; I->P = P;
    I->max_value = (int32_t)maxv;
    I->packed16 = maxv < 65536 ? 1 : 0;
    I->device = dev;
    I->table_bytes = (int64_t)total;
    I->dev_blob = d;
    I->p_host = new int32_t[(size_t)n * m];
    std::memcpy(I->p_host, p, sizeof(int32_t) * (size_t)n * m);
    unsigned char *b = (unsigned char *)d;
    I->flags = flags | (P < m * (m - 1) / 2 ? FSP_INSTANCE_PAIR_SUBSET : 0);
    I->dt.n = n; I->dt.m = m; I->dt.P = P; I->dt.npad = npad;
    I->dt.heads = (flags & FSP_INSTANCE_HEADS) ? 1 : 0;
    {
        const int32_t qmax = *std::max_element(tails.begin(), tails.end());
        I->dt.tails16ok = qmax <= kTailsHalfMax ? 2 : qmax < 65536 ? 1 : 0;
    }
    I->dt.p32 = (const int32_t *)(b + off_p);
    I->dt.colsum32 = (const int32_t *)(b + off_cs);
    I->dt.tails32 = (const int32_t *)(b + off_t);
    I->dt.tails16 = (const uint32_t *)(b + off_t16);
    I->dt.pairs = (const int32_t *)(b + off_pr);
    I->dt.rec32 = (const Rec32 *)(b + off_r32);
    I->dt.rec32sm = (const Rec32 *)(b + off_rsm);
    I->dt.rec16 = (const Rec16 *)(b + off_r16);
    I->dt.recw = (const RecW *)(b + off_rw);
    I->dt.tord = (const uint32_t *)(b + off_to);
    I->dt.bad = (unsigned long long *)(b + off_bad);
    *out = I;
    return FSP_OK;
}

fsp_status check_shape(const int32_t *p, int32_t n, int32_t m, int32_t flags, fsp_instance *out)
{
    if (!out) return FSP_E_INVAL;
    *out = nullptr;
    if (!p || n < 1 || m < 2 || n > kMaxJobs || m > kMaxMachines) return FSP_E_INVAL;
    if (flags & ~FSP_INSTANCE_HEADS) return FSP_E_INVAL;
    return FSP_OK;
}

}  // namespace

fsp_status fsp_create_instance_ex(const int32_t *p, int32_t n, int32_t m, int32_t flags, fsp_instance *out)
{
    fsp_status st = check_shape(p, n, m, flags, out);
    if (st != FSP_OK) return st;
    std::vector<std::pair<int, int>> prs;
    for (int k = 0; k < m; ++k)
        for (int l = k + 1; l < m; ++l) prs.push_back({k, l});
    return create_instance(p, n, m, flags, prs, out);
}

fsp_status fsp_create_instance_pairs(const int32_t *p, int32_t n, int32_t m, const int32_t *pairs, int32_t npairs,
                                     int32_t flags, fsp_instance *out)
{
    fsp_status st = check_shape(p, n, m, flags, out);
    if (st != FSP_OK) return st;
    if (!pairs || npairs < 1 || npairs > m * (m - 1) / 2) return FSP_E_INVAL;
    std::vector<std::pair<int, int>> prs;
    bool last = false;  // a pair ending on the last machine: a complete schedule's bound is its makespan
    for (int i = 0; i < npairs; ++i) {
        const int k = pairs[2 * i], l = pairs[2 * i + 1];
        if (k < 0 || l <= k || l >= m) return FSP_E_INVAL;
        last = last || l == m - 1;
        prs.push_back({k, l});
    }
    if (!last) return FSP_E_INVAL;
    std::sort(prs.begin(), prs.end());
    if (std::adjacent_find(prs.begin(), prs.end()) != prs.end()) return FSP_E_INVAL;  // a repeated pair
    return create_instance(p, n, m, flags, prs, out);
}

fsp_status fsp_destroy_instance(fsp_instance inst)
{
    if (!inst) return FSP_OK;
    hipDeviceSynchronize();
    hipFree(inst->dev_blob);
    delete[] inst->p_host;
    delete inst;
    return FSP_OK;
}

fsp_status fsp_get_instance_info(fsp_instance inst, fsp_instance_info *info)
{
    if (!inst || !info) return FSP_E_INVAL;
    info->n = inst->n;
    info->m = inst->m;
    info->pairs = inst->P;
    info->max_value = inst->max_value;
    info->packed16 = inst->packed16;
    info->flags = inst->flags;
    info->table_bytes = inst->table_bytes;
    return FSP_OK;
}

}  // extern "C"
