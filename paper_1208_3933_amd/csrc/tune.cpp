// Tile-schedule tuner.  For an instance shape, times every schedule of the
// 16-bit scan (waves per 128-node group: 1, 2, 4, 8, 16; a workgroup then
// stages 16 / wpg groups of masks in LDS at once) on a seeded sample pool
// through the batched path, then the fastest schedule in both launch forms of
// the batched scan (persistent or one workgroup per item), keeps the result
// in the process-wide tuning table (used by fsp_bound_pool and the batch
// planner), and can save or load that table as text ("n m waves_per_group
// form" per line).
#include <algorithm>
#include <cstdio>
#include <numeric>
#include <random>
#include <vector>

#include "batch.h"

using namespace fspbb;

namespace {

// Best-of-reps device time (us) of one run of a one-pool batch in a given
// schedule and launch form (the first run warms up).
fsp_status time_batch(fsp_instance inst, const int32_t *dpre, const int32_t *ddep, int32_t *dout, int64_t N,
                      int wpg, int form, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double *us)
{
    fsp_pool_desc d{inst, dpre, ddep, N, dout};
    fsp_batch b = nullptr;
    fsp_status st = create_batch(&d, 1, FSP_BATCH_GRAPH, wpg, form, &b);
    if (st != FSP_OK) return st;
    double t_best = -1;
    for (int r = 0; r <= reps && st == FSP_OK; ++r) {
        hipEventRecord(e0, s);
        st = fsp_batch_run(b, s);
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) st = FSP_E_DEVICE;
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        if (r > 0 && (t_best < 0 || ms < t_best)) t_best = ms;
    }
    fsp_batch_destroy(b);
    *us = t_best * 1e3;
    return st;
}

}  // namespace

extern "C" {

fsp_status fsp_autotune(fsp_instance inst, int64_t sample_nodes, int32_t reps, fsp_tune_result *res)
{
    if (!inst || !res || sample_nodes < 1 || reps < 1) return FSP_E_INVAL;
    if (!inst->packed16) return FSP_E_INVAL;
    *res = fsp_tune_result{};
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != inst->device) hipSetDevice(inst->device);
    const int n = inst->n, m = inst->m;
    const int64_t N = sample_nodes;
    // seeded sample: random permutation rows, depths uniform on 0..n-1
    std::mt19937_64 rng(((uint64_t)n << 32) ^ (uint64_t)m ^ 0x5eedULL);
    std::vector<int32_t> pre((size_t)N * n), dep(N);
    std::vector<int32_t> perm(n);
    for (int64_t i = 0; i < N; ++i) {
        std::iota(perm.begin(), perm.end(), 0);
        for (int t = n - 1; t > 0; --t) std::swap(perm[t], perm[rng() % (uint64_t)(t + 1)]);
        std::copy(perm.begin(), perm.end(), pre.begin() + i * n);
        dep[i] = (int32_t)(rng() % (uint64_t)n);
    }
    int32_t *dpre = nullptr, *ddep = nullptr, *dout = nullptr;
    hipError_t e = hipMalloc(&dpre, pre.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&ddep, dep.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&dout, dep.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(dpre, pre.data(), pre.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ddep, dep.data(), dep.size() * 4, hipMemcpyHostToDevice);
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    fsp_status st = e == hipSuccess ? FSP_OK : FSP_E_DEVICE;
    const int default_wpg = scan_tuning(n, m).waves_per_group;
    double best = -1;
    int best_wpg = default_wpg;
    const int cands[5] = {1, 2, 4, 8, 16};
    for (int c = 0; c < 5 && st == FSP_OK; ++c) {
        const int wpg = cands[c];
        const int64_t gpp = kBatchWaves / wpg;
        if ((size_t)gpp * (n + 1) * 256 > kLdsLimit) continue;  // the tile must fit LDS
        double us = 0;
        st = time_batch(inst, dpre, ddep, dout, N, wpg, kBatchGrid, reps, s, e0, e1, &us);
        if (st != FSP_OK) break;
        res->cand_wpg[res->candidates] = wpg;
        res->cand_us[res->candidates] = us;
        res->candidates++;
        if (wpg == default_wpg) res->default_us = us;
        if (best < 0 || us < best) { best = us; best_wpg = wpg; }
    }
    int form = kBatchGrid;
    if (st == FSP_OK) {
        double pus = 0;
        st = time_batch(inst, dpre, ddep, dout, N, best_wpg, kBatchPersistent, reps, s, e0, e1, &pus);
        res->grid_us = best;
        res->persistent_us = pus;
        if (st == FSP_OK && pus < best) {
            form = kBatchPersistent;
            best = pus;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    hipFree(dpre);
    hipFree(ddep);
    hipFree(dout);
    if (prev >= 0 && prev != inst->device) hipSetDevice(prev);
    if (st != FSP_OK) return st;
    set_scan_tuning(n, m, ScanTuning{best_wpg, 8, form});
    res->waves_per_group = best_wpg;
    res->form = form;
    res->best_us = best;
    return FSP_OK;
}

fsp_status fsp_tune_get(int32_t n, int32_t m, int32_t *waves_per_group, int32_t *tuned)
{
    if (n < 1 || m < 2 || !waves_per_group) return FSP_E_INVAL;
    *waves_per_group = scan_tuning(n, m).waves_per_group;
    if (tuned) *tuned = has_scan_tuning(n, m) ? 1 : 0;
    return FSP_OK;
}

fsp_status fsp_tune_set(int32_t n, int32_t m, int32_t waves_per_group)
{
    if (n < 1 || m < 2) return FSP_E_INVAL;
    if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4 && waves_per_group != 8 &&
        waves_per_group != 16)
        return FSP_E_INVAL;
    ScanTuning t = scan_tuning(n, m);
    t.waves_per_group = waves_per_group;
    t.unroll = 8;
    set_scan_tuning(n, m, t);
    return FSP_OK;
}

fsp_status fsp_tune_get_form(int32_t n, int32_t m, int32_t *form)
{
    if (n < 1 || m < 2 || !form) return FSP_E_INVAL;
    *form = scan_tuning(n, m).form;
    return FSP_OK;
}

fsp_status fsp_tune_set_form(int32_t n, int32_t m, int32_t form)
{
    if (n < 1 || m < 2 || (form != FSP_FORM_PERSISTENT && form != FSP_FORM_GRID)) return FSP_E_INVAL;
    ScanTuning t = scan_tuning(n, m);
    t.form = form;
    set_scan_tuning(n, m, t);
    return FSP_OK;
}

fsp_status fsp_tune_save(const char *path)
{
    if (!path) return FSP_E_INVAL;
    std::vector<std::pair<std::pair<int, int>, ScanTuning>> ent;
    scan_tuning_entries(ent);
    FILE *f = fopen(path, "w");
    if (!f) return FSP_E_INVAL;
    fprintf(f, "# fspbb scan tuning: n m waves_per_group form (0 persistent, 1 one workgroup per item)\n");
    for (auto &kv : ent)
        fprintf(f, "%d %d %d %d\n", kv.first.first, kv.first.second, kv.second.waves_per_group, kv.second.form);
    fclose(f);
    return FSP_OK;
}

fsp_status fsp_tune_load(const char *path)
{
    if (!path) return FSP_E_INVAL;
    FILE *f = fopen(path, "r");
    if (!f) return FSP_E_INVAL;
    char line[256];
    fsp_status st = FSP_OK;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        int n = 0, m = 0, w = 0, form = kBatchGrid;
        const int got = sscanf(line, "%d %d %d %d", &n, &m, &w, &form);
        if (got < 3) continue;
        if (fsp_tune_set(n, m, w) != FSP_OK || fsp_tune_set_form(n, m, form) != FSP_OK) st = FSP_E_INVAL;
    }
    fclose(f);
    return st;
}

}  // extern "C"
