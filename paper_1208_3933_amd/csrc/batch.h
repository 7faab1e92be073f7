// Batched bounding of many pools in one persistent launch (host/device shared).
#pragma once

#include <algorithm>
#include <utility>
#include <vector>

#include "fspbb_internal.h"
#include "ws16.h"

namespace fspbb {

// Blocks of a pool's depth sort: one per 4096 nodes, at most this many (each
// scatter block sums the per-block counts of every bucket itself).
constexpr int kSortMaxBlocks = 64;

// LDS words of the 16-bit decode for n jobs and MV machine slots: the
// scheduled bits of 256 lanes (floor(n / 32) + 1 words each: jobs 0..n) and the (n + 1) rows
// of MV / 2 packed processing-time pairs.  Monotone in n, so a launch sized
// for the largest n of several pools serves all of them.
inline size_t decode16_lds_words(int n, int MV) { return (size_t)((n >> 5) + 1) * 256 + (size_t)(n + 1) * (MV / 2); }

constexpr int kBatchWaves = 16;  // waves per workgroup of the persistent scan
// LDS a workgroup may allocate on gfx950 (160 KB per compute unit).
constexpr size_t kLdsLimit = 160 * 1024;

// A work item stages 16 / wpg groups of (n + 1) mask rows of 256 bytes.  The
// tuned or rule-of-thumb wpg is raised (fewer groups per item, more waves on
// each) until that fits LDS; n <= 512 always fits with one group per item.
inline int fit_waves_per_group(int wpg, int n)
{
    while (wpg < kBatchWaves && (size_t)(kBatchWaves / wpg) * (size_t)(n + 1) * 256 > kLdsLimit) wpg *= 2;
    return wpg;
}
constexpr int64_t kSortMinNodes = 512;  // smaller pools are decoded in pool order

// One pool of a batch.  wpg = waves per 128-node group (divides 16); a work
// item stages 16 / wpg groups of the pool in LDS at once.
struct BatchPool {
    DevTables T;
    Workspace16 W;
    const int32_t *prefixes;
    const int32_t *depths;
    int32_t *out_lb;
    int64_t N, Npad;
    int32_t wpg;
    int32_t sortB;        // blocks of the depth sort; 0 = nodes taken in pool order (W.order null)
    int64_t sort_chunk;   // nodes per depth-sort block
};

// A work item: ngroups consecutive 128-node groups of one pool.
struct WorkItem {
    int32_t pool, group0, ngroups, reserved;
};

// Counting sort of every sorted pool's nodes by depth (W.order), three launches.
hipError_t launch_batch_depth_sort(const BatchPool *pools, const int64_t *blk_off, const int32_t *sort_pools,
                                   int nsort, int64_t nblocks, int nmax, hipStream_t s);
hipError_t launch_batch_decode(int MV, const BatchPool *pools, const int64_t *blk_off, const int32_t *cls_pools,
                               int ncls, int64_t nblocks, size_t lds_bytes, hipStream_t s);
// Launch form of the batched scan: persistent workgroups fed by a counter
// (grid = CUs x occupancy), or one workgroup per work item.
constexpr int kBatchPersistent = FSP_FORM_PERSISTENT, kBatchGrid = FSP_FORM_GRID;
hipError_t launch_batch_scan(const BatchPool *pools, const WorkItem *items, int n_items, uint32_t *counter,
                             int grid, size_t lds_bytes, int form, hipStream_t s);
int batch_scan_blocks_per_cu(size_t lds_bytes);

// Tile schedule of the scan for an instance shape: waves per group and slots
// per scalar record batch.  Filled by the autotuner, else a rule of thumb.
struct ScanTuning {
    int waves_per_group;
    int unroll;
    int form;  // batched-scan launch form preferred for the shape
};
ScanTuning scan_tuning(int n, int m);
// The schedule of an instance: its shape's entry, or for an instance over a
// subset of the machine pairs the rule of thumb for its pair count.
ScanTuning scan_tuning_for(const fsp_instance_s *I);
void set_scan_tuning(int n, int m, ScanTuning t);
bool has_scan_tuning(int n, int m);
void scan_tuning_entries(std::vector<std::pair<std::pair<int, int>, ScanTuning>> &out);

// fsp_batch_create with a forced waves-per-group (0 = tuned) and launch form
// (-1 = from the tuning table).
fsp_status create_batch(const fsp_pool_desc *pools, int32_t n_pools, int32_t flags, int32_t wpg_force,
                        int32_t form_force, fsp_batch *out);

// Launch plan of a batch: pool records, LPT-ordered work items, decode
// classes (pools grouped by machine count rounded up to 4), and the layout
// of one device region = per-pool decode workspace (ws_bytes) followed by the
// metadata the kernels read (meta_bytes).
struct BatchPlan {
    struct Cls {
        int MV = 0;
        std::vector<int32_t> idx;     // pools of this class
        std::vector<int64_t> off;     // decode block offsets, idx.size() + 1
        int64_t nblocks = 0;
        size_t lds = 0;
        int nmax = 0;                 // largest n among the pools
        size_t meta_off = 0, meta_idx = 0;
    };
    std::vector<BatchPool> pools;
    std::vector<size_t> ws_off;
    std::vector<WorkItem> items;
    std::vector<Cls> classes;
    Cls sort;                         // the depth-sorted pools (MV unused); empty = no sort
    size_t scan_lds = 0, ws_bytes = 0, meta_bytes = 0;
    int form = kBatchGrid;
    size_t meta_pools = 0, meta_items = 0, meta_counter = 0;
    int64_t total_nodes = 0;
    std::vector<char> decoded;        // per pool: workspace given by the caller (not laid out)
    char *dmeta = nullptr;            // device address of the metadata once laid out
};

fsp_status check_pools(const fsp_pool_desc *pools, int32_t n_pools, int *dev_out);
// sort_depths: sort each pool's nodes by depth before decoding (fewer
// divergent prefix loops on pools of mixed depths).
// form: the launch form: persistent when every pool's shape prefers it, else
// one workgroup per item; form_force >= 0 overrides.
// ready (optional, one entry per pool): a pool whose entry has a non-null dec
// is already decoded into that workspace (identity order); it is neither
// sorted nor decoded and takes no workspace of the plan.
void plan_batch(const fsp_pool_desc *pools, int32_t n_pools, int32_t wpg_force, bool sort_depths, BatchPlan &pl,
                int32_t form_force = -1, const Workspace16 *ready = nullptr);
// Points the pools' workspaces into `base` (at the plan's offsets) and builds
// the metadata image for device address dmeta (null: right after the
// workspaces, at base + ws_bytes).
void layout_batch(BatchPlan &pl, char *base, std::vector<char> &host_meta, char *dmeta = nullptr);
hipError_t enqueue_batch(const BatchPlan &pl, int grid, hipStream_t s);
int batch_grid(int dev, size_t scan_lds);

// A reusable device region for batches re-planned on every call (the merged
// bounding step of concurrent searches).  The region grows by doubling and is
// kept; the metadata goes up through a pinned staging buffer with one async
// copy.  A call must not start before the previous call's copy has completed
// (the caller synchronizes its stream between calls).
struct BatchArena {
    BatchPlan plan;
    std::vector<char> meta;
    void *dev = nullptr;
    size_t dev_bytes = 0;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipError_t run(const fsp_pool_desc *pools, int32_t n_pools, hipStream_t s, const Workspace16 *ready = nullptr);
    // run in three parts, for a caller that uploads the metadata with its own
    // copy: plan (and grow the workspace region; *meta_bytes = metadata size),
    // write the metadata for device address dmeta into host memory hdst, and,
    // once the copy is enqueued, launch.
    hipError_t plan_only(const fsp_pool_desc *pools, int32_t n_pools, hipStream_t s, const Workspace16 *ready,
                         size_t *meta_bytes);
    void stage(char *dmeta, char *hdst);
    hipError_t launch(hipStream_t s);
    void release(hipStream_t s);
    // The region's size once a plan has needed ws bytes of workspace.
    size_t bytes_after(size_t ws) const { return ws > dev_bytes ? std::max(ws, dev_bytes * 2) : dev_bytes; }
};

}  // namespace fspbb
