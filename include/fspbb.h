/*
 * fspbb.h - C ABI of the MI355X (gfx950) flow-shop bounding library.
 *
 * The library evaluates, on one GPU, the two-machine lower bound of
 * Lageweg, Lenstra and Rinnooy Kan (built on Johnson's rule) over pools of
 * permutation flow-shop sub-problems, and runs the branch-and-bound steps
 * around it, after Melab, Chakroun, Mezmaz and Tuyttens, "A GPU-accelerated
 * Branch-and-Bound Algorithm for the Flow-Shop Scheduling Problem".
 *
 * Conventions shared by every call:
 *   - n jobs (0..n-1), m machines (0..m-1); p[j*m + k] is the processing time
 *     of job j on machine k (the PTM matrix of Table I), row-major int32.
 *   - A sub-problem (node) is a scheduled prefix pi(1..d) followed by the
 *     unscheduled jobs (Sec. II-C).  A pool of N nodes is two device arrays:
 *     prefixes[N*n] (row i holds its d_i scheduled jobs in order in its first
 *     d_i entries; the rest of the row is ignored) and depths[N].
 *   - "dev" pointers are HIP device pointers, "host" pointers are host
 *     memory.  The caller owns every buffer it passes; the library never
 *     frees them and keeps no reference after the call returns.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls marked "async" only enqueue work on that stream.
 *   - Every call returns an fsp_status: 0 = success, < 0 = error, > 0 =
 *     informational.  fsp_status_string() names each code.
 */
#ifndef FSPBB_H
#define FSPBB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fsp_status;

enum {
    FSP_OK = 0,
    FSP_E_INVAL = -1,     /* bad argument: null pointer, n < 1, m < 2, p < 0, N < 0 ... */
    FSP_E_RANGE = -2,     /* a value could overflow the int32 arithmetic of the bound,
                             or a buffer is too small for the result */
    FSP_E_NOMEM = -3,     /* device or host allocation failed */
    FSP_E_DEVICE = -4,    /* a HIP runtime call failed (see fsp_last_error_string) */
    FSP_E_BADNODE = -5,   /* the pool held invalid nodes (their bound is FSP_LB_INVALID) */
    FSP_E_NODEVICE = -6,  /* no gfx950 device is visible */
    FSP_BUDGET = 1,       /* a search stopped at its node budget without a proof */
    FSP_PENDING = 2       /* a served search has not finished yet */
};

/* Bound written for an invalid node: depth outside 0..n, a job outside
 * 0..n-1, or a job repeated in the prefix. */
#define FSP_LB_INVALID (-1)

/* Opaque instance: owns host and device copies of the per-instance tables of
 * Table I (PTM, LM, JM, the machine-pair list MM) and the per-job tails. */
typedef struct fsp_instance_s *fsp_instance;

typedef struct {
    int32_t n, m;          /* jobs, machines */
    int32_t pairs;         /* machine pairs the bound takes: m(m-1)/2, or the subset's size */
    int32_t max_value;     /* (n+m-1) * max p: bound on every intermediate value */
    int32_t packed16;      /* 1 when max_value < 65536: the fast 16-bit path is used */
    int32_t flags;         /* FSP_INSTANCE_* flags it was created with */
    int64_t table_bytes;   /* device bytes held by the instance */
} fsp_instance_info;

/* Instance flag: the bound takes each machine's release as the earliest time
 * any unscheduled job could start on it (RM as "earliest starting times of
 * jobs", Table I, with the minimum over jobs of Fig. 2): for machine k, the
 * least over unscheduled jobs j of max(prefix completion on k, completion of
 * j on k-1 were j scheduled next).  Without it the release is the prefix
 * completion on k.  The bound is never lower, still valid, and the same at
 * m = 2 and with at most one job left.  Applies to every call on the
 * instance: bounding, batches, steps, solves and served searches. */
#define FSP_INSTANCE_HEADS 1

/* Reported in fsp_instance_info.flags (not accepted as an input flag): the
 * instance was created by fsp_create_instance_pairs with fewer pairs than
 * m(m-1)/2. */
#define FSP_INSTANCE_PAIR_SUBSET 2

/* Name of a status code (static string). */
const char *fsp_status_string(fsp_status s);

/* Text of the last HIP error seen by this thread (static buffer). */
const char *fsp_last_error_string(void);

/*
 * fsp_create_instance - copy an instance and build its tables on the device
 * (Sec. II-D: lags, Johnson-with-lags order per machine pair, computed once).
 *   p    host, n*m int32, p[j*m+k] >= 0.  Copied; the caller may free it.
 *   n    >= 1, m >= 2 (with one machine there is no pair and no bound).
 *   out  host, receives the new instance.
 * Errors: FSP_E_INVAL (null, n < 1, m < 2, n > 512, m > 32, p < 0),
 * FSP_E_RANGE ((n+m-1) * max p >= 2^31), FSP_E_NOMEM, FSP_E_DEVICE,
 * FSP_E_NODEVICE.  Uses the current HIP device; the instance's kernels must
 * later run on that same device.
 */
fsp_status fsp_create_instance(const int32_t *p, int32_t n, int32_t m, fsp_instance *out);

/* fsp_create_instance with flags (0 or FSP_INSTANCE_HEADS); other bits:
 * FSP_E_INVAL. */
fsp_status fsp_create_instance_ex(const int32_t *p, int32_t n, int32_t m, int32_t flags, fsp_instance *out);

/*
 * fsp_create_instance_pairs - an instance whose bound is the maximum of the
 * pair values of Fig. 2 over a subset of the machine pairs only (the MM list
 * of Table I replaced by `pairs`).  Each pair's value is unchanged, so the
 * bound is never above the full one, still valid, and cheaper in proportion
 * to the pairs dropped.  A search with it bounds more nodes.
 *   pairs   host, npairs x 2 int32 (k, l), 0 <= k < l < m, no pair twice,
 *           and at least one pair with l = m - 1 (then a complete schedule's
 *           bound is its makespan, which the searches rely on); copied.  The
 *           order does not matter.
 *   npairs  1 .. m(m-1)/2 (all of them gives the plain instance).
 *   flags   as for fsp_create_instance_ex.
 * Errors as for fsp_create_instance_ex, and FSP_E_INVAL for a null list,
 * an npairs out of range, a pair out of range, a repeated pair or no pair
 * ending on the last machine.  Every entry point accepts the instance.
 */
fsp_status fsp_create_instance_pairs(const int32_t *p, int32_t n, int32_t m, const int32_t *pairs, int32_t npairs,
                                     int32_t flags, fsp_instance *out);

/* Release an instance (synchronises the device first).  NULL is a no-op. */
fsp_status fsp_destroy_instance(fsp_instance inst);

/* Shape and table size of an instance. */
fsp_status fsp_get_instance_info(fsp_instance inst, fsp_instance_info *info);

/*
 * fsp_bound_pool - lower bound of every node of a pool (Sec. III-A: one pool
 * of sub-problems bounded in parallel on the GPU; the bound of Sec. II-D,
 * Fig. 2).  Async on stream.
 *   prefixes  dev, N*n int32, row i = the d_i scheduled jobs, then ignored.
 *   depths    dev, N int32, 0 <= d_i <= n (d_i = n gives the makespan).
 *   N         >= 0 (0 is a no-op).
 *   out_lb    dev, N int32: bound of node i, or FSP_LB_INVALID.
 * Invalid nodes do not stop the call: their row gets FSP_LB_INVALID, every
 * other row is computed, and the instance's invalid-node counter is raised;
 * fsp_pool_status() reads it.  Errors (returned at once): FSP_E_INVAL
 * (null pointer with N > 0, N < 0), FSP_E_DEVICE (launch failure).
 */
fsp_status fsp_bound_pool(fsp_instance inst, const int32_t *prefixes, const int32_t *depths,
                          int64_t N, int32_t *out_lb, void *stream);

/*
 * fsp_pool_status - synchronise stream, then return FSP_E_BADNODE if any
 * invalid node was met by fsp_bound_pool on this instance since the last
 * call (and clear the counter), else FSP_OK.  n_bad (host, may be NULL)
 * receives the count.
 */
fsp_status fsp_pool_status(fsp_instance inst, void *stream, int64_t *n_bad);

/*
 * fsp_bound_pool_variant - like fsp_bound_pool with an explicit kernel
 * variant (0 = automatic: 2 when max_value < 65536, else 4; 1 = general
 * 32-bit lane-per-node kernel with register bit sets, 2 = 16-bit packed
 * decode+scan kernels, lane per two nodes, 3 = 32-bit wave-per-node kernels,
 * lane per machine pair, 4 = 32-bit decode+scan kernels, lane per node, masks
 * in LDS).  Used by tests and the benchmark to compare the mappings on the
 * same pool.  FSP_E_INVAL for a variant the instance cannot run (2 needs
 * max_value < 65536).
 */
fsp_status fsp_bound_pool_variant(fsp_instance inst, const int32_t *prefixes,
                                  const int32_t *depths, int64_t N, int32_t *out_lb,
                                  int32_t variant, void *stream);

/*
 * fsp_bound_pool_noalloc - fsp_bound_pool for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid allocation.  The arguments, layout, results,
 * invalid-node handling and stream semantics are those of fsp_bound_pool.
 * The call makes no device or host allocation.  The decode's workspace
 * (about 156 bytes per node at 200 x 20 on the 16-bit path, 276 on the 32-bit
 * path) is a fixed array of FSP_NOALLOC_SCRATCH_BYTES inside the library.
 * Each device the library runs on holds its own copy until the process ends;
 * its address is looked up on the first call on that device.
 * Every call on a device shares that device's array, and a call leaves its
 * contents behind.  Calls that overlap on one device (on different streams,
 * or from several host threads without ordering) therefore race and give
 * wrong bounds: order them on one stream.
 * Errors: as fsp_bound_pool, plus FSP_E_RANGE (nothing launched) when the
 * workspace of N nodes would exceed the array, i.e. N > fsp_noalloc_max_nodes.
 */
#define FSP_NOALLOC_SCRATCH_BYTES (48u << 20)
fsp_status fsp_bound_pool_noalloc(fsp_instance inst, const int32_t *prefixes,
                                  const int32_t *depths, int64_t N, int32_t *out_lb,
                                  void *stream);

/* Largest N fsp_bound_pool_noalloc accepts for this instance (-1 for a null
 * instance).  Host only. */
int64_t fsp_noalloc_max_nodes(fsp_instance inst);

/* ---- batched bounding --------------------------------------------------- */

/* One pool of a batch: an instance and its pool buffers (as fsp_bound_pool). */
typedef struct {
    fsp_instance inst;
    const int32_t *prefixes;   /* dev N*n */
    const int32_t *depths;     /* dev N */
    int64_t N;                 /* >= 0 */
    int32_t *out_lb;           /* dev N */
} fsp_pool_desc;

typedef struct fsp_batch_s *fsp_batch;

/* fsp_batch_create flag: capture the batch's launches in a HIP graph. */
#define FSP_BATCH_GRAPH 1

/*
 * fsp_batch_create - plan the bounding of many pools (of any instances of the
 * 16-bit path, on one device) as one decode launch per machine-count class
 * plus one persistent scan launch whose workgroups take 128-node group tiles
 * from a device queue, longest first.  The tile schedule (groups staged in
 * LDS per tile, waves per group) comes from the tuner (fsp_autotune) or a
 * rule of thumb.  With FSP_BATCH_GRAPH the launches are captured once in a
 * HIP graph; fsp_batch_run then replays it.  The descriptors' buffers must
 * stay valid, at the same addresses, for the life of the batch; their
 * contents may change between runs.
 *   pools   host, n_pools >= 1 descriptors.
 * Errors: FSP_E_INVAL (null, N < 0, an instance outside the 16-bit path or
 * on another device), FSP_E_NOMEM, FSP_E_DEVICE.  The batch owns a device
 * workspace of about (6m + n/8 + 4) bytes per node.
 */
fsp_status fsp_batch_create(const fsp_pool_desc *pools, int32_t n_pools, int32_t flags, fsp_batch *out);

/* fsp_batch_run - enqueue one bounding of every pool of the batch on stream
 * (async).  Invalid nodes get FSP_LB_INVALID and raise their instance's
 * counter, as with fsp_bound_pool.  Runs of one batch must not overlap. */
fsp_status fsp_batch_run(fsp_batch b, void *stream);

/* fsp_batch_destroy - synchronise the device and free the batch. */
fsp_status fsp_batch_destroy(fsp_batch b);

/* Total nodes, work items and scan workgroups of a batch (the grid of a
 * persistent launch, else one per work item). */
fsp_status fsp_batch_info(fsp_batch b, int64_t *total_nodes, int32_t *n_items, int32_t *grid);

/* fsp_bound_pools_batched - one-shot: create (without graph), run, wait, destroy. */
fsp_status fsp_bound_pools_batched(const fsp_pool_desc *pools, int32_t n_pools, void *stream);

/* ---- tile-schedule tuning ------------------------------------------------ */

/* Launch forms of the batched scan: persistent workgroups (CUs x occupancy)
 * taking work items from a device counter, or one workgroup per work item
 * dispatched by the hardware in item order (longest first). */
#define FSP_FORM_PERSISTENT 0
#define FSP_FORM_GRID 1

typedef struct {
    int32_t waves_per_group;  /* chosen schedule: waves per 128-node group */
    int32_t candidates;       /* schedules measured */
    double best_us;           /* device time of one batch run of the sample, chosen schedule */
    double default_us;        /* same for the rule-of-thumb schedule */
    int32_t cand_wpg[8];
    double cand_us[8];        /* per waves-per-group candidate, in the one-per-item form */
    int32_t form;             /* chosen launch form for the chosen schedule */
    int32_t reserved;
    double grid_us, persistent_us;  /* the chosen schedule in each launch form */
} fsp_tune_result;

/*
 * fsp_autotune - time every scan tile schedule for this instance's shape (n,
 * m) on a seeded sample pool of sample_nodes nodes (best of reps runs each),
 * then the fastest in both launch forms, and store the result in the
 * process-wide tuning table, which fsp_bound_pool and fsp_batch_create
 * consult (a batch runs persistent only when every pool's shape prefers it).  The pool size used by the
 * paper was chosen the same way, by trying sizes at run time (Sec. IV-A).
 * Synchronous; allocates and frees its own sample buffers.  16-bit path only.
 */
fsp_status fsp_autotune(fsp_instance inst, int64_t sample_nodes, int32_t reps, fsp_tune_result *res);
/* Tuning table access: current schedule for a shape (tuned = 0 for the rule
 * of thumb), explicit setting (1, 2, 4, 8 or 16), save/load as text. */
fsp_status fsp_tune_get(int32_t n, int32_t m, int32_t *waves_per_group, int32_t *tuned);
fsp_status fsp_tune_set(int32_t n, int32_t m, int32_t waves_per_group);
/* Launch form preferred for a shape (FSP_FORM_GRID unless tuned or set). */
fsp_status fsp_tune_get_form(int32_t n, int32_t m, int32_t *form);
fsp_status fsp_tune_set_form(int32_t n, int32_t m, int32_t form);
/* The table as text, one "n m waves_per_group form" line per shape. */
fsp_status fsp_tune_save(const char *path);
fsp_status fsp_tune_load(const char *path);

/* ---- branch-and-bound ---------------------------------------------------- */

/* ub0 value of fsp_solve: start from the NEH heuristic's schedule. */
#define FSP_UB_NEH (-1)
/* An upper bound that eliminates nothing. */
#define FSP_UB_NONE 0x7fffffff

typedef struct {
    int64_t n_children;   /* children generated and bounded */
    int64_t n_survivors;  /* children kept (not complete, bound < ub_out) */
    int32_t ub_out;       /* min(ub_in, bound of the best complete child) */
    int32_t improved;     /* 1 when a complete child lowered the upper bound */
    int64_t fingerprint;  /* sum over survivors of (S - rank) * (appended job + 1), S survivors,
                             rank in child order: a check of the survivor order */
} fsp_step_result;

/*
 * fsp_branch_and_prune - one pool step of the branch-and-bound (Sec. II-A:
 * branching, bounding, elimination; Sec. III-A: the pool is bounded on the
 * GPU).  Synchronous on stream.
 *   parents, parent_depths  dev, K rows of n int32 and K depths, in pop order.
 *   ub_in       current upper bound (>= 0; FSP_UB_NONE for none).
 *   Each parent of depth d < n gets n - d children, in parent order and, per
 *   parent, in increasing appended job id (forward branching, Sec. II-B).
 *   Every child is bounded.  ub_out = min(ub_in, best complete child); when
 *   it improves, incumbent (dev, n int32, may be NULL) receives the first
 *   complete child in child order that attains it.  The children that are
 *   not complete and whose bound is below ub_out survive and are written in
 *   child order to children (dev cap x n), child_depths (dev cap) and
 *   child_lb (dev cap, may be NULL).
 * Errors: FSP_E_INVAL, FSP_E_BADNODE (an invalid parent: it gets no
 * children), FSP_E_RANGE (more survivors than cap: the first cap are
 * written, res still counts all), FSP_E_NOMEM, FSP_E_DEVICE.
 */
fsp_status fsp_branch_and_prune(fsp_instance inst, const int32_t *parents, const int32_t *parent_depths,
                                int64_t K, int32_t ub_in, int32_t *children, int32_t *child_depths,
                                int32_t *child_lb, int64_t cap, int32_t *incumbent, fsp_step_result *res,
                                void *stream);

typedef struct {
    int32_t opt;           /* best makespan found (the optimum when proven) */
    int32_t proven;        /* 1 when the search completed */
    int64_t nodes_bounded; /* the root plus every child bounded */
    int64_t steps;         /* pool steps */
    int32_t ub0;           /* initial upper bound used */
    int32_t improvements;  /* steps that lowered the upper bound */
    int64_t max_stack;     /* largest device stack, in nodes */
} fsp_solve_result;

/*
 * fsp_solve - depth-first branch-and-bound from the root, pool-synchronous,
 * with the search stack resident on the device.  Each step pops parents from
 * the top of the stack while their children fit in pool_cap (the first is
 * always taken), runs one fsp_branch_and_prune step on them, and pushes the
 * survivors in reverse child order.  The root is bounded first and
 * eliminated when its bound is >= ub0.  Elimination is bound >= upper bound.
 *   ub0         FSP_UB_NEH (start from NEH), FSP_UB_NONE, or a makespan >= 0.
 *   pool_cap    >= 1, children per step.
 *   node_budget >= 1: stop (FSP_BUDGET, proven = 0) once this many nodes
 *               have been bounded.
 *   perm_out    host, n int32: best schedule found (NEH's when nothing
 *               better was found; -1s when ub0 was given and never beaten).
 *   steplog     host, steplog_cap x 6 int64, may be NULL: per step the
 *               parents popped, children bounded, upper bound after the step,
 *               children pushed, stack size after, and the step fingerprint.
 * Returns FSP_OK (proven), FSP_BUDGET, or an error.
 */
fsp_status fsp_solve(fsp_instance inst, int32_t ub0, int64_t pool_cap, int64_t node_budget,
                     fsp_solve_result *res, int32_t *perm_out, int64_t *steplog, int64_t steplog_cap,
                     void *stream);

/* Flag of fsp_solve_ex: select best first instead of depth first (Sec.
 * III-A).  The frontier is ordered by (bound, insertion order).  Each step
 * drops the frontier nodes with bound >= the upper bound, takes parents from
 * the front while their children fit in pool_cap (the first always), runs
 * the same branch/bound/upper-bound step as fsp_solve, and inserts the
 * survivors in child order.  The search is proven when the frontier is empty
 * after the drop.  max_stack reports the largest frontier; steplog[4] the
 * frontier size after each step. */
#define FSP_SOLVE_BEST_FIRST 1

/* Depth first with the steps chosen on the device: the parents of each step
 * are taken from the depths at the top of the device stack, and the counters,
 * upper bound, stack top, step log and stop rule are kept on the device, so
 * the host enqueues several steps (1, 2, 4, ... up to 16) per
 * synchronisation.  The steps, results and step log are those of fsp_solve.
 * Applies to instances whose children are bounded from their parents
 * (max_value < 65536, no FSP_INSTANCE_HEADS); others run host-driven. */
#define FSP_SOLVE_DEVICE_STEPS 2

/* fsp_solve with flags (0 = depth first as fsp_solve, FSP_SOLVE_BEST_FIRST,
 * or FSP_SOLVE_DEVICE_STEPS; the last two are exclusive: FSP_E_INVAL). */
fsp_status fsp_solve_ex(fsp_instance inst, int32_t ub0, int64_t pool_cap, int64_t node_budget, int32_t flags,
                        fsp_solve_result *res, int32_t *perm_out, int64_t *steplog, int64_t steplog_cap,
                        void *stream);

typedef struct {
    int32_t opt;           /* best makespan found (the optimum when proven) */
    int32_t proven;        /* 1 when every subtree was explored within the budget */
    int64_t nodes_bounded; /* children bounded (depends on thread timing; the root is not bounded) */
    int64_t pools;         /* bounding launches (each merges the pools waiting at the time) */
    int32_t threads;       /* host explorers */
    int32_t ub0;           /* initial upper bound used */
    double seconds;        /* wall time of the call */
} fsp_explore_result;

/*
 * fsp_explore - hybrid search: host threads explore the tree, the GPU bounds
 * their pools (Sec. III: the host selects and branches, the GPU bounds; with
 * several host explorers, the multi-threaded exploration left to future work
 * in Sec. V).  Each of `threads` explorers runs a depth-first search on its
 * own host stack over subtrees taken from a shared list (the first levels of
 * the tree, expanded breadth first until there are 4 per explorer): it pops
 * parents while their children fit in pool_cap and hands the parents to one
 * bounding thread, which merges the requests waiting at that moment into one
 * host-to-device copy of parent prefixes, one step that lists and bounds all
 * their children on the device, and one copy back of the bounds (in parent
 * order, then by increasing appended job).  The explorer builds rows only
 * for the children it keeps.  The upper bound is shared (elimination: bound
 * >= it).
 * Node counts depend on thread timing; the optimum does not.  Synchronous.
 *   ub0, pool_cap, node_budget as in fsp_solve; threads 1..256; perm_out host n.
 * Returns FSP_OK (proven), FSP_BUDGET, or an error.
 */
fsp_status fsp_explore(fsp_instance inst, int32_t ub0, int32_t threads, int64_t pool_cap, int64_t node_budget,
                       fsp_explore_result *res, int32_t *perm_out, void *stream);

/* fsp_neh - NEH heuristic schedule (host computation): perm_out (host n, may
 * be NULL) and its makespan. */
fsp_status fsp_neh(fsp_instance inst, int32_t *perm_out, int32_t *makespan);

/*
 * Serving: a loop of concurrent depth-first searches (fsp_solve semantics
 * each) that share every launch.  Searches are admitted first come first
 * served while a slot and the device-memory budget allow; every call to
 * fsp_server_step then advances each admitted search by one pool step, with
 * the step kernels of all of them in one set of launches and all their
 * children bounded by one merged batched launch (Sec. III-A pools, merged
 * across requests).  Search stacks, step scratch and instance tables stay on
 * the device.  A search's result (optimum, schedule, node and step counts,
 * step fingerprints) depends only on its own (instance, ub0, pool_cap,
 * node_budget), not on what it shared launches with.
 */
typedef struct fsp_server_s *fsp_server;

typedef struct {
    int64_t mem_budget_bytes;  /* device bytes for the admitted searches' stacks
                                  and step buffers plus the server's shared step
                                  scratch (> 0).  Admission counts a search at
                                  its initial size; a step that would grow a
                                  search (stack doubling, larger step buffers)
                                  or the shared scratch past the budget holds
                                  that search back to a later call, and when
                                  every admitted search is held back the one
                                  holding the most device memory ends with
                                  FSP_E_NOMEM.
                                  Per-launch workspace that a bound of child
                                  rows takes and returns within the call is
                                  not counted. */
    int32_t max_active;        /* most searches admitted at once (>= 1) */
    int64_t tick_children;     /* cap on children bounded per step call, summed
                                  over searches (0 = none); searches left out
                                  step first in the next call, and one search
                                  always steps */
} fsp_server_config;

typedef struct {
    int32_t active, pending;   /* admitted searches, searches waiting for admission */
    int64_t mem_used;          /* device bytes held by admitted searches and the
                                  shared step scratch now (<= mem_budget_bytes) */
    int64_t ticks;             /* step calls that advanced at least one search */
    int64_t nodes_bounded;     /* over all searches so far */
    int64_t last_children;     /* children bounded by the last step call */
    int32_t last_searches;     /* searches advanced by the last step call */
    int64_t swap_outs;         /* stacks moved to host memory to let another
                                  search step within the budget, so far */
    int64_t swap_ins;          /* stacks brought back, so far */
} fsp_server_stats;

/* fsp_server_create - cfg host; stream: every launch and copy of the server
 * goes to it.  The server keeps references to the instances it is given:
 * an instance must outlive the searches submitted on it. */
fsp_status fsp_server_create(const fsp_server_config *cfg, void *stream, fsp_server *out);

/* fsp_server_submit - queue a search (arguments as in fsp_solve); id_out host.
 * FSP_E_NOMEM when its initial device memory exceeds the whole budget. */
fsp_status fsp_server_submit(fsp_server srv, fsp_instance inst, int32_t ub0, int64_t pool_cap,
                             int64_t node_budget, int64_t *id_out);

/* fsp_server_step - admit what fits, then one step of every admitted search
 * whose step fits the memory budget (synchronous on the stream).  When no
 * admitted search fits, the stacks of the others are moved to host memory,
 * largest first, until the one that waited longest does; a moved search comes
 * back when its step fits again.  Moving changes no result.  done_ids host (done_cap entries, may be NULL):
 * ids of the searches that finished in this call, *n_done their count (ids
 * beyond done_cap are not listed but can still be polled).  stats may be NULL.
 * An error here leaves every admitted search failed with that status. */
fsp_status fsp_server_step(fsp_server srv, int64_t *done_ids, int32_t done_cap, int32_t *n_done,
                           fsp_server_stats *stats);

/* fsp_server_poll - FSP_PENDING while search id runs or waits; then its
 * fsp_solve status (FSP_OK, FSP_BUDGET, FSP_E_NOMEM when the memory budget
 * could not hold its next step even with every other search's stack moved
 * to host memory, or another error) with res and perm_out
 * (host n, may be NULL) filled, once: the result is then forgotten, and
 * later polls of the id give FSP_E_INVAL. */
fsp_status fsp_server_poll(fsp_server srv, int64_t id, fsp_solve_result *res, int32_t *perm_out);

/* fsp_server_destroy - waits for the stream, frees every search. */
fsp_status fsp_server_destroy(fsp_server srv);

/*
 * Kernel timing (instrumentation).  When enabled on an instance, each bound
 * launch records HIP events on its stream around its decode and scan kernels.
 * fsp_timing_read() waits for the recorded events, returns the summed device
 * time of each kernel in milliseconds and the number of launches, and clears
 * the record.  on = 1 records three events per bound launch (start, after
 * the decode, after the scan).  on = 2 records two: a launch's decode time
 * runs from the previous launch's end, which suits back-to-back launches on
 * one stream (the first launch after enabling or reading has its own start).
 */
fsp_status fsp_timing_enable(fsp_instance inst, int32_t on);
fsp_status fsp_timing_read(fsp_instance inst, double *decode_ms, double *scan_ms, int64_t *launches);

/*
 * fsp_release_cached - memory management (not an operation of the method).
 * Device scratch that calls release is kept for reuse by later calls on the
 * same device and stream (at most 16 GiB), and freed memory stays in the
 * library's pool.  This call waits for every device that holds such memory,
 * frees the kept blocks and trims the pools, returning the memory to the
 * driver.  Calls that run concurrently may keep new blocks afterwards.  A
 * stream whose work used library scratch should be synchronized before it is
 * destroyed.  Returns FSP_OK (at once when the process has allocated
 * nothing) or FSP_E_DEVICE.
 */
fsp_status fsp_release_cached(void);

/*
 * Peak probes (measurement support; not an operation of the method).  Each
 * runs one kernel built to saturate one unit of the current device, three
 * times untimed and five times timed with HIP events on `stream`, and returns
 * the rate and the mean duration (ms, optional) of the timed launches:
 *   FSP_PROBE_VALU16  chains of packed 16-bit max and add, the arithmetic of
 *                     the 16-bit pair scan; rate = 16-bit operations per
 *                     second (a packed instruction counts two);
 *   FSP_PROBE_VALU32  the same chains in 32-bit lanes; operations per second;
 *   FSP_PROBE_LDS     conflict-free 16-byte LDS reads; bytes per second;
 *   FSP_PROBE_HBM     a copy between two device buffers of `bytes` bytes each
 *                     (a multiple of 16, at least 1 MiB), which the call
 *                     allocates and frees; bytes read plus written per second.
 * `bytes` is ignored by the other kinds.  Synchronous on `stream`.  Errors:
 * FSP_E_INVAL (unknown kind, null rate, bad size), FSP_E_NOMEM, FSP_E_DEVICE.
 */
#define FSP_PROBE_VALU16 0
#define FSP_PROBE_VALU32 1
#define FSP_PROBE_LDS 2
#define FSP_PROBE_HBM 3
fsp_status fsp_probe_peak(int32_t kind, int64_t bytes, void *stream, double *rate, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* FSPBB_H */
