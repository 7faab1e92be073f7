/*
 * Oracle for the permutation flow-shop lower bound and branch-and-bound.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library and is written to be read
 * against the paper (Melab, Chakroun, Mezmaz, Tuyttens, "A GPU-accelerated
 * Branch-and-Bound Algorithm for the Flow-Shop Scheduling Problem"), not to be
 * fast.  All arithmetic is integer; sums are carried in int64 so that no
 * intermediate can wrap.
 *
 * Indexing: jobs 0..n-1, machines 0..m-1, processing time of job j on machine
 * k is p[j*m + k] (row-major n x m, the PTM matrix of Table I).
 *
 * Readings of the paper taken here (each is also listed with its reason in the
 * design notes of the repository):
 *   - Machine releases (RM) are the completion times of the scheduled prefix
 *     on each machine; the root has all releases 0.  The "heads" variant
 *     takes RM literally as the earliest starting times of the unscheduled
 *     jobs (Table I, Fig. 2 lines taking a minimum of RM over jobs): the
 *     release of machine k is the least, over unscheduled jobs j, of the time
 *     j would start on k if it were scheduled next.
 *   - The tail of machine l (QM) is the minimum over unscheduled jobs of the
 *     job's total time on machines after l; 0 when no job is unscheduled.
 *   - The lag of job j on pair (k,l) (LM) is its total time on the machines
 *     strictly between k and l.
 *   - Johnson's rule with lags for pair (k,l): with a = p[j][k], b = p[j][l],
 *     L = lag, jobs with a <= b come first by increasing a+L, then jobs with
 *     a > b by decreasing b+L; ties by increasing job id (Johnson 1954;
 *     Mitten 1959 for the lags, as used by Lageweg, Lenstra and Rinnooy Kan).
 *   - The bound starts from 0: Fig. 2 initialises it to the largest integer
 *     and then takes a maximum, which can only be a typo.
 *   - Elimination prunes a node whose bound is >= the upper bound; the
 *     paper's strict ">" is available for the brute-force pins (strict_gt).
 *   - The pair-subset variant takes the maximum of Fig. 2 over a given
 *     subset of the machine pairs (the MM list restricted) instead of all
 *     of them; each pair's value is unchanged, so the bound can only drop.
 *     The searches need a pair ending on the last machine, so that a
 *     complete schedule's bound is its makespan.
 *
 * Parity pins live in tests/test_oracle_pins.py (brute force, closed forms,
 * invariants).  Nothing here is "parity unpinned".
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_INVALID (-1)

/* Counters of accesses to the data structures of Table I, filled by
 * orc_bound_counted() so a test can check the access pattern against the
 * table's "number of accesses" column. */
typedef struct {
    int64_t ptm;  /* reads of processing times inside the pair scans */
    int64_t lm;   /* reads of lags inside the pair scans */
    int64_t rm;   /* reads of machine releases by the pair loop */
    int64_t qm;   /* reads of machine tails by the pair loop */
    int64_t mm;   /* reads of the machine-pair list */
} orc_counts;

/* ---------------------------------------------------------------------------
 * Makespan of a (partial) permutation: completion time of its last job on the
 * last machine (Sec. II-B/II-C: jobs visit machines 1..m in order, one job at
 * a time per machine, same job order on every machine).
 * ------------------------------------------------------------------------- */
static void completion_times(const int32_t *p, int m, const int32_t *seq, int len,
                             int64_t *C /* m, in: start state, out: after seq */)
{
    for (int i = 0; i < len; ++i) {
        const int32_t *row = p + (int64_t)seq[i] * m;
        C[0] += row[0];
        for (int k = 1; k < m; ++k) {
            int64_t ready = C[k] > C[k - 1] ? C[k] : C[k - 1];
            C[k] = ready + row[k];
        }
    }
}

int32_t orc_makespan(const int32_t *p, int n, int m, const int32_t *seq, int len)
{
    (void)n;
    int64_t *C = (int64_t *)calloc((size_t)m, sizeof(int64_t));
    completion_times(p, m, seq, len, C);
    int64_t v = C[m - 1];
    free(C);
    return (int32_t)v;
}

/* Checks a node: 0 <= d <= n, prefix jobs in range and pairwise distinct.
 * Fills scheduled[] (1 = in the prefix).  Returns 1 when valid. */
static int decode_node(int n, const int32_t *prefix, int d, unsigned char *scheduled)
{
    if (d < 0 || d > n) return 0;
    memset(scheduled, 0, (size_t)n);
    for (int i = 0; i < d; ++i) {
        int32_t j = prefix[i];
        if (j < 0 || j >= n || scheduled[j]) return 0;
        scheduled[j] = 1;
    }
    return 1;
}

/* A job with its Johnson-with-lags sort fields for one pair (k,l):
 * group 0 holds the jobs with a <= b, ordered by increasing a+L; group 1 the
 * jobs with a > b, ordered by decreasing b+L; ties by increasing tie key.
 * eq_in_s2 moves the a == b jobs to group 1 and tiekey replaces the job id as
 * tie key; both exist only so a test can show the bound does not depend on
 * these choices. */
typedef struct { int group; int64_t primary; int64_t tie; int32_t job; } keyed_job;

static int cmp_keyed(const void *x, const void *y)
{
    const keyed_job *a = (const keyed_job *)x, *b = (const keyed_job *)y;
    if (a->group != b->group) return a->group < b->group ? -1 : 1;
    if (a->group == 0) {                       /* a+L ascending */
        if (a->primary != b->primary) return a->primary < b->primary ? -1 : 1;
    } else {                                   /* b+L descending */
        if (a->primary != b->primary) return a->primary > b->primary ? -1 : 1;
    }
    if (a->tie != b->tie) return a->tie < b->tie ? -1 : 1;
    return (a->job > b->job) - (a->job < b->job);
}

static int64_t lag(const int32_t *p, int m, int j, int k, int l)
{
    int64_t s = 0;
    for (int h = k + 1; h < l; ++h) s += p[(int64_t)j * m + h];
    return s;
}

static keyed_job johnson_fields(int32_t j, int64_t a, int64_t b, int64_t L, int64_t tie,
                                int eq_in_s2)
{
    keyed_job kj;
    int first = eq_in_s2 ? (a < b) : (a <= b);
    kj.group = first ? 0 : 1;
    kj.primary = first ? (a + L) : (b + L);
    kj.tie = tie;
    kj.job = j;
    return kj;
}

/* Which bound: heads = the heads variant of RM; pairsel = NULL for every
 * machine pair, else an m x m matrix with pairsel[k*m + l] = 1 for the pairs
 * (k,l), k<l, the maximum is taken over. */
typedef struct { int heads; const unsigned char *pairsel; } orc_variant;

/* The lower bound of Sec. II-D (Fig. 2) for the node (prefix[0..d-1]).
 *
 * Each machine pair (k,l), k<l, is relaxed to two machines in series with
 * a lag: every other machine is taken to have unlimited capacity, so a job
 * leaving k reaches l after its time on the machines in between.  The
 * unscheduled jobs run through that two-machine system in Johnson-with-lags
 * order, which minimises its makespan; both machines start at their
 * release.  A job finishes on k when k has finished the job before it, and
 * starts on l once l is free and the job has left k and served its lag.
 * The pair's value is l's finishing time plus the tail of l (the least time
 * any unscheduled job still needs after l); the bound is the largest value
 * over the pairs.  Returns ORC_INVALID for an invalid node. */
static int32_t bound_impl(const int32_t *p, int n, int m, const int32_t *prefix, int d,
                          const int32_t *tiekey, int eq_in_s2, orc_counts *cnt,
                          int only_k, int only_l, int64_t *pair_t2, int64_t *pair_q, const orc_variant *v)
{
    const int heads = v ? v->heads : 0;
    const unsigned char *pairsel = v ? v->pairsel : NULL;
    unsigned char *scheduled = (unsigned char *)malloc((size_t)n + 1);
    if (!decode_node(n, prefix, d, scheduled)) { free(scheduled); return ORC_INVALID; }

    /* RM: completion times of the prefix on each machine. */
    int64_t *r = (int64_t *)calloc((size_t)m, sizeof(int64_t));
    completion_times(p, m, prefix, d, r);

    if (heads) {
        /* RM as earliest starting times: job j scheduled next would start on
         * machine k at max(release of k, completion of j on k-1); the
         * machine's release becomes the least such start over unscheduled j. */
        int64_t *h = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
        int any = 0;
        for (int j = 0; j < n; ++j) {
            if (scheduled[j]) continue;
            int64_t prev_done = 0;  /* completion of j on machine k-1 */
            for (int k = 0; k < m; ++k) {
                int64_t start = r[k] > prev_done ? r[k] : prev_done;
                if (!any || start < h[k]) h[k] = start;
                prev_done = start + p[(int64_t)j * m + k];
            }
            any = 1;
        }
        if (any)
            for (int k = 0; k < m; ++k) r[k] = h[k];
        free(h);
    }

    /* QM: min over unscheduled jobs of the time left after machine l. */
    int64_t *q = (int64_t *)calloc((size_t)m, sizeof(int64_t));
    for (int l = 0; l < m; ++l) {
        int64_t best = -1;
        for (int j = 0; j < n; ++j) {
            if (scheduled[j]) continue;
            int64_t t = 0;
            for (int h = l + 1; h < m; ++h) t += p[(int64_t)j * m + h];
            if (best < 0 || t < best) best = t;
        }
        q[l] = best < 0 ? 0 : best;
    }

    keyed_job *order = (keyed_job *)malloc(sizeof(keyed_job) * (size_t)(n + 1));
    int64_t LB = 0;
    for (int k = 0; k < m; ++k) {
        for (int l = k + 1; l < m; ++l) {
            if (only_k >= 0 && (k != only_k || l != only_l)) continue;
            if (pairsel && !pairsel[k * m + l]) continue;
            if (cnt) cnt->mm += 2;
            /* Johnson-with-lags order of the unscheduled jobs for (k,l). */
            int cnt_u = 0;
            for (int j = 0; j < n; ++j) {
                if (scheduled[j]) continue;
                int64_t a = p[(int64_t)j * m + k], b = p[(int64_t)j * m + l];
                int64_t tie = tiekey ? tiekey[j] : j;
                order[cnt_u++] = johnson_fields(j, a, b, lag(p, m, j, k, l), tie, eq_in_s2);
            }
            qsort(order, (size_t)cnt_u, sizeof(keyed_job), cmp_keyed);

            /* finishing times of the last job so far on k and on l */
            int64_t fin_k = r[k], fin_l = r[l];
            if (cnt) cnt->rm += 2;
            for (int i = 0; i < cnt_u; ++i) {
                int j = order[i].job;
                fin_k += p[(int64_t)j * m + k];
                int64_t arrive = fin_k + lag(p, m, j, k, l);
                int64_t start = arrive > fin_l ? arrive : fin_l;
                fin_l = start + p[(int64_t)j * m + l];
                if (cnt) { cnt->ptm += 2; cnt->lm += 1; }
            }
            if (pair_t2) *pair_t2 = fin_l;
            if (pair_q) *pair_q = q[l];
            int64_t value = fin_l + q[l];
            if (cnt) cnt->qm += 1;
            if (value > LB) LB = value;
        }
    }
    free(order); free(q); free(r); free(scheduled);
    return (int32_t)LB;
}

int32_t orc_bound(const int32_t *p, int n, int m, const int32_t *prefix, int d)
{
    return bound_impl(p, n, m, prefix, d, NULL, 0, NULL, -1, -1, NULL, NULL, NULL);
}

/* The bound with the heads variant of RM (see the header). */
int32_t orc_bound_heads(const int32_t *p, int n, int m, const int32_t *prefix, int d)
{
    const orc_variant v = {1, NULL};
    return bound_impl(p, n, m, prefix, d, NULL, 0, NULL, -1, -1, NULL, NULL, &v);
}

/* Same bound with a custom tie-break key per job and a choice of group for
 * the a == b jobs. */
int32_t orc_bound_tie(const int32_t *p, int n, int m, const int32_t *prefix, int d,
                      const int32_t *tiekey, int eq_in_s2)
{
    return bound_impl(p, n, m, prefix, d, tiekey, eq_in_s2, NULL, -1, -1, NULL, NULL, NULL);
}

/* Same bound, counting accesses to the Table I structures. */
int32_t orc_bound_counted(const int32_t *p, int n, int m, const int32_t *prefix, int d,
                          orc_counts *cnt)
{
    memset(cnt, 0, sizeof(*cnt));
    return bound_impl(p, n, m, prefix, d, NULL, 0, cnt, -1, -1, NULL, NULL, NULL);
}

/* One pair only: *t2 = finishing time on l after the scan (before the tail), *q = tail
 * of machine l.  Returns ORC_INVALID for an invalid node, else 0. */
int32_t orc_pair_scan(const int32_t *p, int n, int m, const int32_t *prefix, int d,
                      int k, int l, int64_t *t2, int64_t *q)
{
    if (k < 0 || l <= k || l >= m) return ORC_INVALID;
    int32_t v = bound_impl(p, n, m, prefix, d, NULL, 0, NULL, k, l, t2, q, NULL);
    return v == ORC_INVALID ? ORC_INVALID : 0;
}

/* Bounds of a pool: prefixes is count x n (row i holds depths[i] scheduled
 * jobs first), out[i] = bound or ORC_INVALID.  Returns the number of invalid
 * rows. */
static int64_t bound_pool_v(const int32_t *p, int n, int m, const int32_t *prefixes, const int32_t *depths,
                            int64_t count, int32_t *out, const orc_variant *v)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < count; ++i) {
        out[i] = bound_impl(p, n, m, prefixes + i * (int64_t)n, depths[i], NULL, 0, NULL, -1, -1, NULL, NULL, v);
        if (out[i] == ORC_INVALID) ++bad;
    }
    return bad;
}

int64_t orc_bound_pool_mode(const int32_t *p, int n, int m, const int32_t *prefixes,
                            const int32_t *depths, int64_t count, int32_t *out, int heads)
{
    const orc_variant v = {heads, NULL};
    return bound_pool_v(p, n, m, prefixes, depths, count, out, &v);
}

/* The pair-subset matrix of npairs pairs (pairs[2i], pairs[2i+1]) = (k, l);
 * NULL (every pair) when npairs <= 0.  The caller frees it. */
static unsigned char *pair_matrix(int m, const int32_t *pairs, int npairs)
{
    if (!pairs || npairs <= 0) return NULL;
    unsigned char *sel = (unsigned char *)calloc((size_t)m * (size_t)m, 1);
    for (int i = 0; i < npairs; ++i) {
        int k = pairs[2 * i], l = pairs[2 * i + 1];
        if (k >= 0 && k < l && l < m) sel[k * m + l] = 1;
    }
    return sel;
}

/* Bounds of a pool with the maximum over the given machine pairs only. */
int64_t orc_bound_pool_pairs(const int32_t *p, int n, int m, const int32_t *prefixes, const int32_t *depths,
                             int64_t count, int32_t *out, int heads, const int32_t *pairs, int npairs)
{
    unsigned char *sel = pair_matrix(m, pairs, npairs);
    const orc_variant v = {heads, sel};
    int64_t bad = bound_pool_v(p, n, m, prefixes, depths, count, out, &v);
    free(sel);
    return bad;
}

int64_t orc_bound_pool(const int32_t *p, int n, int m, const int32_t *prefixes,
                       const int32_t *depths, int64_t count, int32_t *out)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < count; ++i) {
        out[i] = orc_bound(p, n, m, prefixes + i * (int64_t)n, depths[i]);
        if (out[i] == ORC_INVALID) ++bad;
    }
    return bad;
}

/* ---------------------------------------------------------------------------
 * Brute force: minimum makespan over all completions of a prefix (n small).
 * ------------------------------------------------------------------------- */
static void brute_rec(const int32_t *p, int n, int m, unsigned char *used, int left,
                      const int64_t *C, int64_t *best)
{
    if (left == 0) {
        if (*best < 0 || C[m - 1] < *best) *best = C[m - 1];
        return;
    }
    int64_t *D = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    for (int j = 0; j < n; ++j) {
        if (used[j]) continue;
        memcpy(D, C, sizeof(int64_t) * (size_t)m);
        int32_t seq = j;
        completion_times(p, m, &seq, 1, D);
        used[j] = 1;
        brute_rec(p, n, m, used, left - 1, D, best);
        used[j] = 0;
    }
    free(D);
}

int32_t orc_brute(const int32_t *p, int n, int m, const int32_t *prefix, int d)
{
    unsigned char *used = (unsigned char *)malloc((size_t)n + 1);
    if (!decode_node(n, prefix, d, used)) { free(used); return ORC_INVALID; }
    int64_t *C = (int64_t *)calloc((size_t)m, sizeof(int64_t));
    completion_times(p, m, prefix, d, C);
    int64_t best = -1;
    brute_rec(p, n, m, used, n - d, C, &best);
    free(C); free(used);
    return (int32_t)best;
}

/* ---------------------------------------------------------------------------
 * NEH constructive heuristic (Nawaz, Enscore and Ham, 1983) for the initial
 * upper bound: order jobs by decreasing total processing time (ties: smaller
 * id first); insert each job, in that order, at the position of the partial
 * sequence that gives the smallest partial makespan (ties: earliest
 * position).  Returns the makespan; perm_out receives the sequence.
 * ------------------------------------------------------------------------- */
int32_t orc_neh(const int32_t *p, int n, int m, int32_t *perm_out)
{
    int32_t *jobs = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *tot = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int j = 0; j < n; ++j) {
        jobs[j] = j;
        tot[j] = 0;
        for (int k = 0; k < m; ++k) tot[j] += p[(int64_t)j * m + k];
    }
    /* insertion sort by (total desc, id asc): plain and stable */
    for (int i = 1; i < n; ++i) {
        int32_t x = jobs[i];
        int t = i - 1;
        while (t >= 0 && (tot[jobs[t]] < tot[x] || (tot[jobs[t]] == tot[x] && jobs[t] > x))) {
            jobs[t + 1] = jobs[t];
            --t;
        }
        jobs[t + 1] = x;
    }
    int32_t *seq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *trial = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int len = 0;
    for (int i = 0; i < n; ++i) {
        int32_t x = jobs[i];
        int best_pos = 0;
        int32_t best_val = 0;
        for (int pos = 0; pos <= len; ++pos) {
            int t = 0;
            for (int a = 0; a < pos; ++a) trial[t++] = seq[a];
            trial[t++] = x;
            for (int a = pos; a < len; ++a) trial[t++] = seq[a];
            int32_t v = orc_makespan(p, n, m, trial, len + 1);
            if (pos == 0 || v < best_val) { best_val = v; best_pos = pos; }
        }
        for (int a = len; a > best_pos; --a) seq[a] = seq[a - 1];
        seq[best_pos] = x;
        ++len;
    }
    int32_t ms = orc_makespan(p, n, m, seq, n);
    if (perm_out) memcpy(perm_out, seq, sizeof(int32_t) * (size_t)n);
    free(trial); free(seq); free(tot); free(jobs);
    return ms;
}

/* ---------------------------------------------------------------------------
 * Branch-and-bound, pool-synchronous depth-first (Sec. II-A operators; the
 * pool of Sec. III-A).  The paper does not fix the order semantics of a pool,
 * so they are fixed here so that node counts are a function of
 * (instance, ub0, pool_cap):
 *   1. The root is bounded (1 node).  If it is eliminated, stop.
 *   2. Selection: pop parents from the top of the stack while the stack is
 *      not empty and the children gathered so far plus the next parent's
 *      (n - depth) children fit in pool_cap (the first parent is always
 *      taken).
 *   3. Branching: for each parent in pop order, one child per unscheduled
 *      job in increasing job id; the child appends that job to the prefix
 *      (forward branching, Sec. II-B).
 *   4. Bounding: every child is bounded; nodes_bounded counts them.
 *   5. Complete children (depth n) are scanned in child order; a bound below
 *      the upper bound replaces it and its permutation becomes the incumbent.
 *   6. Elimination: the remaining children whose bound is below the upper
 *      bound after step 5 (not eliminated) are pushed in reverse child order,
 *      so the first child is on top.
 *   7. Stop when the stack is empty (proven) or nodes_bounded has reached
 *      node_budget (not proven).
 * strict_gt = 1 eliminates only bound > UB (the paper's wording); the default
 * eliminates bound >= UB.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t ub;
    int32_t proven;
    int64_t nodes_bounded;
    int64_t steps;
    int64_t improvements;
    int64_t max_stack;
    /* Wall time of the search and of its bounding (step 4, and the root's
     * bound) alone: the share of the search spent bounding, which the paper
     * gives for its sequential B&B (Sec. I).  Depth-first search only. */
    double seconds_total;
    double seconds_bound;
} orc_bnb_result;

static double now_seconds(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* steplog, when non-NULL, receives per step (up to steplog_cap steps):
 *   [0] parents popped, [1] children bounded, [2] UB after the step,
 *   [3] children pushed, [4] stack size after the step,
 *   [5] sum over pushed children of (position in push order + 1) * (job
 *       appended + 1), a cheap order-sensitive fingerprint of the frontier. */
static int bnb_dfs(const int32_t *p, int n, int m, int32_t ub0, const int32_t *inc0,
                   int64_t pool_cap, int64_t node_budget, int strict_gt,
                   orc_bnb_result *res, int32_t *incumbent_out,
                   int64_t *steplog, int64_t steplog_cap, const orc_variant *v)
{
    memset(res, 0, sizeof(*res));
    if (n < 1 || m < 2 || pool_cap < 1) return -1;
    const double t_start = now_seconds();
    double t_bound = 0.0;
    int32_t UB = ub0;
    int32_t *inc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int have_inc = 0;
    if (inc0) { memcpy(inc, inc0, sizeof(int32_t) * (size_t)n); have_inc = 1; }

    int64_t cap_nodes = 1024, top = 0;
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1) * (size_t)cap_nodes);
    /* node layout: [depth, job_0 .. job_{n-1}] */
#define NODE(i) (stack + (int64_t)(i) * (n + 1))

    int64_t nodes = 1;
    double t0 = now_seconds();
    int32_t root_lb = bound_impl(p, n, m, NULL, 0, NULL, 0, NULL, -1, -1, NULL, NULL, v);
    t_bound += now_seconds() - t0;
    int pruned_root = strict_gt ? (root_lb > UB) : (root_lb >= UB);
    if (!pruned_root) {
        NODE(0)[0] = 0;
        top = 1;
    }
    int64_t steps = 0, improvements = 0, max_stack = top;
    int32_t *children = NULL, *lbs = NULL;
    int64_t child_cap = 0;
    unsigned char *sched = (unsigned char *)malloc((size_t)n);

    while (top > 0 && nodes < node_budget) {
        /* 2. selection */
        int64_t first = top, nchild = 0;
        while (first > 0) {
            int32_t dtop = NODE(first - 1)[0];
            int64_t c = n - dtop;
            if (first < top && nchild + c > pool_cap) break;
            nchild += c;
            --first;
        }
        int64_t npar = top - first;
        if (nchild > child_cap) {
            child_cap = nchild;
            children = (int32_t *)realloc(children, sizeof(int32_t) * (size_t)(n + 1) * (size_t)child_cap);
            lbs = (int32_t *)realloc(lbs, sizeof(int32_t) * (size_t)child_cap);
        }
        /* 3. branching, parents in pop order (top of stack first) */
        int64_t c = 0;
        for (int64_t t = top - 1; t >= first; --t) {
            int32_t *par = NODE(t);
            int32_t d = par[0];
            memset(sched, 0, (size_t)n);
            for (int i = 0; i < d; ++i) sched[par[1 + i]] = 1;
            for (int j = 0; j < n; ++j) {
                if (sched[j]) continue;
                int32_t *ch = children + c * (n + 1);
                ch[0] = d + 1;
                memcpy(ch + 1, par + 1, sizeof(int32_t) * (size_t)d);
                ch[1 + d] = j;
                ++c;
            }
        }
        top = first;
        /* 4. bounding */
        t0 = now_seconds();
        for (int64_t i = 0; i < nchild; ++i) {
            int32_t *ch = children + i * (n + 1);
            lbs[i] = bound_impl(p, n, m, ch + 1, ch[0], NULL, 0, NULL, -1, -1, NULL, NULL, v);
        }
        t_bound += now_seconds() - t0;
        nodes += nchild;
        /* 5. complete children update the upper bound */
        int improved = 0;
        for (int64_t i = 0; i < nchild; ++i) {
            int32_t *ch = children + i * (n + 1);
            if (ch[0] == n && lbs[i] < UB) {
                UB = lbs[i];
                memcpy(inc, ch + 1, sizeof(int32_t) * (size_t)n);
                have_inc = 1;
                improved = 1;
            }
        }
        improvements += improved;  /* steps that lowered the upper bound */
        /* 6. elimination and push in reverse child order */
        int64_t pushed = 0, fp = 0;
        for (int64_t i = nchild - 1; i >= 0; --i) {
            int32_t *ch = children + i * (n + 1);
            if (ch[0] == n) continue;
            int keep = strict_gt ? !(lbs[i] > UB) : (lbs[i] < UB);
            if (!keep) continue;
            if (top >= cap_nodes) {
                cap_nodes *= 2;
                stack = (int32_t *)realloc(stack, sizeof(int32_t) * (size_t)(n + 1) * (size_t)cap_nodes);
            }
            memcpy(NODE(top), ch, sizeof(int32_t) * (size_t)(n + 1));
            ++top;
            ++pushed;
            fp += pushed * (int64_t)(ch[ch[0]] + 1);
        }
        if (top > max_stack) max_stack = top;
        if (steplog && steps < steplog_cap) {
            int64_t *s = steplog + steps * 6;
            s[0] = npar; s[1] = nchild; s[2] = UB; s[3] = pushed; s[4] = top; s[5] = fp;
        }
        ++steps;
    }
#undef NODE
    res->ub = UB;
    res->proven = (top == 0);
    res->nodes_bounded = nodes;
    res->steps = steps;
    res->improvements = improvements;
    res->max_stack = max_stack;
    if (incumbent_out) {
        if (have_inc) memcpy(incumbent_out, inc, sizeof(int32_t) * (size_t)n);
        else for (int j = 0; j < n; ++j) incumbent_out[j] = -1;
    }
    free(sched); free(children); free(lbs); free(stack); free(inc);
    res->seconds_total = now_seconds() - t_start;
    res->seconds_bound = t_bound;
    return 0;
}

/* ---------------------------------------------------------------------------
 * Best-first branch-and-bound, pool-synchronous (Sec. III-A: the GPU-side
 * experiments select the sub-problems of a pool best first).  The frontier
 * holds nodes with their bound and an insertion number, ordered by (bound,
 * insertion number).  Each step:
 *   1. drops the frontier nodes whose bound is >= UB (> UB with strict_gt);
 *   2. takes parents from the front of the order while the children gathered
 *      so far plus the next parent's n - d children fit in pool_cap (the first
 *      parent is always taken);
 *   3-5. branches the parents in that order (children in increasing appended
 *      job), bounds every child and lowers UB with the best complete child,
 *      the first in child order on ties, exactly as the depth-first search;
 *   6. inserts the non-complete children whose bound is below UB, in child
 *      order, with the next insertion numbers.
 * The search stops when the frontier is empty after step 1 (proven) or, if
 * not, when nodes_bounded has reached node_budget.  The result's max_stack is
 * the largest frontier; steplog as for orc_bnb with [4] = frontier size after
 * the step and [5] = sum over inserted children of (S - rank) * (appended job
 * + 1), rank in child order, S the number inserted.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t lb;
    int64_t seq;
    int32_t *node;  /* [depth, job_0 .. job_{n-1}] */
} bf_node;

static int cmp_bf(const void *x, const void *y)
{
    const bf_node *a = (const bf_node *)x, *b = (const bf_node *)y;
    if (a->lb != b->lb) return a->lb < b->lb ? -1 : 1;
    return a->seq < b->seq ? -1 : (a->seq > b->seq ? 1 : 0);
}

static int bnb_best(const int32_t *p, int n, int m, int32_t ub0, const int32_t *inc0,
                    int64_t pool_cap, int64_t node_budget, int strict_gt,
                    orc_bnb_result *res, int32_t *incumbent_out,
                    int64_t *steplog, int64_t steplog_cap, const orc_variant *v)
{
    memset(res, 0, sizeof(*res));
    if (n < 1 || m < 2 || pool_cap < 1) return -1;
    int32_t UB = ub0;
    int32_t *inc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int have_inc = 0;
    if (inc0) { memcpy(inc, inc0, sizeof(int32_t) * (size_t)n); have_inc = 1; }

    int64_t M = 0, capF = 16, seq = 0;
    bf_node *F = (bf_node *)malloc(sizeof(bf_node) * (size_t)capF);
    int64_t nodes = 1;
    int32_t root_lb = bound_impl(p, n, m, NULL, 0, NULL, 0, NULL, -1, -1, NULL, NULL, v);
    if (!(strict_gt ? (root_lb > UB) : (root_lb >= UB))) {
        F[0].lb = root_lb;
        F[0].seq = seq++;
        F[0].node = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
        M = 1;
    }
    int64_t steps = 0, improvements = 0, max_front = M;
    int32_t *children = NULL, *lbs = NULL;
    int64_t child_cap = 0;
    unsigned char *sched = (unsigned char *)malloc((size_t)n);

    for (;;) {
        /* 1. drop the nodes the upper bound eliminates */
        int64_t w = 0;
        for (int64_t i = 0; i < M; ++i) {
            int gone = strict_gt ? (F[i].lb > UB) : (F[i].lb >= UB);
            if (gone) free(F[i].node);
            else F[w++] = F[i];
        }
        M = w;
        if (M == 0 || nodes >= node_budget) break;
        qsort(F, (size_t)M, sizeof(bf_node), cmp_bf);

        /* 2. selection from the front */
        int64_t K = 0, nchild = 0;
        while (K < M) {
            int64_t c = n - F[K].node[0];
            if (K > 0 && nchild + c > pool_cap) break;
            nchild += c;
            ++K;
        }
        if (nchild > child_cap) {
            child_cap = nchild;
            children = (int32_t *)realloc(children, sizeof(int32_t) * (size_t)(n + 1) * (size_t)child_cap);
            lbs = (int32_t *)realloc(lbs, sizeof(int32_t) * (size_t)child_cap);
        }
        /* 3. branching in selection order */
        int64_t c = 0;
        for (int64_t k = 0; k < K; ++k) {
            int32_t *par = F[k].node;
            int32_t d = par[0];
            memset(sched, 0, (size_t)n);
            for (int i = 0; i < d; ++i) sched[par[1 + i]] = 1;
            for (int j = 0; j < n; ++j) {
                if (sched[j]) continue;
                int32_t *ch = children + c * (n + 1);
                ch[0] = d + 1;
                memcpy(ch + 1, par + 1, sizeof(int32_t) * (size_t)d);
                ch[1 + d] = j;
                ++c;
            }
        }
        for (int64_t k = 0; k < K; ++k) free(F[k].node);
        memmove(F, F + K, sizeof(bf_node) * (size_t)(M - K));
        M -= K;
        /* 4. bounding */
        for (int64_t i = 0; i < nchild; ++i) {
            int32_t *ch = children + i * (n + 1);
            lbs[i] = bound_impl(p, n, m, ch + 1, ch[0], NULL, 0, NULL, -1, -1, NULL, NULL, v);
        }
        nodes += nchild;
        /* 5. complete children update the upper bound */
        int improved = 0;
        for (int64_t i = 0; i < nchild; ++i) {
            int32_t *ch = children + i * (n + 1);
            if (ch[0] == n && lbs[i] < UB) {
                UB = lbs[i];
                memcpy(inc, ch + 1, sizeof(int32_t) * (size_t)n);
                have_inc = 1;
                improved = 1;
            }
        }
        improvements += improved;
        /* 6. insertion in child order */
        int64_t S = 0;
        for (int64_t i = 0; i < nchild; ++i) {
            int32_t *ch = children + i * (n + 1);
            if (ch[0] < n && (strict_gt ? !(lbs[i] > UB) : (lbs[i] < UB))) ++S;
        }
        int64_t rank = 0, fp = 0;
        for (int64_t i = 0; i < nchild; ++i) {
            int32_t *ch = children + i * (n + 1);
            if (!(ch[0] < n && (strict_gt ? !(lbs[i] > UB) : (lbs[i] < UB)))) continue;
            if (M >= capF) {
                capF *= 2;
                F = (bf_node *)realloc(F, sizeof(bf_node) * (size_t)capF);
            }
            F[M].lb = lbs[i];
            F[M].seq = seq++;
            F[M].node = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
            memcpy(F[M].node, ch, sizeof(int32_t) * (size_t)(n + 1));
            ++M;
            fp += (S - rank) * (int64_t)(ch[ch[0]] + 1);
            ++rank;
        }
        if (M > max_front) max_front = M;
        if (steplog && steps < steplog_cap) {
            int64_t *s = steplog + steps * 6;
            s[0] = K; s[1] = nchild; s[2] = UB; s[3] = S; s[4] = M; s[5] = fp;
        }
        ++steps;
    }
    res->ub = UB;
    res->proven = (M == 0);
    res->nodes_bounded = nodes;
    res->steps = steps;
    res->improvements = improvements;
    res->max_stack = max_front;
    if (incumbent_out) {
        if (have_inc) memcpy(incumbent_out, inc, sizeof(int32_t) * (size_t)n);
        else for (int j = 0; j < n; ++j) incumbent_out[j] = -1;
    }
    for (int64_t i = 0; i < M; ++i) free(F[i].node);
    free(F); free(sched); free(children); free(lbs); free(inc);
    return 0;
}

/* The searches with the plain bound (heads = 0) or the heads variant, over
 * every machine pair. */
int orc_bnb(const int32_t *p, int n, int m, int32_t ub0, const int32_t *inc0,
            int64_t pool_cap, int64_t node_budget, int strict_gt,
            orc_bnb_result *res, int32_t *incumbent_out,
            int64_t *steplog, int64_t steplog_cap, int heads)
{
    const orc_variant v = {heads, NULL};
    return bnb_dfs(p, n, m, ub0, inc0, pool_cap, node_budget, strict_gt, res, incumbent_out, steplog,
                   steplog_cap, &v);
}

int orc_bnb_best_first(const int32_t *p, int n, int m, int32_t ub0, const int32_t *inc0,
                       int64_t pool_cap, int64_t node_budget, int strict_gt,
                       orc_bnb_result *res, int32_t *incumbent_out,
                       int64_t *steplog, int64_t steplog_cap, int heads)
{
    const orc_variant v = {heads, NULL};
    return bnb_best(p, n, m, ub0, inc0, pool_cap, node_budget, strict_gt, res, incumbent_out, steplog,
                    steplog_cap, &v);
}

/* Either search (best_first = 0: depth first) with the bound over the given
 * machine pairs only (npairs <= 0: every pair). */
int orc_bnb_pairs(const int32_t *p, int n, int m, int32_t ub0, const int32_t *inc0,
                  int64_t pool_cap, int64_t node_budget, int strict_gt,
                  orc_bnb_result *res, int32_t *incumbent_out,
                  int64_t *steplog, int64_t steplog_cap, int heads, int best_first,
                  const int32_t *pairs, int npairs)
{
    /* a complete schedule's bound must be its makespan: some pair ends on
     * the last machine */
    int last = 0;
    for (int i = 0; pairs && i < npairs; ++i) last |= pairs[2 * i + 1] == m - 1;
    if (npairs > 0 && !last) return -1;
    unsigned char *sel = pair_matrix(m, pairs, npairs);
    const orc_variant v = {heads, sel};
    int r = best_first ? bnb_best(p, n, m, ub0, inc0, pool_cap, node_budget, strict_gt, res, incumbent_out,
                                  steplog, steplog_cap, &v)
                       : bnb_dfs(p, n, m, ub0, inc0, pool_cap, node_budget, strict_gt, res, incumbent_out,
                                 steplog, steplog_cap, &v);
    free(sel);
    return r;
}
