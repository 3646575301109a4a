/*
 * bx.h -- C ABI of the MI355X (gfx950) UTIL-table engine.
 *
 * The engine computes, on one GPU, the bucket functions ("UTIL tables") of
 * Bucket Elimination (BE), Mini-Bucket Elimination (MBE) and DPOP, and the
 * value assignment that follows them, for weighted constraint problems,
 * DCOPs (agents simulated on the GPU) and MPE on belief networks, after
 * Fioretto, Pontelli, Yeoh, Dechter, "Accelerating Exact and Approximate
 * Inference for (Distributed) Discrete Optimization with GPUs":
 *   - problem model <X, D, C>, cost functions into R+ u {inf}: Sec. 2;
 *   - BE, Alg. 1 (Sec. 2.1); MBE with a bound on mini-bucket scopes, Alg. 2
 *     (Sec. 2.2); DPOP / pseudo-trees, Sec. 2 (Def. 2) and Sec. 4.1;
 *     MPE, Sec. 3;
 *   - bucket-tables as flat cost arrays in lexicographic row order, Sec. 6.1;
 *   - aggregation (Sec. 6.3, Eq. (3)) and elimination (Sec. 6.4), which the
 *     engine fuses into one pass per table.
 *
 * Conventions for every entry point:
 *   - Return value: BX_OK (0) or a negative bx_status.  No call aborts, throws
 *     or exits; the message of the last failure on the calling thread is
 *     returned by bx_last_error().
 *   - Host pointers passed IN are read during the call only (the library
 *     copies what it keeps).  Handles (bx_problem, bx_plan) are owned by the
 *     library and released by the matching *_destroy, which accept NULL.
 *   - Device memory is owned by the caller: the library never allocates device
 *     memory.  A plan states how many workspace bytes it needs; the caller
 *     passes a device buffer of at least that size (256-byte aligned).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued asynchronously on it.
 *   - Integer costs: int32 in [0, BX_INF_I32]; BX_INF_I32 = INT32_MAX is
 *     infinity (a forbidden combination, Sec. 2) and sums saturate there, so
 *     integer results are exact and independent of summation order.
 *   - Float costs: float32 in [0, +inf].
 *   - Tables are flat and row-major over the scope AS GIVEN: scope[0] is the
 *     most significant digit, scope[arity-1] varies fastest (Sec. 6.1).
 *   - Orders: order[p] is the variable at position p; elimination visits
 *     positions n-1 down to 0 (Alg. 1: i = n downto 1), value assignment
 *     visits 0 up to n-1.
 */
#ifndef BX_H
#define BX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BX_INF_I32 2147483647

typedef enum {
    BX_OK = 0,
    BX_E_INVALID = -1,     /* malformed argument (message says which)            */
    BX_E_NOMEM = -2,       /* host allocation failed, or workspace too small     */
    BX_E_TOO_LARGE = -3,   /* a table exceeds the plan's size limit (Sec. 8: oom) */
    BX_E_DEVICE = -4,      /* a HIP runtime call failed                          */
    BX_E_UNSUPPORTED = -5, /* valid request outside what the library implements */
    BX_E_STATE = -6        /* call out of sequence (e.g. results before execute) */
} bx_status;

typedef enum { BX_COST_I32 = 0, BX_COST_F32 = 1 } bx_cost_type;

/* BE and DPOP are exact; MBE and ADPOP bound every mini-bucket's scope by
 * `ibound` variables, the eliminated one included.  DPOP / ADPOP eliminate
 * along the pre-order of a pseudo-tree (Sec. 4.1, 4.2).
 * BE_SUM / MBE_SUM: the sum-product variant of Sec. 10 (weighted counting,
 * partition function, probability of evidence), BX_COST_F32 problems only:
 * eliminating x maps a(s, x) to -ln sum_x exp(-a(s, x)), so BE_SUM's bound
 * is -ln Z, Z = sum over all assignments of prod exp(-cost) (for tables
 * given as probabilities, prod p).  MBE_SUM sums in the first mini-bucket
 * of each bucket and minimises in the others: a lower bound of -ln Z.  A
 * variable in no function's scope adds -ln |D_v| to the bound.  The value
 * phase is the usual one (least bucket cost); the cost of its assignment is
 * an upper bound of -ln Z. */
typedef enum { BX_ALGO_BE = 0, BX_ALGO_MBE = 1, BX_ALGO_DPOP = 2, BX_ALGO_ADPOP = 3,
               BX_ALGO_BE_SUM = 4, BX_ALGO_MBE_SUM = 5 } bx_algo;

/* Order used when the problem carries none.
 *   MIN_DEGREE: repeatedly eliminate the variable with the fewest neighbours
 *               in the current induced graph (ties: lowest id);
 *   MIN_FILL:   fewest fill edges (ties: fewest neighbours, then lowest id);
 *   DFS:        pre-order of a DFS pseudo-tree rooted at the highest-degree
 *               vertex, children by decreasing degree (ties: lowest id);
 *   DEGREE_SORT: the paper's rule of Sec. 6.2 (x precedes y when x has
 *               fewer neighbours; ties: lowest id). */
typedef enum {
    BX_ORDER_MIN_DEGREE = 0, BX_ORDER_MIN_FILL = 1, BX_ORDER_DFS = 2, BX_ORDER_DEGREE_SORT = 3
} bx_order_heuristic;

/* How an over-full bucket is split into mini-buckets (the partition step of Alg. 2).
 *   GREEDY: functions sorted by (decreasing arity, increasing id) go first-fit
 *           into mini-buckets tried in creation order;
 *   LEARNED: candidates scored by a caller-supplied scorer, greedy kept when
 *           no candidate scores better (bx_plan_create_chooser,
 *           bx_plan_create_learned). */
typedef enum { BX_PART_GREEDY = 0, BX_PART_LEARNED = 1 } bx_partition;

/* Device schedule of the UTIL phase.
 *   PER_BUCKET: one launch per mini-bucket, in elimination order;
 *   LEVEL:      one launch per dependency level (all instances, all
 *               independent mini-buckets of the level);
 *   DATAFLOW:   one persistent launch for the whole phase, a tile starting as
 *               soon as the tables it reads are complete -- disabled in this
 *               build: returns BX_E_UNSUPPORTED;
 *   AUTO:       the autotuned choice (bx_plan_autotune), LEVEL until tuned. */
typedef enum { BX_SCHED_PER_BUCKET = 0, BX_SCHED_LEVEL = 1, BX_SCHED_DATAFLOW = 2,
               BX_SCHED_AUTO = 3 } bx_schedule;

typedef struct bx_problem bx_problem;
typedef struct bx_plan bx_plan;

/* bx_options.flags.  Every flag changes only how the same rows are computed,
 * never the results (comparisons and tests):
 *   NO_BLOCKING:  every mini-bucket uses the one-row-per-slot loop (no
 *                 register blocking over box variables);
 *   FORCE_NT:     the register-blocked rows of every level are stored
 *                 non-temporally (otherwise the autotuner's choice; plain
 *                 until tuned);
 *   STAGE_ALWAYS: every level runs the tiled kernel that stages small lane
 *                 tables in LDS (where a tile qualifies);
 *   STAGE_NEVER:  no level stages (STAGE_ALWAYS wins if both are set);
 *   NO_PACKING:   small mini-buckets are not packed several to a workgroup
 *                 nor fused with their packed neighbours of the bucket tree
 *                 (each takes its own tiles and dependency level);
 *   XCD_ORDER:    every level takes its tiles XCD by XCD (workgroup b runs
 *                 on XCD b mod 8, which takes the (b mod 8)-th contiguous
 *                 part of the level's tiles; otherwise the autotuner's
 *                 choice per level, list order until tuned). */
#define BX_FLAG_NO_BLOCKING 0x1u
#define BX_FLAG_FORCE_NT 0x2u
#define BX_FLAG_STAGE_ALWAYS 0x4u
#define BX_FLAG_STAGE_NEVER 0x8u
#define BX_FLAG_NO_PACKING 0x10u
#define BX_FLAG_XCD_ORDER 0x20u
#define BX_FLAG_ALL 0x3fu

typedef struct {
    bx_algo algo;
    int32_t ibound;              /* MBE/ADPOP: max variables per mini-bucket (>= 1) */
    bx_order_heuristic order;    /* used when the problem has no order / pseudo-tree */
    bx_partition partition;
    bx_schedule schedule;
    int64_t max_table_entries;   /* size limit per table; 0 = 2^31 - 1           */
    uint32_t flags;              /* BX_FLAG_* bits; others must be 0              */
    const char *tune_cache;      /* autotuner results keyed by the plan's shape
                                    class: NULL keeps them in this process only;
                                    else a text file read at bx_plan_autotune and
                                    extended with every newly tuned class       */
    /* Packing of small mini-buckets (0 = the library's default for each):
     * a mini-bucket of at most pack_max_rows output rows (and at most 65536
     * whatever the limit) is packed; packed
     * neighbours of the bucket tree are fused into one workgroup's stages
     * while the group holds at most fuse_max_rows rows, fuse_max_stage_rows
     * rows per stage and fuse_max_stages stages (1: no fusion); a packed tile
     * aims at pack_stage_rows rows per stage. */
    int32_t pack_max_rows;
    int32_t fuse_max_rows;
    int32_t fuse_max_stages;
    int32_t fuse_max_stage_rows;
    int32_t pack_stage_rows;
} bx_options;

/* Fills `opt` with: BE, ibound 0, MIN_FILL, GREEDY, AUTO, no extra limit,
 * no flags, no tuning-cache file, default packing. */
void bx_options_default(bx_options *opt);

/* ---------------------------------------------------------------- problems */

/* A problem with n_vars variables; domain_sizes[i] >= 1 is |D_{x_i}| (Sec. 2).
 * Errors: BX_E_INVALID for n_vars < 0, a NULL pointer with n_vars > 0, or a
 * domain size < 1. */
bx_status bx_problem_create(int32_t n_vars, const int32_t *domain_sizes,
                            bx_cost_type cost_type, bx_problem **out);

/* Adds one cost function f: scope -> costs (Sec. 2).  `scope` lists `arity`
 * distinct variable ids; `table` holds n_entries = prod |D| costs in the
 * layout described at the top (int32 for BX_COST_I32, float for BX_COST_F32).
 * arity 0 is a constant.  Errors: BX_E_INVALID for a repeated or out-of-range
 * variable, a wrong n_entries, a negative / NaN cost. */
bx_status bx_problem_add_function(bx_problem *p, int32_t arity, const int32_t *scope,
                                  const void *table, int64_t n_entries);

/* MPE front end (Sec. 3): adds a conditional probability table given as
 * float64 probabilities in [0, 1] over `scope` (same layout); stored as
 * float32 costs -ln p rounded to nearest (p = 0 -> +inf).  BX_COST_F32 only. */
bx_status bx_problem_add_prob_table(bx_problem *p, int32_t arity, const int32_t *scope,
                                    const double *probs, int64_t n_entries);

/* Fixes the elimination order (a permutation of 0..n-1, see top). */
bx_status bx_problem_set_order(bx_problem *p, const int32_t *order);

/* Fixes a pseudo-tree (Sec. 2, Def. 2): parent[v] = parent of v, -1 for roots.
 * Rejected with BX_E_INVALID unless it is a forest in which every pair of
 * variables sharing a function lies on one root-to-leaf branch.  DPOP and
 * ADPOP eliminate along its pre-order (children by increasing id). */
bx_status bx_problem_set_pseudotree(bx_problem *p, const int32_t *parent);

int32_t bx_problem_num_vars(const bx_problem *p);
void bx_problem_destroy(bx_problem *p);

/* Order the library would use under heuristic h (host only, no device). */
bx_status bx_compute_order(const bx_problem *p, bx_order_heuristic h, int32_t *order_out,
                           int32_t *parent_out /* may be NULL; DFS only */);

/* Induced width of `order` (Sec. 2, Def. 1). */
bx_status bx_induced_width(const bx_problem *p, const int32_t *order, int32_t *width_out);

/* -------------------------------------------------------------------- plans */

/* Builds, on the host, the plan for solving n_probs problems together: the
 * orders, normalised tables (scope sorted so that the eliminated variable is
 * last, Sec. 6.1 / 6.2), buckets (Alg. 1), mini-bucket partitions (the
 * partition step of Alg. 2), stride descriptors (the data of Eq. (3)),
 * dependency levels, tiles and the workspace layout -- the host part of the
 * loop of Alg. 3, done once for every bucket.  The problems may be destroyed
 * afterwards.  BX_E_TOO_LARGE when a mini-bucket table exceeds the size
 * limit (the paper's out-of-memory case, Sec. 8); BX_E_INVALID when DPOP
 * finds a message whose scope differs from the sender's separator (Sec. 4). */
bx_status bx_plan_create(bx_problem *const *probs, int32_t n_probs, const bx_options *opt,
                         bx_plan **out);

/* Bytes of device workspace the plan needs: the normalised input tables, one
 * region per UTIL table (message, Sec. 6.1 bucket-tables), the descriptors,
 * results and counters -- the allocations Alg. 3 makes per bucket with
 * Gpu::Reserve, laid out once. */
bx_status bx_plan_workspace_bytes(const bx_plan *plan, size_t *bytes);

/* Copies the normalised input tables and the descriptors into the workspace
 * (host -> device on `stream`; returns once the copy has completed) -- the
 * host-to-device transfers of Alg. 3, done once for all functions instead of
 * once per function.  Must precede the first execute on a workspace.  Errors:
 * BX_E_INVALID for a NULL or unaligned workspace, BX_E_NOMEM when `bytes` is
 * below bx_plan_workspace_bytes, BX_E_DEVICE for a failed copy. */
bx_status bx_plan_upload(bx_plan *plan, void *d_workspace, size_t bytes, void *stream);

/* Runs the whole device path on `stream`: every UTIL table (aggregation of
 * Sec. 6.3 fused with the elimination of Sec. 6.4), the bounds (Sec. 2.2), the
 * value assignment (Alg. 1/2, second loop) and its cost.  Asynchronous;
 * allocates nothing; may be captured in a hipGraph.  Calls that overlap on one
 * workspace race. */
bx_status bx_plan_execute(bx_plan *plan, void *d_workspace, size_t bytes, void *stream);

/* Same with an explicit schedule (PER_BUCKET / LEVEL / DATAFLOW). */
bx_status bx_plan_execute_sched(bx_plan *plan, void *d_workspace, size_t bytes,
                                bx_schedule sched, void *stream);

/* Waits for `stream`, then copies problem `prob`'s results to the host: the
 * bound (the constant left after elimination: the optimum for BE/DPOP, a lower
 * bound for MBE/ADPOP, Sec. 2.2), the cost of the assignment (an upper bound),
 * and the assignment (n_vars int32, may be NULL).  BX_E_STATE before any
 * execute; BX_E_DEVICE if a copy fails. */
bx_status bx_plan_results(bx_plan *plan, const void *d_workspace, int32_t prob, double *bound,
                          double *ub, int32_t *assignment, void *stream);

/* ---------------------------------------------------------- plan inspection */

/* Per-plan totals: mini-buckets, UTIL rows (outputs), joint entries
 * (sum over mini-buckets of prod |D| over the mini-bucket scope), and the
 * algorithmic bytes of the UTIL phase (every input table read once, every
 * output written once). */
typedef struct {
    int64_t n_minibuckets;
    int64_t util_rows;
    int64_t joint_entries;
    int64_t algo_bytes;
    int32_t n_levels;
    int32_t n_tiles;             /* tiles of the level schedule (all levels)   */
    int32_t max_scope;           /* largest mini-bucket scope (variables)  */
    int32_t value_levels;
    int64_t tile_capacity;       /* tiles the workspace's tile region holds: the
                                    largest tile list of any tiling the planner
                                    or bx_plan_autotune may choose */
} bx_plan_stats;
bx_status bx_plan_get_stats(const bx_plan *plan, bx_plan_stats *stats);

/* Mini-buckets of problem `prob`, in creation order (positions n-1 down to 0,
 * then creation order inside a bucket).  For mini-bucket i: the eliminated
 * variable, the ids of the functions it aggregates (input functions 0..m-1 in
 * insertion order, outputs numbered m, m+1, ... in creation order), and its
 * output's id (-1 when the output is a constant) and scope (sorted by order
 * position). */
bx_status bx_plan_num_minibuckets(const bx_plan *plan, int32_t prob, int32_t *count);
bx_status bx_plan_minibucket_info(const bx_plan *plan, int32_t prob, int32_t i, int32_t *var,
                                  int32_t *n_members, int32_t *members /* cap 256 */,
                                  int32_t *out_id, int32_t *out_arity,
                                  int32_t *out_scope /* cap 64 */, int64_t *out_rows);
/* The elimination order problem `prob` was solved with. */
bx_status bx_plan_order(const bx_plan *plan, int32_t prob, int32_t *order_out);

/* Copies mini-bucket i's UTIL table (out_rows entries, int32 or float, row-major
 * over the output scope in order position, Sec. 6.1) to host memory: the
 * device-to-host copy Alg. 3 makes after every elimination, here for
 * inspection only; synchronous on `stream`.  BX_E_INVALID when n_entries is
 * not the table's size. */
bx_status bx_plan_util_table(const bx_plan *plan, const void *d_workspace, int32_t prob,
                             int32_t i, void *host_out, int64_t n_entries, void *stream);

/* One dependency level of the plan (the unit of the LEVEL schedule: all
 * instances' mini-buckets whose inputs are complete once the earlier levels
 * ran -- the independent branches of Sec. 8.1's analysis run together): its
 * mini-buckets, tiles, UTIL rows, algorithmic bytes (every input table read
 * once, every output written once) and how it runs. */
typedef struct {
    int32_t n_minibuckets;
    int32_t n_tiles;             /* tiles of the level, all paths            */
    int32_t n_row_tiles;         /* of which on the row path                 */
    int32_t n_blocked;           /* register-blocked mini-buckets            */
    int64_t util_rows;
    int64_t algo_bytes;
    int32_t staged;              /* 1: the kernel that stages lane tables    */
    int32_t nontemporal;         /* 1: blocked rows stored non-temporally    */
    int32_t tile_goal;           /* tiles per level aimed at                 */
    int32_t n_lane_tiles;        /* of which on the lane-group path          */
    int32_t n_pack_tiles;        /* of which packed (several small mini-buckets) */
    int32_t n_packed;            /* packed mini-buckets launched at this level   */
} bx_level_info;
bx_status bx_plan_level_info(const bx_plan *plan, int32_t level, bx_level_info *info);

/* Host self-check of the plan's launch schedule (no device work): every
 * mini-bucket is computed once, by one launch level, with its rows covered
 * exactly once; every producer completes in an earlier level, or earlier in
 * the same packed tile (the hand-off inside one workgroup of the fused
 * groups); packed tiles' segment headers are consistent; the per-bucket
 * schedule's tiles cover every mini-bucket.  BX_E_INVALID names the first
 * violation. */
bx_status bx_plan_validate(const bx_plan *plan);

/* Device time in ms of every level of the last timed LEVEL execute (hipEvents
 * around each level's launches; read after bx_plan_results).  ms_out holds
 * n_levels floats (the plan's level count).  BX_E_STATE when the last
 * execute was not a timed LEVEL execute. */
bx_status bx_plan_level_timing(const bx_plan *plan, float *ms_out, int32_t n_levels);

/* Device time in ms of every mini-bucket of problem `prob` (ms_out[n], n =
 * bx_plan_num_minibuckets, creation order) in the last timed PER_BUCKET
 * execute: hipEvents around each mini-bucket's own launches, i.e. one agent's
 * UTIL computation when the problem is a DCOP (Sec. 4.1-4.2).  Read after
 * bx_plan_results.  BX_E_STATE when the last execute was not a timed
 * PER_BUCKET execute. */
bx_status bx_plan_minibucket_timing(const bx_plan *plan, int32_t prob, float *ms_out, int32_t n);

/* Simulated runtime of the distributed (A)DPOP run of problem `prob`, the
 * metric by which Sec. 8 measures the DCOP algorithms: every variable is an
 * agent with its own clock, a message arrives `latency_ms` after the
 * sender's clock at sending.  UTIL: agent v starts when the messages of
 * every producer in its bucket have arrived and computes its mini-buckets
 * one after another (times mb_ms[n] in creation order, or NULL: those of the
 * last timed PER_BUCKET execute); *util_ms = the latest finish.  VALUE
 * (Sec. 4.1, third phase): agent v decides once the values of the other
 * variables of its bucket's functions have arrived, local work taken as
 * zero; *value_ms = the latest decision, *value_hops = the longest chain of
 * VALUE messages.  Outputs may be NULL.  Host only. */
bx_status bx_plan_simulated_runtime(const bx_plan *plan, int32_t prob, const float *mb_ms, double latency_ms,
                                    double *util_ms, double *value_ms, int32_t *value_hops);

/* ------------------------------------------------------------------ tuning */

/* Autotunes the level schedule of this plan: for every dependency level, the
 * tile size (from a fixed set of tiles-per-level goals), the tiled kernel
 * (with or without LDS staging of lane tables) and the kind of row stores
 * (plain or non-temporal) that ran that level fastest
 * (hipEvents on `stream` around each level's launch, minimum over `reps` + 1
 * runs of every combination); BX_SCHED_AUTO then uses the level schedule
 * with those choices.  Runs the plan's kernels on the workspace (inputs must
 * be uploaded); results of the last run are valid afterwards. */
bx_status bx_plan_autotune(bx_plan *plan, void *d_workspace, size_t bytes, int32_t reps,
                           void *stream);

/* Describes the configuration in use as a short text (for logs). */
bx_status bx_plan_describe(const bx_plan *plan, char *buf, size_t cap);

/* Timing of the last execute, in ms, from hipEvents recorded on the execute
 * stream while timing is enabled (read after bx_plan_results): util_ms spans
 * the whole UTIL phase including gaps between launches; util_kernel_ms sums
 * the intervals bracketing each UTIL launch (LEVEL schedule; equals util_ms
 * otherwise); value_ms spans the value-assignment kernel. */
bx_status bx_plan_set_timing(bx_plan *plan, int32_t enabled);
bx_status bx_plan_last_timing(const bx_plan *plan, float *util_ms, float *util_kernel_ms,
                              float *value_ms);

/* Captures one execute with schedule `sched` (the UTIL launches and the value
 * kernel) on `stream` (non-NULL) into a hipGraph bound to `d_workspace`, and
 * keeps it in the plan; bx_plan_graph_launch replays it on any stream.  The
 * graph holds kernel nodes only.  bx_plan_autotune discards it (it changes
 * the launches); bx_plan_graph_launch then returns BX_E_STATE until the
 * graph is created again. */
bx_status bx_plan_graph_create(bx_plan *plan, void *d_workspace, size_t bytes, bx_schedule sched,
                               void *stream);
bx_status bx_plan_graph_launch(bx_plan *plan, void *stream);

void bx_plan_destroy(bx_plan *plan);

/* ------------------------------------------------------ learned partitions */

/* The partition step of Alg. 2 asks only for some partition of an over-full bucket whose
 * parts hold at most `ibound` variables; any such partition keeps the MBE
 * bound valid (Sec. 2.2).  For every bucket whose scope exceeds the i-bound
 * the planner builds up to 6 distinct candidates -- candidate 0 is always
 * the greedy rule of BX_PART_GREEDY -- and describes each by
 * bx_partition_num_features() floats.  A bucket whose scope fits is never
 * split, so exact runs stay exact. */
int32_t bx_partition_num_features(void);

/* Called by the planner with every pending decision of a round (instances of
 * a batch advance together; an instance has at most one decision per round,
 * taken in elimination order): decision d belongs to problem
 * decision_problem[d] and owns candidates cand_offsets[d] ..
 * cand_offsets[d+1]-1, whose features are the rows of `features`
 * (row-major, bx_partition_num_features() floats each).  Must write
 * choices[d] in [0, count); a non-BX_OK return aborts planning with that
 * status. */
typedef bx_status (*bx_partition_chooser)(void *user, int32_t n_decisions, const int32_t *decision_problem,
                                          const int32_t *cand_offsets, const float *features,
                                          int32_t *choices);

/* bx_plan_create with partition decisions taken by `chooser` (for BX_ALGO_MBE
 * and BX_ALGO_ADPOP; `opt->partition` is ignored). */
bx_status bx_plan_create_chooser(bx_problem *const *probs, int32_t n_probs, const bx_options *opt,
                                 bx_partition_chooser chooser, void *user, bx_plan **out);

/* Decisions taken while planning, and how many differ from the greedy rule. */
bx_status bx_plan_partition_stats(const bx_plan *plan, int64_t *decisions, int64_t *non_greedy);

/* A plan made with a chooser keeps its decisions, in the order the chooser
 * saw them.  Decision d: problem, eliminated variable, the bucket's function
 * ids (fn_ids: capacity 256; ids as in bx_plan_minibucket_info), the number
 * of candidates and the one taken.  Candidate c of decision d:
 * part_of_fn[i] = index of the part that holds fn_ids[i]. */
bx_status bx_plan_num_decisions(const bx_plan *plan, int32_t *n_decisions, int64_t *n_candidates);
bx_status bx_plan_decision_info(const bx_plan *plan, int32_t d, int32_t *prob, int32_t *var, int32_t *n_fns,
                                int32_t *fn_ids, int32_t *n_cands, int32_t *choice);
bx_status bx_plan_candidate_parts(const bx_plan *plan, int32_t d, int32_t c, int32_t *part_of_fn);

/* Candidate values: after bx_plan_execute, for every recorded decision d and
 * candidate c (flat index = candidates of the earlier decisions + c),
 *     d_out[.] = (1/S) sum_{s<S} sum_k min_x sum_{f in part k} f(u = s, x)
 * over the plan's own tables, i.e. the part of the mini-bucket bound the
 * candidate keeps at that bucket (the partition step of Alg. 2; any part
 * split loses sum_k min <= min sum, Sec. 2.2).  Variables u of the bucket
 * other than x are sampled: the digit of u in sample s is
 * d_rnd[(d * S + s) * 32 + slot(u)] mod |D_u|, slot(u) = rank of u among the
 * bucket's variables in increasing id (d_rnd: n_decisions * S * 32 uint32,
 * caller-filled).  Integer sums (over the parts too) saturate at BX_INF_I32.  Buckets with more
 * than 32 such variables, more than 64 functions or |D_x| > 16 get NaN.
 * d_scratch: device memory of bx_plan_candidate_scratch_bytes() bytes,
 * 256-byte aligned.  Synchronises `stream`. */
bx_status bx_plan_candidate_scratch_bytes(const bx_plan *plan, size_t *bytes);
bx_status bx_plan_candidate_values(bx_plan *plan, const void *d_workspace, size_t bytes, int32_t samples,
                                   const uint32_t *d_rnd, double *d_out, void *d_scratch, size_t scratch_bytes,
                                   void *stream);

/* Candidate-scoring network: 2 hidden ReLU layers of `hidden` (= 128) units
 * and one linear output.  Parameters live in caller-owned device memory:
 * fp32 d_params[bx_mlp_num_params()] laid out as W1[hidden][n_in], b1[hidden],
 * W2[hidden][hidden], b2[hidden], W3[hidden], b3 (row j of W1/W2 = inputs of
 * unit j), and a bf16 copy d_params_bf16 of the same length for inference. */
typedef struct {
    int32_t n_in;            /* input features, 1..64 */
    int32_t hidden;          /* 128 */
    float *d_params;
    uint16_t *d_params_bf16;
} bx_mlp;

int64_t bx_mlp_num_params(int32_t n_in, int32_t hidden);

/* FP32 forward pass of `batch` rows of d_x (row-major [batch][n_in]); writes
 * the outputs d_y[batch] and the activations d_act[batch][2*hidden] (both
 * hidden layers after ReLU) needed by the backward pass. */
bx_status bx_mlp_forward(const bx_mlp *m, const float *d_x, float *d_act, float *d_y, int32_t batch,
                         void *stream);

/* FP32 backward pass: given dL/dy in d_dy[batch], writes dL/dparams summed over
 * the batch into d_grads (the d_params layout); d_work[batch][2*hidden] is
 * caller-provided scratch. */
bx_status bx_mlp_backward(const bx_mlp *m, const float *d_x, const float *d_act, const float *d_dy,
                          float *d_grads, float *d_work, int32_t batch, void *stream);

/* bx_mlp_backward for callers that cannot allocate device memory (code under
 * hipGraph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the per-sample scratch in a
 * static array of the library, one per GPU, instead of d_work.  At most
 * BX_MLP_NOALLOC_MAX_BATCH samples (BX_E_TOO_LARGE above, before any device
 * work).  Allocates nothing: the array's address is looked up once per
 * device (on the calling thread's current device, which must own `stream`
 * and the buffers).  Calls on one GPU share the array, so calls that overlap
 * on one GPU race; serialise them (one stream, or events). */
#define BX_MLP_NOALLOC_MAX_BATCH 4096
bx_status bx_mlp_backward_noalloc(const bx_mlp *m, const float *d_x, const float *d_act, const float *d_dy,
                                  float *d_grads, int32_t batch, void *stream);

/* One Adam step on d_params (moments d_m, d_v, zero-initialised by the
 * caller; step counts from 1). */
bx_status bx_mlp_adam_step(const bx_mlp *m, const float *d_grads, float *d_m, float *d_v, float lr,
                           float beta1, float beta2, float eps, int32_t step, void *stream);

/* d_params_bf16 <- d_params rounded to nearest-even bf16. */
bx_status bx_mlp_pack_bf16(const bx_mlp *m, void *stream);

/* Mean squared error against d_target[batch] and its gradient:
 * d_loss[0] = (1/batch) sum_b (y_b - t_b)^2, d_dy[b] = (2/batch)(y_b - t_b).
 * One workgroup; the sum is taken in a fixed order (deterministic). */
bx_status bx_mlp_mse(const float *d_y, const float *d_target, float *d_dy, float *d_loss, int32_t batch,
                     void *stream);

/* Inference with the bf16 weights: inputs and the activations of both hidden
 * layers are rounded to bf16, products accumulate in fp32; writes d_y[batch]. */
bx_status bx_mlp_infer_bf16(const bx_mlp *m, const float *d_x, float *d_y, int32_t batch, void *stream);

/* bx_plan_create with partitions chosen by the network: every candidate is
 * scored on the device (bx_mlp_infer_bf16, features staged in the caller's
 * d_buf, at least (bx_partition_num_features() + 1) * 4 bytes per candidate
 * of a round); a decision takes the best candidate whose score exceeds the
 * greedy candidate's by more than `margin`, else the greedy partition.
 * Synchronises `stream` once per round. */
bx_status bx_plan_create_learned(bx_problem *const *probs, int32_t n_probs, const bx_options *opt,
                                 const bx_mlp *model, void *d_buf, size_t buf_bytes, float margin,
                                 void *stream, bx_plan **out);

/* ------------------------------------------------------ streamed execution */

/* Tables beyond device memory (the concurrent transfer and execution of
 * Sec. 6.3, taken to the whole table set): every table -- the normalised
 * inputs and every UTIL message -- lives in a caller-provided host buffer
 * h_tables (pinned memory, hipHostMalloc or torch pin_memory, for the copies
 * to overlap) laid out like the plan's table and message regions.  The
 * mini-buckets run one after another in creation order: each one's input
 * tables are copied in, and its output is computed in chunks of chunk_rows
 * rows into two device buffers, each chunk copied out on a second stream
 * while the next is computed.  Scalar outputs stay on the device and a last
 * kernel adds them into bounds[n_probs] (the value phase needs every table on
 * the device and is not run).  The device workspace then holds the largest
 * mini-bucket's inputs plus two chunks, whatever the total size of the
 * tables.  The plan must be made with BX_FLAG_NO_BLOCKING (blocked row order
 * is not a row range; BX_E_UNSUPPORTED otherwise); chunk_rows >= 256.
 * bx_plan_stream_bytes: the device workspace and host buffer this needs.
 * bx_plan_stream_table: mini-bucket i's output from h_tables after a streamed
 * execute (non-scalar outputs).  Synchronises `stream`. */
bx_status bx_plan_stream_bytes(const bx_plan *plan, int64_t chunk_rows, size_t *device_bytes, size_t *host_bytes);
bx_status bx_plan_execute_streamed(bx_plan *plan, void *d_workspace, size_t bytes, void *h_tables,
                                   size_t host_bytes, int64_t chunk_rows, void *stream, double *bounds);
bx_status bx_plan_stream_table(const bx_plan *plan, const void *h_tables, int32_t prob, int32_t i, void *host_out,
                               int64_t n_entries);

/* ----------------------------------------------------- branch and bound */

/* Depth-first branch and bound with the mini-bucket bound as its heuristic,
 * recomputed at every node (the use Sec. 10 proposes for MBE inside a
 * search).  Variables are assigned root first along the elimination order
 * (the problem's, else `opt->order`); expanding a node conditions the problem
 * on every value of the next variable and bounds all those children in one
 * batched device pass of `opt->algo` (BX_ALGO_MBE at `opt->ibound`, or BE).
 * Each child's value phase gives a complete assignment that may improve the
 * incumbent (the root's starts it); a child whose bound reaches the
 * incumbent is pruned, one whose bound equals its own assignment's cost is
 * solved.  Integer costs (BX_COST_I32) only.
 *   d_workspace / bytes: device memory for the plans, reused pass after pass
 *     (at least bx_bnb_workspace_bytes; a batch that does not fit is split;
 *     BX_E_NOMEM if one child alone does not fit);
 *   max_nodes: expansions allowed (0: no limit); when reached, the best
 *     assignment found so far is returned with stats[3] = 0;
 *   *value, assignment[n_vars] (caller-allocated): the optimum (or best found)
 *     and an assignment reaching it;
 *   stats[4]: nodes expanded, device passes, nodes pruned, 1 if optimal.
 * Synchronises `stream` after every pass. */
bx_status bx_bnb_workspace_bytes(const bx_problem *p, const bx_options *opt, size_t *bytes);
bx_status bx_bnb_solve(const bx_problem *p, const bx_options *opt, void *d_workspace, size_t bytes,
                       void *stream, int64_t max_nodes, double *value, int32_t *assignment, int64_t *stats);

/* ------------------------------------------------------------ measurement */

/* Bandwidth reference for the roofline of the UTIL kernels (the paper
 * reports run times only, Sec. 8; this states what the device's memory
 * delivers to a plain streaming kernel): kind 0 copies `bytes` from d_src to
 * d_dst, kind 1 writes `bytes` to d_dst, kind 2 reads `bytes` of d_src and
 * writes one int32 per workgroup to d_dst (at least `grid` * 4 bytes).  16-byte
 * vector accesses, `grid` workgroups of 256 threads (0: 8 per compute unit),
 * grid-stride.  bytes must be a multiple of 16 and the pointers 16-byte
 * aligned (BX_E_INVALID otherwise).  Asynchronous on `stream`. */
bx_status bx_stream_probe(int32_t kind, void *d_dst, const void *d_src, size_t bytes, int32_t grid,
                          void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *bx_last_error(void);
/* Version string. */
const char *bx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BX_H */
