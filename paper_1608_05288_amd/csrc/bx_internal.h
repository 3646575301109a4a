// Internal structures of the UTIL-table engine: the host plan and the
// descriptors the device kernels read.  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bx.h"

namespace bx {

// Largest number of variables in a mini-bucket output scope.  A table over
// more variables would exceed 2^31 entries for every domain size >= 2.
constexpr int kMaxVars = 31;
// Table starts are aligned to this many 4-byte elements (256 bytes), so no
// two tables share a cache line.
constexpr int64_t kAlignElems = 64;
constexpr int32_t kInfI32 = 2147483647;
// Largest domain size accepted, and the number of candidate values the value
// phase examines per step (its LDS buffer); a step never splits a variable.
constexpr int32_t kMaxDomain = 1024;
constexpr int32_t kValuePairCap = 2048;

// ------------------------------------------------------------------ device
// Everything the kernels read lives in one caller-provided workspace.  Table
// positions are element offsets (4-byte elements) from the workspace base.

// One mini-bucket: output g[s] = min_{x in D} sum_f f[base_f(s) + x], s over
// the output scope (Sec. 6.3-6.4, fused).
// Threads per workgroup of the UTIL kernels, lane functions and eliminated
// domain the tiled path handles, and outer indices per tile at most.
constexpr int kUtilThreads = 256;
constexpr int kTileLaneFns = 8;
constexpr int kTileMaxD = 8;
constexpr int kTileMaxOuter = 256;
constexpr int kTileOuterFns = 8;         // outer-only functions the tiled path pre-sums
constexpr int kTileConstFns = 8;         // functions of the eliminated variable alone
constexpr int kTileMaxRun = 32;          // lane functions * D entries read per row
constexpr int kStageMaxD = 4;            // staging of lane tables in LDS: D <= 4,
constexpr int kStageMaxFns = 4;          //   lane functions <= 4,
constexpr int kStageEntries = 4096;      //   entries staged per tile,
constexpr int kStageReuse = 4;           //   each staged entry read at least this often
constexpr int64_t kTileMaxTable = int64_t(1) << 30;   // tables addressed with 32-bit byte offsets
constexpr int32_t kRowTileRows = 256;      // rows per tile on the row path (one per thread)
constexpr int32_t kMinTileRows = 1024;     // finest tiling the tuner may pick
constexpr int32_t kMaxTileRows = 65536;      // coarsest tile
constexpr int32_t kDefaultTilesGoal = 2048;   // tiles per level aimed at
constexpr int32_t kTuneGoals[] = {512, 768, 1024, 1536, 2048, 3072, 4096, 6144};   // tiles per level the tuner tries
// Register blocking of the tiled path: each thread computes a box of
// da x db rows (all values of two outer variables) and loads a lane function
// once per value combination of the box variables it depends on.
constexpr int kBlockMaxD = 5;            // eliminated domain handled
constexpr int kBlockMaxD2 = 4;           //   ... with two box variables (D = 5: b alone)
constexpr int kBlockMaxDb = 4;           // domain of box variable b, visited fastest (2..4),
constexpr int kBlockMaxDb1 = 5;          //   or 2..5 when b is the only box variable
constexpr int kBlockMaxDa = 4;           // domain of box variable a (absent, or 2..4)
constexpr int kBlockRowCol = kTileLaneFns - 1;   // LDS column holding the output outer index
constexpr int kBlockMaxInner = 8;        // inner variables (p_in <= 256 with domains >= 2)
// Lane-group path (eliminated domain above kTileMaxD): G lanes share a row.
constexpr int kLaneMaxFns = 8;           // functions per mini-bucket it handles
constexpr int kLanePasses = 8;           // passes of 256 / G rows per tile
// Packed path: small mini-buckets, one output row per thread, rows of several
// mini-buckets in one workgroup.  A group of packed mini-buckets forming a
// connected part of the bucket tree (a root and some of its descendants) is
// computed by one workgroup in stages, children before parents, with a
// workgroup barrier between stages (no device-wide wait): the group runs in
// the launch after its last outside producer.
// Defaults of the bx_options packing fields:
constexpr int kPackMaxRows = 256;        // output rows of a packable mini-bucket
constexpr int kPackRowLimit = 1 << 16;   //   and its cap whatever the option (the packed
                                         //   row decode divides in single precision)
constexpr int kFuseMaxRows = 1024;       // rows of one group (all its stages)
constexpr int kFuseMaxStages = 4;        // stages of one group
constexpr int kFuseMaxStageRows = 256;   // rows of one group's stage
constexpr int kPackStageRows = 256;      // rows per stage a packed tile aims at
// Fixed limits (a packed tile's descriptors are copied to LDS whole):
constexpr int kPackMaxFns = 6;           // functions of a packable mini-bucket
constexpr int kPackMaxVars = 12;         // output variables of a packable mini-bucket
constexpr int kPackMaxD = 64;            // eliminated domain of a packable mini-bucket
constexpr int kPackMaxStride = 65535;    // strides and domains stored in 16 bits
constexpr int kPackMaxSegs = 32;         // mini-buckets per packed tile

// Tiled path: output rows are split as row = o * p_in + r, r over the n_inner
// fastest output variables (p_in <= kUtilThreads), o over the others.  Thread
// t owns r = t % p_in and outer slot t / p_in (q slots per pass); the outer
// part of every table offset is computed once per outer index.  Row path: a
// full decode per row (any D, any number of functions).
struct alignas(16) DevMb {
    int64_t out_off;     // element offset of the output table
    int64_t out_rows;    // rows of the output table (prod of dims)
    int64_t n_outer;     // out_rows / p_in
    int32_t nv;          // output variables
    int32_t D;           // domain of the eliminated variable (stride 1 everywhere)
    int32_t f_begin;     // first DevFn of this mini-bucket
    int32_t nf;          // functions aggregated
    int32_t nfl;         // the first nfl functions depend on inner and outer
                         //   variables, the next nf - nfl - nfi - nfc on outer
                         //   ones only
    int32_t n_inner;     // inner (fastest) output variables
    int32_t p_in;        // rows per outer index = prod of the inner dims
    int32_t q;           // outer indices per pass = kUtilThreads / p_in
    int32_t path;        // 0: tiled, 1: row, 2: lane groups, 3: packed
    int32_t inst;        // problem index in the batch
    int32_t level;       // dependency level
    int32_t n_tiles;     // tiles of this mini-bucket
    int32_t blk;         // tiled path: 1 = register-blocked row loop
    int32_t da, db;      // blocked: box = da x db outer indices (db: 1 when unused)
    int32_t g0, ga, gb;  // blocked: lane functions [0,g0) depend on neither box
                         //   variable, [g0,ga) on the second only, [ga,gb) on
                         //   the first only, [gb,nfl) on both
    int32_t nfc;         // tiled path: the last nfc functions depend on x alone,
    int32_t nfi;         //   the nfi before them on inner variables (and x) only
    int32_t lanes;       // lane-group path: lanes per row (8, 16, 32 or 64)
    int32_t red;         // elimination: 0 minimum over x, 1 -ln sum_x exp(-.) (sum-product)
    int32_t pad3[3];
    int32_t dims[kMaxVars + 1];   // output dims, most significant first; for a
                                  // blocked mini-bucket the outer variables are
                                  // in visiting order (box variables last)
    int32_t ostr[kMaxVars + 1];   // blocked: outer-index stride of each outer
                                  // variable in the output table (visiting order)
};

struct alignas(16) DevFn {
    int64_t tab_off;     // element offset of the table
    int32_t src_mb;      // mini-bucket producing it (-1: an input table)
    int32_t io_max;      // tiled path: inner part of the offset at the last inner position
    int32_t stride[kMaxVars + 1]; // stride of output variable j in this table (0: absent)
};

// A unit of device work: rows [begin, end) of mini-bucket mb (row tiles), or
// outer indices [begin, end) (tiled kernel).
struct alignas(16) DevTile {
    int32_t mb;
    int32_t pad;
    int64_t begin;
    int64_t end;
};

// Packed path: one packed tile = DevTile{begin, end} over DevSeg entries,
// stage by stage; a stage is a run of segments whose `first` starts at 0.
// Everything a row of a packed mini-bucket needs, in one 256-byte record.
struct alignas(16) DevSeg {
    int64_t out_off;                  // output table
    int64_t tab_off[kPackMaxFns];     // input tables
    int32_t mb;          // packed mini-bucket (all its rows)
    int32_t first;       // position of its first row among the stage's rows
    int32_t stage_segs;  // segments of the stage, and rows of the stage (the
    int32_t stage_rows;  //   same on every segment of one stage)
    int32_t nv, nf, D, red;   // red: as in DevMb
    // output dims, most significant first, right-aligned (the fastest output
    // variable at kPackMaxVars - 1; unused leading slots: dim 1, stride 0)
    uint16_t dims[kPackMaxVars];
    uint16_t stride[kPackMaxFns][kPackMaxVars];   // stride of output variable slot j in table f (0: absent)
};
static_assert(sizeof(DevSeg) == 256, "DevSeg layout");

// Value assignment: one entry per (problem, variable), grouped by value level.
struct alignas(16) DevVar {
    int32_t var;         // variable id within its problem
    int32_t D;
    int32_t f_begin;     // first DevVFn (functions of the full bucket)
    int32_t nf;
    int32_t pair_begin;  // first DevPair of this variable
    int32_t occ_begin;   // first (function, stride) occurrence of this variable
    int32_t occ_n;       //   in the problem's functions (value and UB lists)
    int32_t pad;
};

// A function looked up by the value phase: entry = tab_off + sum sigma[var]*stride + x.
struct alignas(16) DevVFn {
    int64_t tab_off;
    int32_t t_begin;     // first (var, stride) term
    int32_t nt;          // terms (the bucket variable itself excluded for VALUE;
                         //        every scope variable included for the UB list)
};

struct alignas(16) DevPair {  // one candidate value of one variable
    int32_t var_entry;   // index into DevVar
    int32_t x;
    int32_t f_begin;     // the variable's functions (copied from DevVar: one
    int32_t nf;          //   dependent load less per value step)
};

struct alignas(16) DevInst {  // per problem
    int32_t n;           // variables
    int32_t is_f32;
    int32_t lvl_begin;   // first value level (index into level offsets)
    int32_t n_lvl;
    int32_t ub_begin;    // first DevVFn of the input-function list (UB)
    int32_t ub_n;
    int32_t const_begin; // first scalar message offset
    int32_t const_n;
    int64_t sigma_off;   // byte offset of the assignment (int32[n]) in the results area
    double host_const;   // sum of the constant input functions
    double bound_const;  // added to the bound only (sum-product: -ln |D_v| of unconstrained variables)
    int32_t vfn_begin;   // this problem's DevVFn range (value and UB lists),
    int32_t vfn_n;       //   (var, stride) term range, DevVar range, DevPair
    int32_t term_begin;  //   range and (function, stride) occurrence range
    int32_t term_n;      //   (the terms grouped by variable): the value
    int32_t var_begin;   //   kernel copies all but the terms to LDS when
    int32_t var_n;       //   they fit its arena
    int32_t pair_begin;
    int32_t pair_n;
    int32_t occ_begin;
    int32_t occ_n;
};

struct alignas(16) DevResult {  // per problem, written by the device
    double bound;
    double ub;
    int32_t status;      // 0 ok, nonzero: a dependency wait gave up
    int32_t pad[3];
};

// --------------------------------------------------------------------- host

struct Function {
    std::vector<int32_t> scope;     // as given by the caller
    std::vector<int32_t> ti;
    std::vector<float> tf;
};

struct Problem {
    int32_t n = 0;
    std::vector<int32_t> dom;
    bx_cost_type ct = BX_COST_I32;
    std::vector<Function> fns;
    std::vector<int32_t> order;     // empty: not set
    std::vector<int32_t> parent;    // empty: not set
};

// A function of the elimination (input after normalisation, or a message).
struct PFn {
    int32_t id = 0;
    std::vector<int32_t> scope;     // sorted by increasing order position
    int64_t size = 1;
    int64_t off = -1;               // element offset in the workspace
    int32_t src_mb = -1;            // producing mini-bucket (global index), -1: input
    int32_t input_index = -1;       // caller's function index for inputs
};

struct PMb {                        // a planned mini-bucket
    int32_t inst = 0;
    int32_t var = 0;                // eliminated variable
    int32_t k = 0;                  // index inside its bucket
    std::vector<int32_t> members;   // function ids (instance-local)
    std::vector<int32_t> U;         // joint scope sorted by position, var last
    int64_t out_rows = 1;
    int32_t out_id = -1;            // function id of the output, -1: constant
    int64_t out_off = 0;
    int32_t level = 0;              // launch level (dependency level after packing)
    int32_t dep_level = 0;          // dependency level (1 + the latest producer's)
    int32_t group = -1;             // packed: its group (root mini-bucket index), else -1
    int32_t stage = 0;              // packed: stage inside its group (children first)
    int32_t red = 0;                // 1: eliminated by summation (sum-product), else minimum
    int32_t first_tile = 0;         // its own tiles (packed: row tiles of the per-bucket schedule)
    int32_t n_tiles = 0;
    int32_t done_tile = 0;          // one past the level-schedule tile that completes it
    int64_t algo_bytes = 0;         // every input table read once + the output written once
};

struct PInst {
    int32_t n = 0;
    std::vector<double> fn_range;               // input cost range per function id (0 for outputs)
    std::vector<int32_t> dom;
    std::vector<int32_t> order, pos, parent;
    std::vector<PFn> fns;                       // index == id
    std::vector<std::vector<int32_t>> bucket;   // function ids per variable (full bucket)
    std::vector<int32_t> mbs;                   // global mini-bucket indices, creation order
    double host_const = 0.0;                    // constant inputs (saturating for int)
    double bound_const = 0.0;                   // sum-product: -ln |D_v| of unconstrained variables
    int32_t m_inputs = 0;
};

struct Candidate {
    std::vector<std::vector<int32_t>> parts;
    int32_t generator = 0;
};

// A partition decision taken while planning with a chooser, kept for the
// candidate-value pass (the order is the one the chooser saw).
struct Decision {
    int32_t inst = 0, var = 0;
    std::vector<int32_t> B;            // bucket function ids
    std::vector<Candidate> cands;      // candidate 0: the greedy partition
    int32_t choice = 0;
};

// candidate-value pass (bx_cand.hip): per decision, per function
constexpr int kCandSlots = 32;         // bucket variables (other than the eliminated one) sampled
constexpr int kCandMaxD = 16;          // eliminated domain handled
constexpr int kCandMaxFns = 64;        // functions per bucket handled
struct alignas(16) DevCDec {
    int32_t D, nfn, fn_begin, nslot, slot_begin, ncand, part_begin, out_begin;
    int32_t valid, pad[3];
};
struct alignas(16) DevCFn {
    int64_t tab_off;
    int32_t nterm, term_begin;
};

struct Plan {
    bx_options opt{};               // opt.tune_cache is not kept (see tune_cache)
    std::string tune_cache;         // tuning-cache file ("" = none)
    bx_cost_type ct = BX_COST_I32;
    std::vector<PInst> inst;
    std::vector<PMb> mbs;

    // device images (uploaded)
    std::vector<DevMb> dmb;
    std::vector<DevFn> dfn;
    std::vector<DevTile> dtile;              // row tiles
    std::vector<int32_t> level_tile_begin;   // tiles grouped by level, size n_levels+1
    std::vector<int32_t> level_row_begin;    // first row-path tile of each level
    std::vector<int32_t> level_lane_begin;   // first lane-group tile of each level
    std::vector<int32_t> level_pack_begin;   // first packed tile of each level (= its first tile)
    std::vector<int32_t> level_tiled_begin;  // first tiled-path tile of each level (after the packed ones)
    std::vector<DevSeg> dseg;                // segments of the packed tiles
    size_t seg_cap = 0, off_seg = 0;         // segment region (entries, byte offset)
    int32_t n_groups = 0, n_packed = 0;      // packed groups and mini-buckets
    bool sum_mode = false;                   // sum-product plan (BE_SUM / MBE_SUM)
    bool pack_allowed = true;                // BX_FLAG_NO_PACKING not set
    bool pack_on = true;                     // packing in use (the autotuner may turn it off)
    int32_t pack_max_rows = kPackMaxRows, fuse_max_rows = kFuseMaxRows, fuse_max_stages = kFuseMaxStages,
            fuse_max_stage_rows = kFuseMaxStageRows, pack_stage_rows = kPackStageRows;
    std::vector<uint8_t> level_stage;        // per level: the tiled kernel that stages lane tables
    std::vector<int32_t> level_goal;         // per level: tiles aimed at (autotuned)
    std::vector<uint8_t> level_nt;           // per level: tiled-path rows stored non-temporally
    std::vector<uint8_t> level_xcd;          // per level: tiles taken XCD by XCD (autotuned)
    std::vector<DevVar> dvar;
    std::vector<DevVFn> dvfn;
    std::vector<int32_t> dterm;              // (var, stride) pairs
    std::vector<int32_t> docc;               // (function, stride) pairs grouped by variable
    std::vector<DevPair> dpair;
    std::vector<int32_t> vlevel_var_begin;   // DevVar offsets of value levels (all insts)
    std::vector<int32_t> vlevel_pair_begin;  // DevPair offsets of value levels
    std::vector<DevInst> dinst;
    std::vector<int64_t> dconst;             // element offsets of scalar messages
    std::vector<uint8_t> tables;             // normalised input tables (host image)

    // workspace layout (bytes)
    size_t off_counters = 0, n_counters = 0;
    size_t tile_cap = 0;                     // tiles the tile region holds
    size_t off_mb = 0, off_fn = 0, off_tile = 0, off_var = 0, off_vfn = 0, off_term = 0, off_occ = 0,
           off_pair = 0, off_vlv = 0, off_vlp = 0, off_inst = 0, off_const = 0;
    size_t off_zeros = 0;                    // 256 zero bytes (never written)
    size_t off_tables = 0, tables_bytes = 0;
    size_t off_msgs = 0, msgs_bytes = 0;
    size_t off_results = 0, results_bytes = 0;
    size_t off_sigma = 0;
    size_t total_bytes = 0;
    size_t static_bytes = 0;                 // [0, static_bytes) is uploaded

    int32_t n_levels = 0;
    int64_t n_decisions = 0, n_nongreedy = 0;   // learned-partition decisions taken
    std::vector<Decision> decisions;         // recorded when planned with a chooser
    int64_t n_candidates = 0;
    std::vector<uint8_t> cand_image;         // host image of the candidate-value descriptors
    int32_t max_value_levels = 0;
    int32_t max_scope = 0;
    int64_t util_rows = 0, joint_entries = 0, algo_bytes = 0;
    int64_t total_vars = 0;

    // tuning / execution state
    int32_t rows_per_tile = 0;
    int32_t block = 256;
    bx_schedule tuned = BX_SCHED_LEVEL;
    bool tuned_valid = false;
    bool timing = false;
    bool capturing = false;
    bx_schedule timed_sched = BX_SCHED_AUTO;   // schedule of the last timed execute
    float last_util_ms = 0.f, last_value_ms = 0.f, last_util_kernel_ms = 0.f;
    std::vector<float> last_level_ms;        // per level, last timed LEVEL execute
    bool tune_cached = false;                // the last autotune reused a stored choice
    float tune_pass_ms[2] = {0.f, 0.f};      // last autotune: LEVEL and PER_BUCKET pass times
    float tune_pack_ms[2] = {0.f, 0.f};      // last autotune: tuned LEVEL pass, packing off / on (0: not tried)
    void *ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<void *> lev_ev;              // per-level (start, end) events when timing
    std::vector<void *> mb_ev;               // per-mini-bucket (start, end) events (timed PER_BUCKET)
    std::vector<float> last_mb_ms;           // per mini-bucket, last timed PER_BUCKET execute
    void *graph = nullptr, *graph_exec = nullptr;
    void *graph_ws = nullptr;
    bool executed = false;
};

// A candidate partition of an over-full bucket (function ids per part) and
// the rule that produced it.
constexpr int32_t kPartBaseFeatures = 16;               // per candidate
constexpr int32_t kPartFeatures = 2 * kPartBaseFeatures;  // + difference to the greedy candidate

// Chooses one candidate per pending decision.  cand_offsets has n_dec + 1
// entries into the rows of `features` (kPartFeatures floats per candidate);
// candidate 0 of every decision is the greedy partition.
using Chooser = bx_status (*)(void *ctx, int32_t n_dec, const int32_t *dec_inst,
                              const int32_t *cand_offsets, const float *features, int32_t *choices);

// partition candidates and features (bx_partition.cpp)
std::vector<Candidate> candidate_partitions(const PInst &I, const std::vector<int32_t> &B, int ibound,
                                            uint64_t seed);
void partition_features(const PInst &I, const std::vector<int32_t> &B, int32_t v, int ibound,
                        const Candidate &c, const std::vector<double> &fn_range, float *f);

// planner (bx_plan.cpp)
bx_status validate_problem(const Problem &p);
bx_status compute_order(const Problem &p, bx_order_heuristic h, std::vector<int32_t> &order,
                        std::vector<int32_t> &parent);
int32_t induced_width(const Problem &p, const std::vector<int32_t> &order);
bx_status build_plan(const std::vector<const Problem *> &probs, const bx_options &opt, Plan &plan,
                     Chooser chooser = nullptr, void *chooser_ctx = nullptr);
bx_status fill_descriptors(Plan &plan);
void schedule_levels(Plan &plan);              // launch levels and packed groups
bx_status set_packing(Plan &plan, bool on);     // re-plan paths, levels and tiles with packing on / off
bx_status validate_schedule(const Plan &plan); // host self-check of tiles, segments and levels
void retile(Plan &plan, int32_t tiles_goal);   // the same goal on every level
void retile_levels(Plan &plan);                // the goals in plan.level_goal
int64_t outer_per_tile(const DevMb &d, int32_t target_rows);

// device side (bx_exec.hip)
bx_status dev_upload(Plan &plan, void *ws, size_t bytes, void *stream);
bx_status dev_execute(Plan &plan, void *ws, size_t bytes, bx_schedule sched, void *stream);
bx_status dev_results(Plan &plan, const void *ws, int32_t prob, double *bound, double *ub,
                      int32_t *assignment, void *stream);
bx_status dev_copy_table(const Plan &plan, const void *ws, int64_t off, int64_t n, void *host,
                         void *stream);
bx_status dev_autotune(Plan &plan, void *ws, size_t bytes, int32_t reps, void *stream);
void dev_release(Plan &plan);
bx_status dev_graph_create(Plan &plan, void *ws, size_t bytes, bx_schedule sched, void *stream);
bx_status dev_graph_launch(Plan &plan, void *stream);
bx_status dev_stream_probe(int32_t kind, void *dst, const void *src, size_t bytes, int32_t grid,
                           void *stream);
bool level_stage_on(const Plan &P, int level);   // staging kernel on this level (flags or tuner)
bool level_nt_on(const Plan &P, int level);      // blocked rows stored non-temporally
bool level_xcd_on(const Plan &P, int level);     // tiles taken XCD by XCD
bx_status simulated_runtime(const Plan &P, int32_t prob, const float *mb_ms, double latency_ms,
                            double *util_ms, double *value_ms, int32_t *value_hops);

// network scoring of partition candidates (bx_mlp.hip)
struct LearnedCtx {
    const bx_mlp *model;
    void *d_buf;
    size_t buf_bytes;
    float margin;
    void *stream;
};
int64_t mlp_num_params(int32_t n_in, int32_t hidden);
bx_status mlp_forward(const bx_mlp *m, const float *x, float *act, float *y, int32_t batch, void *stream);
bx_status mlp_backward(const bx_mlp *m, const float *x, const float *act, const float *dy, float *grads,
                       float *work, int32_t batch, void *stream);
bx_status mlp_backward_noalloc(const bx_mlp *m, const float *x, const float *act, const float *dy, float *grads,
                               int32_t batch, void *stream);
bx_status mlp_adam(const bx_mlp *m, const float *grads, float *mom, float *vel, float lr, float beta1,
                   float beta2, float eps, int32_t step, void *stream);
bx_status mlp_pack_bf16(const bx_mlp *m, void *stream);
bx_status mlp_mse(const float *y, const float *t, float *dy, float *loss, int32_t batch, void *stream);
bx_status mlp_infer_bf16(const bx_mlp *m, const float *x, float *y, int32_t batch, void *stream);
size_t cand_scratch_bytes(const Plan &P);
bx_status dev_candidate_values(Plan &P, const void *ws, size_t ws_bytes, int32_t samples, const uint32_t *rnd,
                               double *out, void *scratch, size_t scratch_bytes, void *stream);
bx_status mlp_choose(void *ctx, int32_t n_dec, const int32_t *dec_inst, const int32_t *off, const float *feats,
                     int32_t *choices);

// branch and bound with the mini-bucket bound (bx_bnb.cpp); stats[4]: nodes
// expanded, device passes, nodes pruned, 1 if the optimum is proved
bx_status bnb_solve(const Problem &p, const bx_options &opt, void *ws, size_t bytes, void *stream,
                    int64_t max_nodes, double *value, int32_t *assignment, int64_t *stats);

// streamed execution (bx_stream.hip): tables in pinned host memory, each
// mini-bucket's inputs copied in and its output copied out in chunks
bx_status stream_bytes(const Plan &plan, int64_t chunk_rows, size_t *dev_bytes, size_t *host_bytes);
bx_status dev_execute_streamed(Plan &plan, void *ws, size_t bytes, void *host, size_t host_bytes,
                               int64_t chunk_rows, void *stream, double *bounds);

// errors (bx_capi.cpp)
bx_status set_error(bx_status s, const std::string &msg);

}  // namespace bx
