// Host side of the device path: upload, the UTIL launch schedules
// (one launch per mini-bucket, or one per dependency level: all instances
// and all independent mini-buckets of the level together), hipGraph capture
// and replay, per-level timing, the autotuner, and result copies.  The
// kernels live in bx_k_*.hip (see bx_util_kernels.h and bx_k_misc.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "bx_device.h"

namespace bx {

bx_status dev_upload_tiles(Plan &P, void *ws, hipStream_t st);

namespace {

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return set_error(BX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)


Descs make_descs(const Plan &P, void *ws) {
    char *w = static_cast<char *>(ws);
    Descs d;
    d.mb = reinterpret_cast<const DevMb *>(w + P.off_mb);
    d.fn = reinterpret_cast<const DevFn *>(w + P.off_fn);
    d.tile = reinterpret_cast<const DevTile *>(w + P.off_tile);
    d.seg = reinterpret_cast<const DevSeg *>(w + P.off_seg);
    d.ws = w;
    d.zeros = w + P.off_zeros;
    d.n_tiles = (int32_t)P.dtile.size();
    d.nt = 0;
    d.xcd = 0;
    d.pf_t0 = d.pf_n = d.pf_extra = d.pf_xcd = 0;
    d.sink = reinterpret_cast<int32_t *>(w + P.off_counters) + 2;
    return d;
}

VDescs make_vdescs(const Plan &P, void *ws) {
    char *w = static_cast<char *>(ws);
    VDescs d;
    d.inst = reinterpret_cast<const DevInst *>(w + P.off_inst);
    d.var = reinterpret_cast<const DevVar *>(w + P.off_var);
    d.vfn = reinterpret_cast<const DevVFn *>(w + P.off_vfn);
    d.term = reinterpret_cast<const int32_t *>(w + P.off_term);
    d.occ = reinterpret_cast<const int32_t *>(w + P.off_occ);
    d.pair = reinterpret_cast<const DevPair *>(w + P.off_pair);
    d.vlv = reinterpret_cast<const int32_t *>(w + P.off_vlv);
    d.vlp = reinterpret_cast<const int32_t *>(w + P.off_vlp);
    d.cst = reinterpret_cast<const int64_t *>(w + P.off_const);
    d.res = reinterpret_cast<DevResult *>(w + P.off_results);
    d.ws = w;
    d.sigma_base = w + P.off_sigma;
    return d;
}

// Tiles [t0, t_lane) in one launch whatever paths they take (packed, tiled,
// row); lane-group tiles [t_lane, t1) in a second one.
void launch_range(const Plan &P, Descs d, int32_t t0, int32_t t_lane, int32_t t1, bool stage, bool nt,
                  bool xcd, hipStream_t st) {
    d.nt = nt ? 1 : 0;
    d.xcd = xcd ? 1 : 0;
    if (P.ct == BX_COST_I32) {
        launch_tiles_i32(d, t0, t_lane - t0, stage, nt, st);
        launch_lanes_i32(d, t_lane, t1 - t_lane, st);
    } else if (P.sum_mode) {
        launch_tiles_fs(d, t0, t_lane - t0, stage, nt, st);
        launch_lanes_fs(d, t_lane, t1 - t_lane, st);
    } else {
        launch_tiles_f32(d, t0, t_lane - t0, stage, nt, st);
        launch_lanes_f32(d, t_lane, t1 - t_lane, st);
    }
}

}  // namespace

// Staging, store kind and tile order of level l: the autotuner's choice
// unless a flag forces one.
bool level_stage_on(const Plan &P, int l) {
    if (P.opt.flags & BX_FLAG_STAGE_ALWAYS) return true;
    if (P.opt.flags & BX_FLAG_STAGE_NEVER) return false;
    return P.level_stage[l] != 0;
}

bool level_nt_on(const Plan &P, int l) {
    return (P.opt.flags & BX_FLAG_FORCE_NT) || P.level_nt[l] != 0;
}

bool level_xcd_on(const Plan &P, int l) { return (P.opt.flags & BX_FLAG_XCD_ORDER) || P.level_xcd[l] != 0; }

namespace {

bx_status launch_util(Plan &P, void *ws, bx_schedule sched, hipStream_t st) {
    Descs d = make_descs(P, ws);
    if (P.dtile.empty()) return BX_OK;
    if (sched == BX_SCHED_PER_BUCKET) {
        // timed: an event pair around every mini-bucket's launches
        const bool ev = P.timing && !P.capturing && P.mb_ev.size() == 2 * P.mbs.size();
        for (const PInst &I : P.inst)
            for (int32_t g : I.mbs) {
                const PMb &mb = P.mbs[g];
                if (mb.n_tiles == 0) continue;
                const int32_t t0 = mb.first_tile, t1 = mb.first_tile + mb.n_tiles;
                if (ev) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.mb_ev[2 * g]), st));
                // (a packed mini-bucket runs alone on row tiles of its own)
                launch_range(P, d, t0, P.dmb[g].path == 2 ? t0 : t1, t1, level_stage_on(P, mb.level),
                             level_nt_on(P, mb.level), level_xcd_on(P, mb.level), st);
                if (ev) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.mb_ev[2 * g + 1]), st));
            }
    } else if (sched == BX_SCHED_LEVEL) {
        const bool ev = P.timing && !P.capturing;
        for (int l = 0; l < P.n_levels; ++l) {
            const int32_t t0 = P.level_tile_begin[l], t1 = P.level_tile_begin[l + 1];
            if (t1 <= t0) continue;
            if (ev) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.lev_ev[2 * l]), st));
            // the launch also warms the next level's descriptors (its tiled-
            // kernel tiles, when not too many)
            Descs dl = d;
            for (int l2 = l + 1; l2 < P.n_levels; ++l2) {
                if (P.level_tile_begin[l2 + 1] <= P.level_tile_begin[l2]) continue;
                const int32_t n2 = P.level_lane_begin[l2] - P.level_tile_begin[l2];
                if (n2 > 0 && n2 <= kWarmMaxTiles) {
                    dl.pf_t0 = P.level_tile_begin[l2];
                    dl.pf_n = n2;
                    dl.pf_extra = kWarmBlocks;
                    dl.pf_xcd = level_xcd_on(P, l2) ? 1 : 0;
                }
                break;
            }
            launch_range(P, dl, t0, P.level_lane_begin[l], t1, level_stage_on(P, l), level_nt_on(P, l),
                         level_xcd_on(P, l), st);
            if (ev) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.lev_ev[2 * l + 1]), st));
        }
    } else {
        return set_error(BX_E_UNSUPPORTED, "the dataflow schedule is disabled");
    }
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

bx_status launch_value(Plan &P, void *ws, hipStream_t st) {
    VDescs d = make_vdescs(P, ws);
    if (P.ct == BX_COST_I32) launch_value_i32(d, (int32_t)P.inst.size(), st);
    else launch_value_f32(d, (int32_t)P.inst.size(), st);
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

template <class V>
void put(std::vector<uint8_t> &img, size_t off, const std::vector<V> &v) {
    if (!v.empty()) std::memcpy(img.data() + off, v.data(), v.size() * sizeof(V));
}

bx_status run(Plan &P, void *ws, bx_schedule sched, hipStream_t st) {
    bx_status s = launch_util(P, ws, sched, st);
    if (s != BX_OK) return s;
    if (P.timing && !P.capturing) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[1]), st));
    return launch_value(P, ws, st);
}

bx_status ensure_events(Plan &P) {
    for (int i = 0; i < 3; ++i)
        if (!P.ev[i]) HIP_TRY(hipEventCreate(reinterpret_cast<hipEvent_t *>(&P.ev[i])));
    if (P.lev_ev.size() != 2 * (size_t)P.n_levels) {
        for (void *e : P.lev_ev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
        P.lev_ev.assign(2 * (size_t)P.n_levels, nullptr);
        for (void *&e : P.lev_ev) HIP_TRY(hipEventCreate(reinterpret_cast<hipEvent_t *>(&e)));
    }
    return BX_OK;
}

// Event pairs around every mini-bucket's launches (timed PER_BUCKET runs).
bx_status ensure_mb_events(Plan &P) {
    if (P.mb_ev.size() == 2 * P.mbs.size()) return BX_OK;
    for (void *e : P.mb_ev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    P.mb_ev.assign(2 * P.mbs.size(), nullptr);
    for (void *&e : P.mb_ev) HIP_TRY(hipEventCreate(reinterpret_cast<hipEvent_t *>(&e)));
    return BX_OK;
}

// A captured graph bakes in the launches (grid sizes, tile ranges, kernel
// variants); anything that changes them discards it.
void drop_graph(Plan &P) {
    if (P.graph_exec) { (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(P.graph_exec)); P.graph_exec = nullptr; }
    if (P.graph) { (void)hipGraphDestroy(static_cast<hipGraph_t>(P.graph)); P.graph = nullptr; }
    P.graph_ws = nullptr;
}

// Whole UTIL pass with `sched`, timed by events on `st` (ms).
bx_status time_pass(Plan &P, void *ws, bx_schedule sched, hipStream_t st, float *ms) {
    hipEvent_t e0 = static_cast<hipEvent_t>(P.ev[0]), e1 = static_cast<hipEvent_t>(P.ev[2]);
    const bool was_timing = P.timing;
    P.timing = false;
    HIP_TRY(hipEventRecord(e0, st));
    bx_status s = launch_util(P, ws, sched, st);
    P.timing = was_timing;
    if (s != BX_OK) return s;
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    return BX_OK;
}

// Per level, the tile goal (one of kTuneGoals), the tiled kernel (with or
// without LDS staging) and the tile order (in list order or XCD by XCD) that
// ran the level fastest: minimum over reps of the level's own events, every
// combination timed on the whole level pass.  Then, on whole passes, plain
// or non-temporal stores of the blocked rows and the chosen tile orders or
// list order everywhere, whichever ran fastest (these choices change what
// the next level finds in the caches, so they are timed on whole passes).
bx_status tune_levels(Plan &P, void *ws, int32_t reps, hipStream_t st) {
    bx_status s = ensure_events(P);
    if (s != BX_OK) return s;
    std::vector<float> best(P.n_levels, 1e30f);
    std::vector<int32_t> goal(P.n_levels, kDefaultTilesGoal);
    std::vector<uint8_t> stage(P.n_levels, 1), xcd(P.n_levels, 0);
    const bool was_timing = P.timing;
    P.timing = true;
    for (int32_t g : kTuneGoals) {
        retile(P, g);
        s = dev_upload_tiles(P, ws, st);
        if (s != BX_OK) { P.timing = was_timing; return s; }
        std::fill(P.level_nt.begin(), P.level_nt.end(), (uint8_t)0);
        for (int pass = 0; pass < 4 * reps; ++pass) {
            const int v = pass & 1, x = (pass >> 1) & 1;
            std::fill(P.level_stage.begin(), P.level_stage.end(), (uint8_t)v);
            std::fill(P.level_xcd.begin(), P.level_xcd.end(), (uint8_t)x);
            s = launch_util(P, ws, BX_SCHED_LEVEL, st);
            if (s != BX_OK) { P.timing = was_timing; return s; }
            HIP_TRY(hipStreamSynchronize(st));
            for (int l = 0; l < P.n_levels; ++l) {
                if (P.level_tile_begin[l + 1] <= P.level_tile_begin[l]) continue;
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, static_cast<hipEvent_t>(P.lev_ev[2 * l]),
                                            static_cast<hipEvent_t>(P.lev_ev[2 * l + 1])));
                if (ms < best[l]) {
                    best[l] = ms;
                    goal[l] = g;
                    stage[l] = (uint8_t)v;
                    xcd[l] = (uint8_t)x;
                }
            }
        }
    }
    P.timing = was_timing;
    P.level_goal = goal;
    P.level_stage = stage;
    P.level_xcd = xcd;
    retile_levels(P);
    s = dev_upload_tiles(P, ws, st);
    if (s != BX_OK) return s;
    float pass_ms[2] = {1e30f, 1e30f};
    for (int pass = 0; pass < 2 * reps; ++pass) {
        const int w = pass & 1;
        std::fill(P.level_nt.begin(), P.level_nt.end(), (uint8_t)w);
        float ms = 0.f;
        s = time_pass(P, ws, BX_SCHED_LEVEL, st, &ms);
        if (s != BX_OK) return s;
        pass_ms[w] = std::min(pass_ms[w], ms);
    }
    std::fill(P.level_nt.begin(), P.level_nt.end(), (uint8_t)(pass_ms[1] < pass_ms[0] ? 1 : 0));
    return BX_OK;
}

// ------------------------------------------------------------ tuning cache
// What the autotuner chose for a plan, keyed by the plan's shape class: the
// device, the cost type, the flags and, level by level, every mini-bucket's
// table shape and code path -- everything the timings depend on and nothing
// they do not (the cost values).  Plans of one shape class (e.g. instances
// of one generator with other seeds) reuse the choice without timing.
struct TuneEntry {
    bx_schedule sched = BX_SCHED_LEVEL;
    uint8_t nt = 0;
    uint8_t pack = 0;              // packing of small mini-buckets on
    std::vector<int32_t> goal;
    std::vector<uint8_t> stage;
    std::vector<uint8_t> xcd;
};

uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;
    return h;
}

uint64_t shape_class(const Plan &P) {
    uint64_t h = 0xcbf29ce484222325ull;
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        h = fnv(h, prop.gcnArchName, std::strlen(prop.gcnArchName));
        h = fnv(h, &prop.multiProcessorCount, sizeof prop.multiProcessorCount);
    }
    // the packing limits and, per mini-bucket, what does not depend on the
    // packing mode in use (dependency level, not launch level; no code path)
    const int32_t head[7] = {(int32_t)P.ct, (int32_t)P.opt.flags, P.pack_max_rows, P.fuse_max_rows,
                             P.fuse_max_stages, P.fuse_max_stage_rows, P.pack_stage_rows};
    h = fnv(h, head, sizeof head);
    for (size_t g = 0; g < P.dmb.size(); ++g) {
        const DevMb &d = P.dmb[g];
        const int64_t v[9] = {P.mbs[g].dep_level, d.out_rows, d.D, d.nv, d.nf, d.nfl, d.nfi, d.nfc,
                              (int64_t)P.mbs[g].members.size()};
        h = fnv(h, v, sizeof v);
        h = fnv(h, d.dims, sizeof(int32_t) * (size_t)d.nv);
    }
    return h;
}

std::map<uint64_t, TuneEntry> &tune_memory() {
    static std::map<uint64_t, TuneEntry> m;
    return m;
}
std::mutex &tune_mutex() {
    static std::mutex m;
    return m;
}

// One line per entry: "bxtune2 <key hex> <sched> <nt> <pack> <levels> g:s g:s ...",
// s = staging (bit 0) | XCD order (bit 1).
bool read_cache_file(const char *path, uint64_t key, TuneEntry &out) {
    std::FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char tag[16];
    unsigned long long k = 0;
    int sched = 0, nt = 0, pack = 0, nl = 0;
    bool found = false;
    while (!found && std::fscanf(f, "%15s %llx %d %d %d %d", tag, &k, &sched, &nt, &pack, &nl) == 6) {
        TuneEntry e;
        bool ok = std::strcmp(tag, "bxtune2") == 0 && nl >= 0 && nl < (1 << 20);
        for (int l = 0; ok && l < nl; ++l) {
            int g = 0, s = 0;
            if (std::fscanf(f, "%d:%d", &g, &s) != 2) ok = false;
            e.goal.push_back(g);
            e.stage.push_back((uint8_t)(s & 1));
            e.xcd.push_back((uint8_t)((s >> 1) & 1));
        }
        if (!ok) break;
        if (k == key && (sched == BX_SCHED_LEVEL || sched == BX_SCHED_PER_BUCKET)) {
            e.sched = (bx_schedule)sched;
            e.nt = (uint8_t)(nt != 0);
            e.pack = (uint8_t)(pack != 0);
            out = e;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void append_cache_file(const char *path, uint64_t key, const TuneEntry &e) {
    std::FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "bxtune2 %016llx %d %d %d %d", (unsigned long long)key, (int)e.sched, (int)e.nt,
                 (int)e.pack, (int)e.goal.size());
    for (size_t l = 0; l < e.goal.size(); ++l)
        std::fprintf(f, " %d:%d", e.goal[l], (int)e.stage[l] | (l < e.xcd.size() && e.xcd[l] ? 2 : 0));
    std::fprintf(f, "\n");
    std::fclose(f);
}

bool tile_goal_known(int32_t g) {
    for (int32_t x : kTuneGoals)
        if (x == g) return true;
    return false;
}

}  // namespace

bx_status dev_upload(Plan &P, void *ws, size_t bytes, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return set_error(BX_E_INVALID, "workspace must be 256-byte aligned");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    for (const PInst &I : P.inst)
        if (I.n > kSigmaCap) return set_error(BX_E_UNSUPPORTED, "more than 16384 variables in one problem");
    if (P.dtile.size() > P.tile_cap)
        return set_error(BX_E_INVALID, "internal: the tile list exceeds its workspace region");
    if (P.dseg.size() > P.seg_cap)
        return set_error(BX_E_INVALID, "internal: the segment list exceeds its workspace region");
    std::vector<uint8_t> img(P.static_bytes, 0);
    put(img, P.off_mb, P.dmb);
    put(img, P.off_fn, P.dfn);
    put(img, P.off_tile, P.dtile);
    put(img, P.off_seg, P.dseg);
    put(img, P.off_var, P.dvar);
    put(img, P.off_vfn, P.dvfn);
    put(img, P.off_term, P.dterm);
    put(img, P.off_occ, P.docc);
    put(img, P.off_pair, P.dpair);
    put(img, P.off_vlv, P.vlevel_var_begin);
    put(img, P.off_vlp, P.vlevel_pair_begin);
    put(img, P.off_inst, P.dinst);
    put(img, P.off_const, P.dconst);
    put(img, P.off_tables, P.tables);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    P.executed = false;
    return BX_OK;
}

// Re-uploads only the tile list and the mini-bucket descriptors (after a retile).
bx_status dev_upload_tiles(Plan &P, void *ws, hipStream_t st) {
    if (P.dtile.size() > P.tile_cap)
        return set_error(BX_E_INVALID, "internal: the tile list exceeds its workspace region");
    char *w = static_cast<char *>(ws);
    HIP_TRY(hipMemcpyAsync(w + P.off_mb, P.dmb.data(), P.dmb.size() * sizeof(DevMb), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + P.off_fn, P.dfn.data(), P.dfn.size() * sizeof(DevFn), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + P.off_tile, P.dtile.data(), P.dtile.size() * sizeof(DevTile),
                           hipMemcpyHostToDevice, st));
    if (P.dseg.size() > P.seg_cap)
        return set_error(BX_E_INVALID, "internal: the segment list exceeds its workspace region");
    if (!P.dseg.empty())
        HIP_TRY(hipMemcpyAsync(w + P.off_seg, P.dseg.data(), P.dseg.size() * sizeof(DevSeg), hipMemcpyHostToDevice,
                               st));
    HIP_TRY(hipStreamSynchronize(st));
    return BX_OK;
}

bx_status dev_execute(Plan &P, void *ws, size_t bytes, bx_schedule sched, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (sched == BX_SCHED_AUTO) sched = P.tuned_valid ? P.tuned : BX_SCHED_LEVEL;
    if (sched == BX_SCHED_DATAFLOW)
        return set_error(BX_E_UNSUPPORTED, "the dataflow schedule is disabled");
    const bool timed = P.timing && !P.capturing;
    if (timed) {
        bx_status es = ensure_events(P);
        if (es == BX_OK && sched == BX_SCHED_PER_BUCKET) es = ensure_mb_events(P);
        if (es != BX_OK) return es;
        HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[0]), st));
    }
    bx_status s = run(P, ws, sched, st);
    if (s != BX_OK) return s;
    if (timed) HIP_TRY(hipEventRecord(static_cast<hipEvent_t>(P.ev[2]), st));
    P.executed = true;
    P.timed_sched = timed ? sched : BX_SCHED_AUTO;
    return BX_OK;
}

bx_status dev_results(Plan &P, const void *ws, int32_t prob, double *bound, double *ub,
                      int32_t *assignment, void *stream) {
    if (!P.executed) return set_error(BX_E_STATE, "results requested before execute");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *w = static_cast<const char *>(ws);
    DevResult r{};
    HIP_TRY(hipMemcpyAsync(&r, w + P.off_results + sizeof(DevResult) * prob, sizeof r,
                           hipMemcpyDeviceToHost, st));
    const PInst &I = P.inst[prob];
    if (assignment && I.n > 0)
        HIP_TRY(hipMemcpyAsync(assignment, w + P.off_sigma + P.dinst[prob].sigma_off,
                               sizeof(int32_t) * I.n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (P.timed_sched != BX_SCHED_AUTO) {
        HIP_TRY(hipEventElapsedTime(&P.last_util_ms, static_cast<hipEvent_t>(P.ev[0]),
                                    static_cast<hipEvent_t>(P.ev[1])));
        HIP_TRY(hipEventElapsedTime(&P.last_value_ms, static_cast<hipEvent_t>(P.ev[1]),
                                    static_cast<hipEvent_t>(P.ev[2])));
        P.last_util_kernel_ms = P.last_util_ms;
        P.last_level_ms.clear();
        if (P.timed_sched == BX_SCHED_LEVEL) {
            float sum = 0.f;
            P.last_level_ms.assign(P.n_levels, 0.f);
            for (int l = 0; l < P.n_levels; ++l) {
                if (P.level_tile_begin[l + 1] <= P.level_tile_begin[l]) continue;
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, static_cast<hipEvent_t>(P.lev_ev[2 * l]),
                                            static_cast<hipEvent_t>(P.lev_ev[2 * l + 1])));
                P.last_level_ms[l] = ms;
                sum += ms;
            }
            P.last_util_kernel_ms = sum;
        }
        P.last_mb_ms.clear();
        if (P.timed_sched == BX_SCHED_PER_BUCKET && P.mb_ev.size() == 2 * P.mbs.size()) {
            P.last_mb_ms.assign(P.mbs.size(), 0.f);
            for (size_t g = 0; g < P.mbs.size(); ++g) {
                if (P.mbs[g].n_tiles == 0) continue;
                HIP_TRY(hipEventElapsedTime(&P.last_mb_ms[g], static_cast<hipEvent_t>(P.mb_ev[2 * g]),
                                            static_cast<hipEvent_t>(P.mb_ev[2 * g + 1])));
            }
        }
        P.timed_sched = BX_SCHED_AUTO;
    }
    if (r.status != 0) return set_error(BX_E_DEVICE, "device reported a failure");
    if (bound) *bound = r.bound;
    if (ub) *ub = r.ub;
    return BX_OK;
}

// Captures one execute (UTIL launches + value kernel) into a hipGraph bound
// to this workspace; dev_graph_launch replays it.  The captured kernels
// contain no memset nodes.
bx_status dev_graph_create(Plan &P, void *ws, size_t bytes, bx_schedule sched, void *stream) {
    if (!ws) return set_error(BX_E_INVALID, "workspace is NULL");
    if (bytes < P.total_bytes) return set_error(BX_E_NOMEM, "workspace smaller than the plan needs");
    if (!stream) return set_error(BX_E_INVALID, "graph capture needs a non-null stream");
    if (sched == BX_SCHED_AUTO) sched = P.tuned_valid ? P.tuned : BX_SCHED_LEVEL;
    if (sched == BX_SCHED_DATAFLOW)
        return set_error(BX_E_UNSUPPORTED, "the dataflow schedule is disabled");
    hipStream_t st = static_cast<hipStream_t>(stream);
    drop_graph(P);
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    P.capturing = true;
    bx_status s = run(P, ws, sched, st);
    P.capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != BX_OK) { if (g) (void)hipGraphDestroy(g); return s; }
    if (e != hipSuccess) return set_error(BX_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return set_error(BX_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    P.graph = g;
    P.graph_exec = ge;
    P.graph_ws = ws;
    return BX_OK;
}

bx_status dev_graph_launch(Plan &P, void *stream) {
    if (!P.graph_exec)
        return set_error(BX_E_STATE, "no graph: call bx_plan_graph_create first (autotuning discards it)");
    HIP_TRY(hipGraphLaunch(static_cast<hipGraphExec_t>(P.graph_exec), static_cast<hipStream_t>(stream)));
    P.executed = true;
    return BX_OK;
}

bx_status dev_copy_table(const Plan &P, const void *ws, int64_t off, int64_t n, void *host,
                         void *stream) {
    (void)P;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *w = static_cast<const char *>(ws);
    HIP_TRY(hipMemcpyAsync(host, w + off * 4, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return BX_OK;
}

// Chooses, for BX_SCHED_AUTO, the per-level tile goals and staging and the
// blocked rows' store kind (tune_levels), then the schedule: one launch per
// level or one per mini-bucket, whichever ran a whole UTIL pass faster.  A
// shape class seen before (in this process, or in the options' cache file)
// takes the stored choice without timing.  The captured graph, if any, is
// discarded.
bx_status dev_autotune(Plan &P, void *ws, size_t bytes, int32_t reps, void *stream) {
    if (!ws || bytes < P.total_bytes) return set_error(BX_E_INVALID, "workspace missing or too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (reps < 1) reps = 1;
    drop_graph(P);
    const uint64_t key = shape_class(P);
    TuneEntry e;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        auto it = tune_memory().find(key);
        if (it != tune_memory().end()) { e = it->second; have = true; }
    }
    if (!have && !P.tune_cache.empty()) have = read_cache_file(P.tune_cache.c_str(), key, e);
    for (int32_t g : e.goal) have = have && tile_goal_known(g);
    if (have && e.pack != (uint8_t)P.pack_on) {
        if (e.pack && !P.pack_allowed) have = false;
        else {
            bx_status s = set_packing(P, e.pack != 0);
            if (s != BX_OK) return s;
        }
    }
    if (have && (int)e.goal.size() == P.n_levels) {
        P.level_goal = e.goal;
        P.level_stage = e.stage;
        P.level_xcd = e.xcd;
        retile_levels(P);
        std::fill(P.level_nt.begin(), P.level_nt.end(), e.nt);
        bx_status s = dev_upload_tiles(P, ws, st);
        if (s == BX_OK) s = run(P, ws, e.sched, st);
        if (s != BX_OK) return s;
        P.tuned = e.sched;
        P.tuned_valid = true;
        P.tune_cached = true;
        P.executed = true;
        return BX_OK;
    }
    // the level schedule tuned with packing on and off (when allowed), the
    // faster kept: whole passes, minimum over reps + 1 runs
    auto tune_mode = [&](TuneEntry &te, float &ms_out) -> bx_status {
        bx_status s2 = ensure_events(P);
        if (s2 == BX_OK) s2 = dev_upload_tiles(P, ws, st);
        if (s2 == BX_OK) s2 = run(P, ws, BX_SCHED_LEVEL, st);   // warm-up
        if (s2 == BX_OK) s2 = tune_levels(P, ws, reps + 1, st);
        if (s2 != BX_OK) return s2;
        ms_out = 1e30f;
        for (int r = 0; r <= reps; ++r) {
            float ms = 0.f;
            s2 = time_pass(P, ws, BX_SCHED_LEVEL, st, &ms);
            if (s2 != BX_OK) return s2;
            ms_out = std::min(ms_out, ms);
        }
        te.goal = P.level_goal;
        te.stage = P.level_stage;
        te.xcd = P.level_xcd;
        te.nt = P.level_nt.empty() ? 0 : P.level_nt[0];
        te.pack = (uint8_t)P.pack_on;
        return BX_OK;
    };
    float lv = 1e30f;
    bx_status s = tune_mode(e, lv);
    if (s != BX_OK) return s;
    P.tune_pack_ms[P.pack_on ? 1 : 0] = lv;
    P.tune_pack_ms[P.pack_on ? 0 : 1] = 0.f;
    if (P.pack_allowed) {
        TuneEntry other;
        float lv2 = 1e30f;
        s = set_packing(P, !P.pack_on);
        if (s == BX_OK) s = tune_mode(other, lv2);
        if (s != BX_OK) return s;
        P.tune_pack_ms[P.pack_on ? 1 : 0] = lv2;
        if (lv2 < lv) {
            e = other;
            lv = lv2;
        } else {   // back to the first mode and its tuning
            s = set_packing(P, e.pack != 0);
            if (s != BX_OK) return s;
            P.level_goal = e.goal;
            P.level_stage = e.stage;
            P.level_xcd = e.xcd;
            retile_levels(P);
            std::fill(P.level_nt.begin(), P.level_nt.end(), e.nt);
            s = dev_upload_tiles(P, ws, st);
            if (s != BX_OK) return s;
        }
    }
    // schedule: whole passes of the per-bucket schedule against the level one
    float pb = 1e30f;
    for (int r = 0; r <= reps; ++r) {
        float ms = 0.f;
        s = time_pass(P, ws, BX_SCHED_PER_BUCKET, st, &ms);
        if (s != BX_OK) return s;
        pb = std::min(pb, ms);
        if (pb > 4.f * lv) break;      // far behind: no need for more samples
    }
    e.sched = pb < lv ? BX_SCHED_PER_BUCKET : BX_SCHED_LEVEL;
    s = run(P, ws, e.sched, st);   // leaves valid results
    if (s != BX_OK) return s;
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        tune_memory()[key] = e;
    }
    if (!P.tune_cache.empty()) append_cache_file(P.tune_cache.c_str(), key, e);
    P.tuned = e.sched;
    P.tuned_valid = true;
    P.tune_cached = false;
    P.tune_pass_ms[0] = lv;
    P.tune_pass_ms[1] = pb;
    P.executed = true;
    return BX_OK;
}

bx_status dev_stream_probe(int32_t kind, void *dst, const void *src, size_t bytes, int32_t grid, void *stream) {
    if (kind < 0 || kind > 2) return set_error(BX_E_INVALID, "unknown probe kind");
    if (bytes % 16 || bytes == 0) return set_error(BX_E_INVALID, "bytes must be a positive multiple of 16");
    if ((kind != 2 && (!dst || reinterpret_cast<uintptr_t>(dst) % 16)) ||
        (kind != 1 && (!src || reinterpret_cast<uintptr_t>(src) % 16)) || (kind == 2 && !dst))
        return set_error(BX_E_INVALID, "NULL or unaligned buffer");
    if (grid <= 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = 8 * cus;
    }
    launch_stream(kind, dst, src, (int64_t)(bytes / 16), grid, static_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return BX_OK;
}

void dev_release(Plan &P) {
    for (void *&e : P.ev)
        if (e) { (void)hipEventDestroy(static_cast<hipEvent_t>(e)); e = nullptr; }
    for (void *e : P.lev_ev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    P.lev_ev.clear();
    for (void *e : P.mb_ev) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    P.mb_ev.clear();
    drop_graph(P);
}

}  // namespace bx
