// extern "C" entry points of include/bx.h: argument checks, ownership and
// error reporting around the planner (bx_plan.cpp) and the device side
// (bx_exec.hip).  No exception crosses the ABI.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include <algorithm>

#include "bx_internal.h"

struct bx_problem {
    bx::Problem p;
};
struct bx_plan {
    bx::Plan p;
};

namespace bx {
namespace {
thread_local std::string g_last_error;
}
bx_status set_error(bx_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}
const char *last_error_cstr() { return g_last_error.c_str(); }
}  // namespace bx

using bx::set_error;

#define BX_GUARD_BEGIN try {
#define BX_GUARD_END                                                          \
    }                                                                         \
    catch (const std::bad_alloc &) {                                          \
        return set_error(BX_E_NOMEM, "host allocation failed");               \
    }                                                                         \
    catch (const std::exception &e) {                                         \
        return set_error(BX_E_INVALID, std::string("internal error: ") + e.what()); \
    }                                                                         \
    catch (...) {                                                             \
        return set_error(BX_E_INVALID, "internal error");                     \
    }

extern "C" {

void bx_options_default(bx_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->algo = BX_ALGO_BE;
    opt->ibound = 0;
    opt->order = BX_ORDER_MIN_FILL;
    opt->partition = BX_PART_GREEDY;
    opt->schedule = BX_SCHED_AUTO;
    opt->max_table_entries = 0;
    opt->flags = 0;
    opt->tune_cache = nullptr;
}

bx_status bx_problem_create(int32_t n_vars, const int32_t *domain_sizes, bx_cost_type cost_type,
                            bx_problem **out) {
    BX_GUARD_BEGIN
    if (!out) return set_error(BX_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_vars < 0) return set_error(BX_E_INVALID, "n_vars < 0");
    if (n_vars > 0 && !domain_sizes) return set_error(BX_E_INVALID, "domain_sizes is NULL");
    if (cost_type != BX_COST_I32 && cost_type != BX_COST_F32)
        return set_error(BX_E_INVALID, "unknown cost type");
    for (int32_t i = 0; i < n_vars; ++i)
        if (domain_sizes[i] < 1 || domain_sizes[i] > bx::kMaxDomain)
            return set_error(BX_E_INVALID, "domain size must be in [1, 1024]");
    bx_problem *p = new bx_problem;
    p->p.n = n_vars;
    p->p.dom.assign(domain_sizes, domain_sizes + n_vars);
    p->p.ct = cost_type;
    *out = p;
    return BX_OK;
    BX_GUARD_END
}

static bx_status check_scope(const bx::Problem &P, int32_t arity, const int32_t *scope,
                             int64_t n_entries) {
    if (arity < 0) return set_error(BX_E_INVALID, "arity < 0");
    if (arity > 0 && !scope) return set_error(BX_E_INVALID, "scope is NULL");
    int64_t size = 1;
    for (int32_t j = 0; j < arity; ++j) {
        if (scope[j] < 0 || scope[j] >= P.n) return set_error(BX_E_INVALID, "scope variable out of range");
        for (int32_t q = 0; q < j; ++q)
            if (scope[q] == scope[j]) return set_error(BX_E_INVALID, "repeated variable in scope");
        size *= P.dom[scope[j]];
        if (size > (int64_t)1 << 40) return set_error(BX_E_TOO_LARGE, "table too large");
    }
    if (size != n_entries)
        return set_error(BX_E_INVALID, "n_entries " + std::to_string(n_entries) +
                                           " differs from the product of the domains " + std::to_string(size));
    return BX_OK;
}

bx_status bx_problem_add_function(bx_problem *p, int32_t arity, const int32_t *scope,
                                  const void *table, int64_t n_entries) {
    BX_GUARD_BEGIN
    if (!p) return set_error(BX_E_INVALID, "problem is NULL");
    bx_status s = check_scope(p->p, arity, scope, n_entries);
    if (s != BX_OK) return s;
    if (!table) return set_error(BX_E_INVALID, "table is NULL");
    bx::Function f;
    f.scope.assign(scope, scope + arity);
    if (p->p.ct == BX_COST_I32) {
        const int32_t *t = static_cast<const int32_t *>(table);
        for (int64_t i = 0; i < n_entries; ++i)
            if (t[i] < 0) return set_error(BX_E_INVALID, "negative cost");
        f.ti.assign(t, t + n_entries);
    } else {
        const float *t = static_cast<const float *>(table);
        for (int64_t i = 0; i < n_entries; ++i)
            if (!(t[i] >= 0.f)) return set_error(BX_E_INVALID, "negative or NaN cost");
        f.tf.assign(t, t + n_entries);
    }
    p->p.fns.push_back(std::move(f));
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_problem_add_prob_table(bx_problem *p, int32_t arity, const int32_t *scope,
                                    const double *probs, int64_t n_entries) {
    BX_GUARD_BEGIN
    if (!p) return set_error(BX_E_INVALID, "problem is NULL");
    if (p->p.ct != BX_COST_F32) return set_error(BX_E_INVALID, "probability tables need BX_COST_F32");
    bx_status s = check_scope(p->p, arity, scope, n_entries);
    if (s != BX_OK) return s;
    if (!probs) return set_error(BX_E_INVALID, "probs is NULL");
    bx::Function f;
    f.scope.assign(scope, scope + arity);
    f.tf.resize(n_entries);
    for (int64_t i = 0; i < n_entries; ++i) {
        double q = probs[i];
        if (!(q >= 0.0 && q <= 1.0)) return set_error(BX_E_INVALID, "probability outside [0, 1]");
        // MPE as min-sum (Sec. 3): cost = -ln p, rounded to the nearest float
        f.tf[i] = q == 0.0 ? INFINITY : (float)(-std::log(q));
        if (f.tf[i] == -0.0f) f.tf[i] = 0.0f;
    }
    p->p.fns.push_back(std::move(f));
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_problem_set_order(bx_problem *p, const int32_t *order) {
    BX_GUARD_BEGIN
    if (!p) return set_error(BX_E_INVALID, "problem is NULL");
    if (p->p.n > 0 && !order) return set_error(BX_E_INVALID, "order is NULL");
    std::vector<char> seen(p->p.n, 0);
    for (int32_t i = 0; i < p->p.n; ++i) {
        if (order[i] < 0 || order[i] >= p->p.n || seen[order[i]])
            return set_error(BX_E_INVALID, "order is not a permutation");
        seen[order[i]] = 1;
    }
    p->p.order.assign(order, order + p->p.n);
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_problem_set_pseudotree(bx_problem *p, const int32_t *parent) {
    BX_GUARD_BEGIN
    if (!p) return set_error(BX_E_INVALID, "problem is NULL");
    if (p->p.n > 0 && !parent) return set_error(BX_E_INVALID, "parent is NULL");
    std::vector<int32_t> par(parent, parent + p->p.n);
    // validated fully at plan time (needs the final function set); check shape now
    for (int32_t v = 0; v < p->p.n; ++v)
        if (par[v] < -1 || par[v] >= p->p.n || par[v] == v)
            return set_error(BX_E_INVALID, "pseudo-tree: parent out of range");
    p->p.parent = std::move(par);
    return BX_OK;
    BX_GUARD_END
}

int32_t bx_problem_num_vars(const bx_problem *p) { return p ? p->p.n : -1; }

void bx_problem_destroy(bx_problem *p) { delete p; }

bx_status bx_compute_order(const bx_problem *p, bx_order_heuristic h, int32_t *order_out,
                           int32_t *parent_out) {
    BX_GUARD_BEGIN
    if (!p || (p->p.n > 0 && !order_out)) return set_error(BX_E_INVALID, "NULL argument");
    std::vector<int32_t> o, par;
    bx_status s = bx::compute_order(p->p, h, o, par);
    if (s != BX_OK) return s;
    std::copy(o.begin(), o.end(), order_out);
    if (parent_out) std::copy(par.begin(), par.end(), parent_out);
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_induced_width(const bx_problem *p, const int32_t *order, int32_t *width_out) {
    BX_GUARD_BEGIN
    if (!p || !width_out || (p->p.n > 0 && !order)) return set_error(BX_E_INVALID, "NULL argument");
    std::vector<int32_t> o(order, order + p->p.n);
    std::vector<char> seen(p->p.n, 0);
    for (int32_t v : o) {
        if (v < 0 || v >= p->p.n || seen[v]) return set_error(BX_E_INVALID, "order is not a permutation");
        seen[v] = 1;
    }
    *width_out = bx::induced_width(p->p, o);
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_plan_create(bx_problem *const *probs, int32_t n_probs, const bx_options *opt,
                         bx_plan **out) {
    BX_GUARD_BEGIN
    if (!out) return set_error(BX_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!probs || n_probs < 1) return set_error(BX_E_INVALID, "no problems");
    bx_options o;
    if (opt) o = *opt; else bx_options_default(&o);
    if (o.flags & ~BX_FLAG_ALL) return set_error(BX_E_INVALID, "unknown bits in flags");
    if (o.pack_max_rows < 0 || o.fuse_max_rows < 0 || o.fuse_max_stages < 0 || o.fuse_max_stage_rows < 0 ||
        o.pack_stage_rows < 0)
        return set_error(BX_E_INVALID, "packing limits must be >= 0");
    if (o.algo < BX_ALGO_BE || o.algo > BX_ALGO_MBE_SUM) return set_error(BX_E_INVALID, "unknown algorithm");
    if (o.partition != BX_PART_GREEDY)
        return set_error(BX_E_UNSUPPORTED, "only the greedy partition is available in bx_plan_create");
    std::vector<const bx::Problem *> ps;
    for (int32_t i = 0; i < n_probs; ++i) {
        if (!probs[i]) return set_error(BX_E_INVALID, "problem is NULL");
        ps.push_back(&probs[i]->p);
    }
    bx_plan *pl = new bx_plan;
    bx_status s = bx::build_plan(ps, o, pl->p);
    if (s != BX_OK) { delete pl; return s; }
    *out = pl;
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_plan_workspace_bytes(const bx_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return set_error(BX_E_INVALID, "NULL argument");
    *bytes = plan->p.total_bytes;
    return BX_OK;
}

bx_status bx_plan_upload(bx_plan *plan, void *d_workspace, size_t bytes, void *stream) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    return bx::dev_upload(plan->p, d_workspace, bytes, stream);
    BX_GUARD_END
}

bx_status bx_plan_execute(bx_plan *plan, void *d_workspace, size_t bytes, void *stream) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    return bx::dev_execute(plan->p, d_workspace, bytes, plan->p.opt.schedule, stream);
    BX_GUARD_END
}

bx_status bx_plan_execute_sched(bx_plan *plan, void *d_workspace, size_t bytes, bx_schedule sched,
                                void *stream) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    if (sched < BX_SCHED_PER_BUCKET || sched > BX_SCHED_AUTO) return set_error(BX_E_INVALID, "unknown schedule");
    return bx::dev_execute(plan->p, d_workspace, bytes, sched, stream);
    BX_GUARD_END
}

bx_status bx_plan_results(bx_plan *plan, const void *d_workspace, int32_t prob, double *bound,
                          double *ub, int32_t *assignment, void *stream) {
    BX_GUARD_BEGIN
    if (!plan || !d_workspace) return set_error(BX_E_INVALID, "NULL argument");
    if (prob < 0 || prob >= (int32_t)plan->p.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    return bx::dev_results(plan->p, d_workspace, prob, bound, ub, assignment, stream);
    BX_GUARD_END
}

bx_status bx_plan_get_stats(const bx_plan *plan, bx_plan_stats *st) {
    if (!plan || !st) return set_error(BX_E_INVALID, "NULL argument");
    const bx::Plan &P = plan->p;
    st->n_minibuckets = (int64_t)P.mbs.size();
    st->util_rows = P.util_rows;
    st->joint_entries = P.joint_entries;
    st->algo_bytes = P.algo_bytes;
    st->n_levels = P.n_levels;
    st->n_tiles = P.level_tile_begin.empty() ? 0 : P.level_tile_begin[P.n_levels];   // level schedule
    st->max_scope = P.max_scope;
    st->value_levels = P.max_value_levels;
    st->tile_capacity = (int64_t)P.tile_cap;
    return BX_OK;
}

bx_status bx_plan_num_minibuckets(const bx_plan *plan, int32_t prob, int32_t *count) {
    if (!plan || !count) return set_error(BX_E_INVALID, "NULL argument");
    if (prob < 0 || prob >= (int32_t)plan->p.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    *count = (int32_t)plan->p.inst[prob].mbs.size();
    return BX_OK;
}

bx_status bx_plan_minibucket_info(const bx_plan *plan, int32_t prob, int32_t i, int32_t *var,
                                  int32_t *n_members, int32_t *members, int32_t *out_id,
                                  int32_t *out_arity, int32_t *out_scope, int64_t *out_rows) {
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    if (prob < 0 || prob >= (int32_t)plan->p.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    const bx::PInst &I = plan->p.inst[prob];
    if (i < 0 || i >= (int32_t)I.mbs.size()) return set_error(BX_E_INVALID, "mini-bucket index out of range");
    const bx::PMb &mb = plan->p.mbs[I.mbs[i]];
    if (var) *var = mb.var;
    if (n_members) *n_members = (int32_t)mb.members.size();
    if (members)
        for (size_t k = 0; k < mb.members.size() && k < 256; ++k) members[k] = mb.members[k];
    if (out_id) *out_id = mb.out_id;
    if (out_arity) *out_arity = (int32_t)mb.U.size() - 1;
    if (out_scope)
        for (size_t k = 0; k + 1 < mb.U.size() && k < 64; ++k) out_scope[k] = mb.U[k];
    if (out_rows) *out_rows = mb.out_rows;
    return BX_OK;
}

bx_status bx_plan_order(const bx_plan *plan, int32_t prob, int32_t *order_out) {
    if (!plan || !order_out) return set_error(BX_E_INVALID, "NULL argument");
    if (prob < 0 || prob >= (int32_t)plan->p.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    const bx::PInst &I = plan->p.inst[prob];
    std::copy(I.order.begin(), I.order.end(), order_out);
    return BX_OK;
}

bx_status bx_plan_util_table(const bx_plan *plan, const void *d_workspace, int32_t prob, int32_t i,
                             void *host_out, int64_t n_entries, void *stream) {
    BX_GUARD_BEGIN
    if (!plan || !d_workspace || !host_out) return set_error(BX_E_INVALID, "NULL argument");
    if (prob < 0 || prob >= (int32_t)plan->p.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    const bx::PInst &I = plan->p.inst[prob];
    if (i < 0 || i >= (int32_t)I.mbs.size()) return set_error(BX_E_INVALID, "mini-bucket index out of range");
    const bx::PMb &mb = plan->p.mbs[I.mbs[i]];
    if (n_entries != mb.out_rows) return set_error(BX_E_INVALID, "n_entries differs from the table size");
    return bx::dev_copy_table(plan->p, d_workspace, mb.out_off, mb.out_rows, host_out, stream);
    BX_GUARD_END
}

bx_status bx_plan_stream_bytes(const bx_plan *plan, int64_t chunk_rows, size_t *device_bytes, size_t *host_bytes) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    return bx::stream_bytes(plan->p, chunk_rows, device_bytes, host_bytes);
    BX_GUARD_END
}

bx_status bx_plan_execute_streamed(bx_plan *plan, void *d_workspace, size_t bytes, void *h_tables,
                                   size_t host_bytes, int64_t chunk_rows, void *stream, double *bounds) {
    BX_GUARD_BEGIN
    if (!plan || !bounds) return set_error(BX_E_INVALID, "NULL argument");
    return bx::dev_execute_streamed(plan->p, d_workspace, bytes, h_tables, host_bytes, chunk_rows, stream, bounds);
    BX_GUARD_END
}

bx_status bx_plan_stream_table(const bx_plan *plan, const void *h_tables, int32_t prob, int32_t i, void *host_out,
                               int64_t n_entries) {
    BX_GUARD_BEGIN
    if (!plan || !h_tables || !host_out) return set_error(BX_E_INVALID, "NULL argument");
    const bx::Plan &P = plan->p;
    if (prob < 0 || prob >= (int32_t)P.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    const bx::PInst &I = P.inst[prob];
    if (i < 0 || i >= (int32_t)I.mbs.size()) return set_error(BX_E_INVALID, "mini-bucket index out of range");
    const bx::PMb &mb = P.mbs[I.mbs[i]];
    if (n_entries != mb.out_rows) return set_error(BX_E_INVALID, "n_entries differs from the table size");
    if (mb.out_id < 0) return set_error(BX_E_INVALID, "a scalar output stays on the device (it is in the bound)");
    const char *src = static_cast<const char *>(h_tables) + (size_t)(mb.out_off * 4 - (int64_t)P.off_tables);
    std::memcpy(host_out, src, (size_t)n_entries * 4);
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_plan_level_info(const bx_plan *plan, int32_t level, bx_level_info *info) {
    if (!plan || !info) return set_error(BX_E_INVALID, "NULL argument");
    const bx::Plan &P = plan->p;
    if (level < 0 || level >= P.n_levels) return set_error(BX_E_INVALID, "level out of range");
    bx_level_info r{};
    for (size_t g = 0; g < P.mbs.size(); ++g) {
        if (P.mbs[g].level != level) continue;
        ++r.n_minibuckets;
        r.util_rows += P.mbs[g].out_rows;
        r.algo_bytes += P.mbs[g].algo_bytes;
        r.n_blocked += P.dmb[g].blk != 0;
        r.n_packed += P.dmb[g].path == 3;
    }
    r.n_tiles = P.level_tile_begin[level + 1] - P.level_tile_begin[level];
    r.n_row_tiles = P.level_lane_begin[level] - P.level_row_begin[level];
    r.n_lane_tiles = P.level_tile_begin[level + 1] - P.level_lane_begin[level];
    r.n_pack_tiles = P.level_tiled_begin[level] - P.level_pack_begin[level];
    r.staged = bx::level_stage_on(P, level) ? 1 : 0;
    r.nontemporal = bx::level_nt_on(P, level) ? 1 : 0;
    r.tile_goal = P.level_goal.empty() ? 0 : P.level_goal[level];
    *info = r;
    return BX_OK;
}

bx_status bx_plan_validate(const bx_plan *plan) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    return bx::validate_schedule(plan->p);
    BX_GUARD_END
}

bx_status bx_plan_level_timing(const bx_plan *plan, float *ms_out, int32_t n_levels) {
    if (!plan || !ms_out) return set_error(BX_E_INVALID, "NULL argument");
    const bx::Plan &P = plan->p;
    if (n_levels != P.n_levels) return set_error(BX_E_INVALID, "n_levels differs from the plan's level count");
    if ((int32_t)P.last_level_ms.size() != P.n_levels)
        return set_error(BX_E_STATE, "no timed LEVEL execute has been read back");
    std::copy(P.last_level_ms.begin(), P.last_level_ms.end(), ms_out);
    return BX_OK;
}

bx_status bx_plan_minibucket_timing(const bx_plan *plan, int32_t prob, float *ms_out, int32_t n) {
    if (!plan || !ms_out) return set_error(BX_E_INVALID, "NULL argument");
    const bx::Plan &P = plan->p;
    if (prob < 0 || prob >= (int32_t)P.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    const bx::PInst &I = P.inst[prob];
    if (n != (int32_t)I.mbs.size()) return set_error(BX_E_INVALID, "n differs from the problem's mini-bucket count");
    if (P.last_mb_ms.size() != P.mbs.size())
        return set_error(BX_E_STATE, "no timed PER_BUCKET execute has been read back");
    for (int32_t k = 0; k < n; ++k) ms_out[k] = P.last_mb_ms[I.mbs[k]];
    return BX_OK;
}

bx_status bx_plan_simulated_runtime(const bx_plan *plan, int32_t prob, const float *mb_ms, double latency_ms,
                                    double *util_ms, double *value_ms, int32_t *value_hops) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    const bx::Plan &P = plan->p;
    if (prob < 0 || prob >= (int32_t)P.inst.size()) return set_error(BX_E_INVALID, "problem index out of range");
    if (!(latency_ms >= 0.0)) return set_error(BX_E_INVALID, "latency must be >= 0");
    const bx::PInst &I = P.inst[prob];
    std::vector<float> t(I.mbs.size());
    if (mb_ms) {
        std::copy(mb_ms, mb_ms + I.mbs.size(), t.begin());
    } else {
        if (P.last_mb_ms.size() != P.mbs.size())
            return set_error(BX_E_STATE, "no timed PER_BUCKET execute has been read back");
        for (size_t k = 0; k < I.mbs.size(); ++k) t[k] = P.last_mb_ms[I.mbs[k]];
    }
    return bx::simulated_runtime(P, prob, t.data(), latency_ms, util_ms, value_ms, value_hops);
    BX_GUARD_END
}

bx_status bx_bnb_workspace_bytes(const bx_problem *p, const bx_options *opt, size_t *bytes) {
    BX_GUARD_BEGIN
    if (!p || !opt || !bytes) return set_error(BX_E_INVALID, "NULL argument");
    if (opt->flags & ~BX_FLAG_ALL) return set_error(BX_E_INVALID, "unknown bits in flags");
    // the root plan and the first expansion's batch (one child per value of
    // the first variable), with a quarter of slack for deeper batches
    bx::Problem q = p->p;
    if (q.order.empty()) {
        std::vector<int32_t> parent;
        bx_status s = bx::compute_order(q, opt->order, q.order, parent);
        if (s != BX_OK) return s;
    }
    bx::Plan root;
    std::vector<const bx::Problem *> ps{&q};
    bx_status s = bx::build_plan(ps, *opt, root);
    if (s != BX_OK) return s;
    size_t need = root.total_bytes;
    if (q.n > 0) {
        std::vector<const bx::Problem *> batch(q.dom[q.order[0]], &q);
        bx::Plan first;
        s = bx::build_plan(batch, *opt, first);
        if (s != BX_OK) return s;
        need = std::max(need, first.total_bytes);
    }
    *bytes = need + need / 4;
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_bnb_solve(const bx_problem *p, const bx_options *opt, void *d_workspace, size_t bytes,
                       void *stream, int64_t max_nodes, double *value, int32_t *assignment, int64_t *stats) {
    BX_GUARD_BEGIN
    if (!p || !opt) return set_error(BX_E_INVALID, "NULL argument");
    if (opt->flags & ~BX_FLAG_ALL) return set_error(BX_E_INVALID, "unknown bits in flags");
    if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % 256)
        return set_error(BX_E_INVALID, "workspace must be a non-NULL 256-byte aligned device pointer");
    if (max_nodes < 0) return set_error(BX_E_INVALID, "max_nodes must be >= 0");
    return bx::bnb_solve(p->p, *opt, d_workspace, bytes, stream, max_nodes, value, assignment, stats);
    BX_GUARD_END
}

bx_status bx_stream_probe(int32_t kind, void *d_dst, const void *d_src, size_t bytes, int32_t grid,
                          void *stream) {
    BX_GUARD_BEGIN
    return bx::dev_stream_probe(kind, d_dst, d_src, bytes, grid, stream);
    BX_GUARD_END
}

bx_status bx_plan_autotune(bx_plan *plan, void *d_workspace, size_t bytes, int32_t reps, void *stream) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    return bx::dev_autotune(plan->p, d_workspace, bytes, reps, stream);
    BX_GUARD_END
}

bx_status bx_plan_describe(const bx_plan *plan, char *buf, size_t cap) {
    if (!plan || !buf || cap == 0) return set_error(BX_E_INVALID, "NULL argument");
    const bx::Plan &P = plan->p;
    static const char *names[] = {"per-bucket", "level", "dataflow", "auto"};
    bx_schedule s = P.tuned_valid ? P.tuned : P.opt.schedule;
    if (s == BX_SCHED_AUTO) s = BX_SCHED_LEVEL;
    int staged = 0, blocked = 0, nt = 0, xcd = 0;
    for (int l = 0; l < P.n_levels; ++l) {
        staged += bx::level_stage_on(P, l);
        nt += bx::level_nt_on(P, l);
        xcd += bx::level_xcd_on(P, l);
    }
    for (const bx::DevMb &d : P.dmb) blocked += d.blk != 0;
    // levels per tile goal
    std::string goals;
    for (int32_t g : bx::kTuneGoals) {
        int n = 0;
        for (int32_t x : P.level_goal) n += x == g;
        goals += (goals.empty() ? "" : ",") + std::to_string(g) + ":" + std::to_string(n);
    }
    std::snprintf(buf, cap,
                  "schedule=%s tuned=%d cached=%d tile_goals=%s block=%d levels=%d staged_levels=%d "
                  "nontemporal_levels=%d xcd_levels=%d blocked_minibuckets=%d packing=%d packed_minibuckets=%d "
                  "groups=%d "
                  "tuned_ms_unpacked=%.3f tuned_ms_packed=%.3f tiles=%d flags=%u",
                  names[s], (int)P.tuned_valid, (int)P.tune_cached, goals.c_str(), bx::kUtilThreads, P.n_levels,
                  staged, nt, xcd, blocked, (int)P.pack_on, P.n_packed, P.n_groups, P.tune_pack_ms[0],
                  P.tune_pack_ms[1], P.level_tile_begin.empty() ? 0 : P.level_tile_begin[P.n_levels],
                  (unsigned)P.opt.flags);
    return BX_OK;
}

bx_status bx_plan_set_timing(bx_plan *plan, int32_t enabled) {
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    plan->p.timing = enabled != 0;
    return BX_OK;
}

bx_status bx_plan_last_timing(const bx_plan *plan, float *util_ms, float *util_kernel_ms,
                              float *value_ms) {
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    if (util_ms) *util_ms = plan->p.last_util_ms;
    if (util_kernel_ms) *util_kernel_ms = plan->p.last_util_kernel_ms;
    if (value_ms) *value_ms = plan->p.last_value_ms;
    return BX_OK;
}

bx_status bx_plan_graph_create(bx_plan *plan, void *d_workspace, size_t bytes, bx_schedule sched,
                               void *stream) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    if (sched < BX_SCHED_PER_BUCKET || sched > BX_SCHED_AUTO) return set_error(BX_E_INVALID, "unknown schedule");
    return bx::dev_graph_create(plan->p, d_workspace, bytes, sched, stream);
    BX_GUARD_END
}

bx_status bx_plan_graph_launch(bx_plan *plan, void *stream) {
    BX_GUARD_BEGIN
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    return bx::dev_graph_launch(plan->p, stream);
    BX_GUARD_END
}

void bx_plan_destroy(bx_plan *plan) {
    if (!plan) return;
    bx::dev_release(plan->p);
    delete plan;
}

int32_t bx_partition_num_features(void) { return bx::kPartFeatures; }

namespace {
struct ChooserCtx {
    bx_partition_chooser fn;
    void *user;
};
bx_status call_chooser(void *c, int32_t n_dec, const int32_t *dec_inst, const int32_t *off, const float *feats,
                       int32_t *choices) {
    ChooserCtx *ctx = static_cast<ChooserCtx *>(c);
    bx_status s = ctx->fn(ctx->user, n_dec, dec_inst, off, feats, choices);
    if (s != BX_OK && bx::last_error_cstr()[0] == '\0') return set_error(s, "partition chooser failed");
    return s;
}

bx_status plan_with(bx_problem *const *probs, int32_t n_probs, const bx_options *opt, bx::Chooser ch,
                    void *ctx, bx_plan **out) {
    if (!out) return set_error(BX_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!probs || n_probs < 1) return set_error(BX_E_INVALID, "no problems");
    if (!opt) return set_error(BX_E_INVALID, "options are NULL");
    bx_options o = *opt;
    if (o.algo != BX_ALGO_MBE && o.algo != BX_ALGO_ADPOP)
        return set_error(BX_E_INVALID, "partition choices apply to MBE / ADPOP");
    if (o.flags & ~BX_FLAG_ALL) return set_error(BX_E_INVALID, "unknown bits in flags");
    if (o.pack_max_rows < 0 || o.fuse_max_rows < 0 || o.fuse_max_stages < 0 || o.fuse_max_stage_rows < 0 ||
        o.pack_stage_rows < 0)
        return set_error(BX_E_INVALID, "packing limits must be >= 0");
    o.partition = BX_PART_LEARNED;
    std::vector<const bx::Problem *> ps;
    for (int32_t i = 0; i < n_probs; ++i) {
        if (!probs[i]) return set_error(BX_E_INVALID, "problem is NULL");
        ps.push_back(&probs[i]->p);
    }
    bx_plan *pl = new bx_plan;
    bx_status s = bx::build_plan(ps, o, pl->p, ch, ctx);
    if (s != BX_OK) { delete pl; return s; }
    *out = pl;
    return BX_OK;
}
}  // namespace

bx_status bx_plan_create_chooser(bx_problem *const *probs, int32_t n_probs, const bx_options *opt,
                                 bx_partition_chooser chooser, void *user, bx_plan **out) {
    BX_GUARD_BEGIN
    if (!chooser) return set_error(BX_E_INVALID, "chooser is NULL");
    ChooserCtx ctx{chooser, user};
    bx::set_error(BX_OK, "");
    return plan_with(probs, n_probs, opt, call_chooser, &ctx, out);
    BX_GUARD_END
}

bx_status bx_plan_partition_stats(const bx_plan *plan, int64_t *decisions, int64_t *non_greedy) {
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    if (decisions) *decisions = plan->p.n_decisions;
    if (non_greedy) *non_greedy = plan->p.n_nongreedy;
    return BX_OK;
}

bx_status bx_plan_num_decisions(const bx_plan *plan, int32_t *n_decisions, int64_t *n_candidates) {
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    if (n_decisions) *n_decisions = (int32_t)plan->p.decisions.size();
    if (n_candidates) *n_candidates = plan->p.n_candidates;
    return BX_OK;
}

bx_status bx_plan_decision_info(const bx_plan *plan, int32_t d, int32_t *prob, int32_t *var, int32_t *n_fns,
                                int32_t *fn_ids, int32_t *n_cands, int32_t *choice) {
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    if (d < 0 || d >= (int32_t)plan->p.decisions.size()) return set_error(BX_E_INVALID, "decision out of range");
    const bx::Decision &D = plan->p.decisions[d];
    if (prob) *prob = D.inst;
    if (var) *var = D.var;
    if (n_fns) *n_fns = (int32_t)D.B.size();
    if (fn_ids) {
        if (D.B.size() > 256) return set_error(BX_E_UNSUPPORTED, "more than 256 functions in the bucket");
        for (size_t i = 0; i < D.B.size(); ++i) fn_ids[i] = D.B[i];
    }
    if (n_cands) *n_cands = (int32_t)D.cands.size();
    if (choice) *choice = D.choice;
    return BX_OK;
}

bx_status bx_plan_candidate_parts(const bx_plan *plan, int32_t d, int32_t c, int32_t *part_of_fn) {
    if (!plan || !part_of_fn) return set_error(BX_E_INVALID, "NULL argument");
    if (d < 0 || d >= (int32_t)plan->p.decisions.size()) return set_error(BX_E_INVALID, "decision out of range");
    const bx::Decision &D = plan->p.decisions[d];
    if (c < 0 || c >= (int32_t)D.cands.size()) return set_error(BX_E_INVALID, "candidate out of range");
    for (size_t k = 0; k < D.cands[c].parts.size(); ++k)
        for (int32_t id : D.cands[c].parts[k])
            part_of_fn[std::find(D.B.begin(), D.B.end(), id) - D.B.begin()] = (int32_t)k;
    return BX_OK;
}

bx_status bx_plan_candidate_scratch_bytes(const bx_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return set_error(BX_E_INVALID, "NULL argument");
    BX_GUARD_BEGIN
    *bytes = bx::cand_scratch_bytes(plan->p);
    return BX_OK;
    BX_GUARD_END
}

bx_status bx_plan_candidate_values(bx_plan *plan, const void *d_workspace, size_t bytes, int32_t samples,
                                   const uint32_t *d_rnd, double *d_out, void *d_scratch, size_t scratch_bytes,
                                   void *stream) {
    if (!plan) return set_error(BX_E_INVALID, "plan is NULL");
    BX_GUARD_BEGIN
    if (!plan->p.executed) return set_error(BX_E_STATE, "candidate values need an executed plan");
    return bx::dev_candidate_values(plan->p, d_workspace, bytes, samples, d_rnd, d_out, d_scratch, scratch_bytes,
                                    stream);
    BX_GUARD_END
}

int64_t bx_mlp_num_params(int32_t n_in, int32_t hidden) {
    if (n_in < 1 || hidden < 1) return -1;
    return bx::mlp_num_params(n_in, hidden);
}

bx_status bx_mlp_forward(const bx_mlp *m, const float *d_x, float *d_act, float *d_y, int32_t batch,
                         void *stream) {
    BX_GUARD_BEGIN
    return bx::mlp_forward(m, d_x, d_act, d_y, batch, stream);
    BX_GUARD_END
}

bx_status bx_mlp_backward(const bx_mlp *m, const float *d_x, const float *d_act, const float *d_dy,
                          float *d_grads, float *d_work, int32_t batch, void *stream) {
    BX_GUARD_BEGIN
    return bx::mlp_backward(m, d_x, d_act, d_dy, d_grads, d_work, batch, stream);
    BX_GUARD_END
}

bx_status bx_mlp_backward_noalloc(const bx_mlp *m, const float *d_x, const float *d_act, const float *d_dy,
                                  float *d_grads, int32_t batch, void *stream) {
    BX_GUARD_BEGIN
    return bx::mlp_backward_noalloc(m, d_x, d_act, d_dy, d_grads, batch, stream);
    BX_GUARD_END
}

bx_status bx_mlp_adam_step(const bx_mlp *m, const float *d_grads, float *d_m, float *d_v, float lr,
                           float beta1, float beta2, float eps, int32_t step, void *stream) {
    BX_GUARD_BEGIN
    return bx::mlp_adam(m, d_grads, d_m, d_v, lr, beta1, beta2, eps, step, stream);
    BX_GUARD_END
}

bx_status bx_mlp_pack_bf16(const bx_mlp *m, void *stream) {
    BX_GUARD_BEGIN
    return bx::mlp_pack_bf16(m, stream);
    BX_GUARD_END
}

bx_status bx_mlp_mse(const float *d_y, const float *d_target, float *d_dy, float *d_loss, int32_t batch,
                     void *stream) {
    BX_GUARD_BEGIN
    return bx::mlp_mse(d_y, d_target, d_dy, d_loss, batch, stream);
    BX_GUARD_END
}

bx_status bx_mlp_infer_bf16(const bx_mlp *m, const float *d_x, float *d_y, int32_t batch, void *stream) {
    BX_GUARD_BEGIN
    return bx::mlp_infer_bf16(m, d_x, d_y, batch, stream);
    BX_GUARD_END
}

bx_status bx_plan_create_learned(bx_problem *const *probs, int32_t n_probs, const bx_options *opt,
                                 const bx_mlp *model, void *d_buf, size_t buf_bytes, float margin,
                                 void *stream, bx_plan **out) {
    BX_GUARD_BEGIN
    if (!model || !model->d_params_bf16) return set_error(BX_E_INVALID, "model or its bf16 weights are NULL");
    if (model->n_in != bx::kPartFeatures)
        return set_error(BX_E_INVALID, "the model's input width differs from bx_partition_num_features()");
    if (!d_buf) return set_error(BX_E_INVALID, "device buffer is NULL");
    bx::LearnedCtx ctx{model, d_buf, buf_bytes, margin, stream};
    return plan_with(probs, n_probs, opt, bx::mlp_choose, &ctx, out);
    BX_GUARD_END
}

const char *bx_last_error(void) { return bx::last_error_cstr(); }

const char *bx_version(void) { return "bx 0.1 (gfx950)"; }

}  // extern "C"
