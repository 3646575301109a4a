// Depth-first branch and bound over a WCSP with the mini-bucket bound as its
// heuristic, recomputed at every node: the use of MBE the paper's
// conclusion (Sec. 10) proposes, where the cost of recomputing the bound at
// each search node is what a GPU can cut.  Every expansion conditions the
// problem on each value of the next variable and bounds all those children
// in ONE batched device pass (one plan with one problem per child, the level
// schedule of the UTIL phase over all of them).
//
// Search: variables are assigned root first along the elimination order the
// plan uses (order[0], order[1], ...).  A child's lower bound is the MBE
// bound of the conditioned problem (its fully assigned functions become
// constants); the value phase of the same pass gives a complete assignment
// whose cost (the child's upper bound) may improve the incumbent.  Children
// are explored in increasing bound; a node is pruned when its bound reaches
// the incumbent, and not expanded when its bound equals its own upper bound
// (the bound is then exact for that subtree).  The optimum is proved when
// the stack empties.  Integer costs only.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "bx_internal.h"

namespace bx {

namespace {

// The problem with val[v] >= 0 assigned: every function restricted to those
// values, over its unassigned variables in their original scope order (a
// function with no unassigned variable left becomes a constant).  The
// variables stay, unconstrained once assigned.
Problem condition(const Problem &p, const std::vector<int32_t> &val) {
    Problem q;
    q.n = p.n;
    q.dom = p.dom;
    q.ct = p.ct;
    q.order = p.order;
    for (const Function &f : p.fns) {
        Function g;
        for (int32_t v : f.scope)
            if (val[v] < 0) g.scope.push_back(v);
        int64_t size = 1;
        for (int32_t v : g.scope) size *= p.dom[v];
        g.ti.resize((size_t)size);
        std::vector<int32_t> dig(g.scope.size(), 0);   // odometer over g.scope, last fastest
        for (int64_t r = 0; r < size; ++r) {
            int64_t src = 0;
            size_t k = 0;
            for (int32_t v : f.scope) src = src * p.dom[v] + (val[v] >= 0 ? val[v] : dig[k++]);
            g.ti[(size_t)r] = f.ti[(size_t)src];
            for (int j = (int)dig.size() - 1; j >= 0; --j) {
                if (++dig[j] < p.dom[g.scope[j]]) break;
                dig[j] = 0;
            }
        }
        q.fns.push_back(std::move(g));
    }
    return q;
}

struct Node {
    std::vector<int32_t> val;   // -1: unassigned
    int32_t depth;              // variables order[0..depth) are assigned
    double lb;
};

}  // namespace

bx_status bnb_solve(const Problem &p0, const bx_options &opt, void *ws, size_t bytes, void *stream,
                    int64_t max_nodes, double *value, int32_t *assignment, int64_t *stats) {
    if (p0.ct != BX_COST_I32) return set_error(BX_E_UNSUPPORTED, "branch and bound takes integer costs");
    if (opt.algo != BX_ALGO_MBE && opt.algo != BX_ALGO_BE)
        return set_error(BX_E_INVALID, "branch and bound bounds with BE or MBE");
    bx_status s = validate_problem(p0);
    if (s != BX_OK) return s;
    Problem p = p0;
    if (p.order.empty()) {
        std::vector<int32_t> parent;
        s = compute_order(p, opt.order, p.order, parent);
        if (s != BX_OK) return s;
    }
    const int n = p.n;
    int64_t nodes = 0, passes = 0, pruned = 0;

    // bounds of a batch of conditioned problems, in as few device passes as
    // the workspace allows
    auto bound_batch = [&](const std::vector<std::vector<int32_t>> &vals, std::vector<double> &lb,
                           std::vector<double> &ub, std::vector<std::vector<int32_t>> &sig) -> bx_status {
        const size_t m = vals.size();
        lb.assign(m, 0.0);
        ub.assign(m, 0.0);
        sig.assign(m, std::vector<int32_t>(n > 0 ? n : 1, 0));
        std::vector<Problem> probs;
        probs.reserve(m);
        for (const auto &v : vals) probs.push_back(condition(p, v));
        size_t i0 = 0;
        while (i0 < m) {
            size_t cnt = m - i0;
            for (;;) {   // the largest run of children whose plan fits the workspace
                std::vector<const Problem *> ps;
                for (size_t i = i0; i < i0 + cnt; ++i) ps.push_back(&probs[i]);
                Plan plan;
                bx_status st = build_plan(ps, opt, plan);
                if (st != BX_OK) return st;
                if (plan.total_bytes > bytes) {
                    if (cnt == 1) return set_error(BX_E_NOMEM, "a conditioned problem needs a larger workspace");
                    cnt = (cnt + 1) / 2;
                    continue;
                }
                st = dev_upload(plan, ws, bytes, stream);
                if (st == BX_OK) st = dev_execute(plan, ws, bytes, BX_SCHED_LEVEL, stream);
                if (st != BX_OK) return st;
                ++passes;
                for (size_t i = 0; i < cnt; ++i) {
                    st = dev_results(plan, ws, (int32_t)i, &lb[i0 + i], &ub[i0 + i], sig[i0 + i].data(), stream);
                    if (st != BX_OK) return st;
                }
                dev_release(plan);
                break;
            }
            i0 += cnt;
        }
        return BX_OK;
    };

    // the root: its MBE bound and assignment start the search
    std::vector<double> lb, ub;
    std::vector<std::vector<int32_t>> sig;
    s = bound_batch({std::vector<int32_t>(n, -1)}, lb, ub, sig);
    if (s != BX_OK) return s;
    double best = ub[0];
    std::vector<int32_t> best_sig = sig[0];
    std::vector<Node> stack;
    if (lb[0] < best) stack.push_back(Node{std::vector<int32_t>(n, -1), 0, lb[0]});
    bool proved = true;
    while (!stack.empty()) {
        Node nd = std::move(stack.back());
        stack.pop_back();
        if (nd.lb >= best) { ++pruned; continue; }
        if (max_nodes > 0 && nodes >= max_nodes) { proved = false; break; }
        ++nodes;
        const int32_t v = p.order[nd.depth];
        std::vector<std::vector<int32_t>> kids(p.dom[v], nd.val);
        for (int32_t x = 0; x < p.dom[v]; ++x) kids[x][v] = x;
        s = bound_batch(kids, lb, ub, sig);
        if (s != BX_OK) return s;
        std::vector<int32_t> idx;
        for (int32_t x = 0; x < p.dom[v]; ++x) {
            if (ub[x] < best) {   // the child's complete assignment: prefix + its value phase
                best = ub[x];
                best_sig = sig[x];
                for (int u = 0; u < n; ++u)
                    if (kids[x][u] >= 0) best_sig[u] = kids[x][u];
            }
            idx.push_back(x);
        }
        // deepest-first with the smallest bound on top of the stack
        std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return lb[a] > lb[b]; });
        for (int32_t x : idx) {
            if (lb[x] >= best) { ++pruned; continue; }
            if (lb[x] >= ub[x] || nd.depth + 1 >= n) continue;   // exact below this child
            stack.push_back(Node{kids[x], nd.depth + 1, lb[x]});
        }
    }
    if (value) *value = best;
    if (assignment)
        for (int u = 0; u < n; ++u) assignment[u] = best_sig[u];
    if (stats) {
        stats[0] = nodes;
        stats[1] = passes;
        stats[2] = pruned;
        stats[3] = proved ? 1 : 0;
    }
    return BX_OK;
}

}  // namespace bx
