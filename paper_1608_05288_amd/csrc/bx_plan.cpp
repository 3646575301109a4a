// Host planner of the UTIL-table engine.
//
// Turns problems <X, D, C> (Sec. 2) into a device plan: elimination order or
// pseudo-tree (Sec. 2 Def. 1-2, Sec. 6.2), normalised bucket-tables (scope
// sorted by order position so the eliminated variable is last, Sec. 6.1 and
// the remark closing Sec. 6.4), buckets (Alg. 1), mini-bucket
// partitions under an i-bound (Alg. 2), stride descriptors (the
// mul/div/mod data of Eq. (3), Sec. 6.3), dependency levels, tiles, the
// value-assignment schedule and the workspace layout.
#include <algorithm>
#include <set>
#include <tuple>
#include <cmath>
#include <cstring>
#include <numeric>

#include "bx_internal.h"

namespace bx {

namespace {

// ---------------------------------------------------------------- graph
// Adjacency as bit rows: row v has bit u set when v and u share a function.
struct BitGraph {
    int n = 0;
    int words = 0;
    std::vector<uint64_t> bits;
    explicit BitGraph(int n_) : n(n_), words((n_ + 63) / 64), bits((size_t)n_ * words, 0) {}
    uint64_t *row(int v) { return bits.data() + (size_t)v * words; }
    const uint64_t *row(int v) const { return bits.data() + (size_t)v * words; }
    bool has(int v, int u) const { return (row(v)[u >> 6] >> (u & 63)) & 1u; }
    void set(int v, int u) { row(v)[u >> 6] |= (uint64_t)1 << (u & 63); }
    void link(int a, int b) { if (a != b) { set(a, b); set(b, a); } }
};

BitGraph primal(const Problem &p) {
    BitGraph g(p.n);
    for (const Function &f : p.fns)
        for (size_t a = 0; a < f.scope.size(); ++a)
            for (size_t b = a + 1; b < f.scope.size(); ++b) g.link(f.scope[a], f.scope[b]);
    return g;
}

int popcount_and(const uint64_t *a, const uint64_t *b, int words) {
    int c = 0;
    for (int w = 0; w < words; ++w) c += __builtin_popcountll(a[w] & b[w]);
    return c;
}

// Greedy min-degree / min-fill: the chosen vertex is eliminated next, so it
// takes the highest free position of the order.
void greedy_order(BitGraph g, bool fill, std::vector<int32_t> &order) {
    const int n = g.n, W = g.words;
    std::vector<uint64_t> alive(W, 0);
    for (int v = 0; v < n; ++v) alive[v >> 6] |= (uint64_t)1 << (v & 63);
    std::vector<uint64_t> nb(W), tmp(W);
    std::vector<int> deg(n, 0);
    std::vector<int64_t> fil(n, 0);
    // degree and fill (pairs of live neighbours that are not yet adjacent) of v
    auto score = [&](int v) {
        const uint64_t *rv = g.row(v);
        deg[v] = popcount_and(rv, alive.data(), W);
        int64_t f = 0;
        if (fill && deg[v] > 1) {
            for (int w = 0; w < W; ++w) tmp[w] = rv[w] & alive[w];
            for (int w = 0; w < W; ++w) {
                uint64_t m = tmp[w];
                while (m) {
                    const int a = w * 64 + __builtin_ctzll(m);
                    m &= m - 1;
                    const uint64_t *ra = g.row(a);
                    int missing = 0;
                    for (int q = 0; q < W; ++q) missing += __builtin_popcountll(tmp[q] & ~ra[q]);
                    f += missing - 1;   // a itself is not adjacent to a
                }
            }
            f /= 2;
        }
        fil[v] = f;
    };
    // live vertices by (fill, degree, id) -- the smallest is eliminated next,
    // ties to the lowest id (min-degree: fill kept at 0)
    using Key = std::tuple<int64_t, int, int>;
    auto key = [&](int v) { return Key(fill ? fil[v] : 0, deg[v], v); };
    std::set<Key> q;
    for (int v = 0; v < n; ++v) {
        score(v);
        q.insert(key(v));
    }
    order.assign(n, 0);
    std::vector<int> N;
    for (int p = n - 1; p >= 0; --p) {
        const int best = std::get<2>(*q.begin());
        q.erase(q.begin());
        order[p] = best;
        const uint64_t *rb = g.row(best);
        N.clear();
        for (int w = 0; w < W; ++w) {
            nb[w] = rb[w] & alive[w];
            uint64_t m = nb[w];
            while (m) {
                N.push_back(w * 64 + __builtin_ctzll(m));
                m &= m - 1;
            }
        }
        // Only the neighbours' scores change, except that a fill edge (a, c)
        // between two of them makes the pair adjacent for every live common
        // neighbour u outside them: fill(u) drops by one.  (u's degree and
        // neighbourhood are unchanged: u is not adjacent to `best`.)
        if (fill) {
            for (size_t i = 0; i < N.size(); ++i)
                for (size_t j = i + 1; j < N.size(); ++j) {
                    const int a = N[i], c = N[j];
                    if (g.has(a, c)) continue;
                    const uint64_t *ra = g.row(a), *rc = g.row(c);
                    for (int w = 0; w < W; ++w) tmp[w] = ra[w] & rc[w] & alive[w] & ~nb[w];
                    tmp[best >> 6] &= ~((uint64_t)1 << (best & 63));
                    for (int w = 0; w < W; ++w) {
                        uint64_t m = tmp[w];
                        while (m) {
                            const int u = w * 64 + __builtin_ctzll(m);
                            m &= m - 1;
                            q.erase(key(u));
                            --fil[u];
                            q.insert(key(u));
                        }
                    }
                }
        }
        // connect the live neighbours of `best` pairwise, then remove it
        for (int a : N) {
            uint64_t *ra = g.row(a);
            for (int w = 0; w < W; ++w) ra[w] |= nb[w];
            ra[a >> 6] &= ~((uint64_t)1 << (a & 63));
        }
        alive[best >> 6] &= ~((uint64_t)1 << (best & 63));
        for (int a : N) {
            q.erase(key(a));
            score(a);
            q.insert(key(a));
        }
    }
}

std::vector<int> static_degrees(const BitGraph &g) {
    std::vector<int> d(g.n, 0);
    for (int v = 0; v < g.n; ++v)
        for (int w = 0; w < g.words; ++w) d[v] += __builtin_popcountll(g.row(v)[w]);
    return d;
}

// DFS pseudo-tree: roots are the highest-degree unvisited vertices, the walk
// enters unvisited neighbours by decreasing degree; ties to the lowest id.
void dfs_tree(const BitGraph &g, std::vector<int32_t> &order, std::vector<int32_t> &parent) {
    const int n = g.n;
    std::vector<int> deg = static_degrees(g);
    std::vector<char> seen(n, 0);
    order.clear();
    parent.assign(n, -1);
    std::vector<int> stack;
    while ((int)order.size() < n) {
        int root = -1;
        for (int v = 0; v < n; ++v)
            if (!seen[v] && (root < 0 || deg[v] > deg[root])) root = v;
        seen[root] = 1;
        order.push_back(root);
        stack.assign(1, root);
        while (!stack.empty()) {
            int v = stack.back();
            int next = -1;
            for (int u = 0; u < n; ++u)
                if (!seen[u] && g.has(v, u) && (next < 0 || deg[u] > deg[next])) next = u;
            if (next < 0) { stack.pop_back(); continue; }
            seen[next] = 1;
            parent[next] = v;
            order.push_back(next);
            stack.push_back(next);
        }
    }
}

// Pre-order of a given forest: roots and children by increasing id.
std::vector<int32_t> preorder(const std::vector<int32_t> &parent) {
    const int n = (int)parent.size();
    std::vector<std::vector<int32_t>> kids(n);
    std::vector<int32_t> roots, out;
    for (int v = 0; v < n; ++v) {
        if (parent[v] < 0) roots.push_back(v); else kids[parent[v]].push_back(v);
    }
    std::vector<int32_t> stack;
    for (int r : roots) {
        stack.push_back(r);
        while (!stack.empty()) {
            int v = stack.back();
            stack.pop_back();
            out.push_back(v);
            for (auto it = kids[v].rbegin(); it != kids[v].rend(); ++it) stack.push_back(*it);
        }
    }
    return out;
}

bx_status check_pseudotree(const Problem &p, const std::vector<int32_t> &parent) {
    const int n = p.n;
    if ((int)parent.size() != n) return set_error(BX_E_INVALID, "pseudo-tree: wrong length");
    for (int v = 0; v < n; ++v)
        if (parent[v] < -1 || parent[v] >= n || parent[v] == v)
            return set_error(BX_E_INVALID, "pseudo-tree: parent out of range");
    // depth by walking up; a walk longer than n means a cycle
    std::vector<int> depth(n, -1);
    for (int v = 0; v < n; ++v) {
        int d = 0, a = v;
        while (parent[a] >= 0) {
            a = parent[a];
            if (++d > n) return set_error(BX_E_INVALID, "pseudo-tree: cycle");
        }
        depth[v] = d;
    }
    auto is_ancestor = [&](int a, int v) {
        for (int u = parent[v]; u >= 0; u = parent[u]) if (u == a) return true;
        return false;
    };
    for (const Function &f : p.fns)
        for (size_t i = 0; i < f.scope.size(); ++i)
            for (size_t j = i + 1; j < f.scope.size(); ++j) {
                int a = f.scope[i], b = f.scope[j];
                if (!is_ancestor(a, b) && !is_ancestor(b, a))
                    return set_error(BX_E_INVALID,
                                     "pseudo-tree: variables " + std::to_string(a) + " and " +
                                         std::to_string(b) + " share a function but lie on different branches");
            }
    return BX_OK;
}

// separator of every variable (Sec. 4): ancestors linked to it or to one of
// its descendants
std::vector<std::vector<char>> separators(const Problem &p, const std::vector<int32_t> &parent) {
    const int n = p.n;
    BitGraph g = primal(p);
    std::vector<std::vector<char>> sep(n, std::vector<char>(n, 0));
    for (int d = 0; d < n; ++d) {
        // d contributes its ancestor-neighbours to the separator of every
        // node on its path to the root (itself included) that lies below them
        std::vector<int> path;
        for (int a = d; a >= 0; a = parent[a]) path.push_back(a);
        for (size_t i = 0; i < path.size(); ++i) {
            int node = path[i];
            for (size_t j = i + 1; j < path.size(); ++j)
                if (g.has(d, path[j])) sep[node][path[j]] = 1;
        }
    }
    return sep;
}

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

// ------------------------------------------------------------- validation
bx_status validate_problem(const Problem &p) {
    for (size_t fi = 0; fi < p.fns.size(); ++fi) {
        for (int32_t v : p.fns[fi].scope)
            if (v < 0 || v >= p.n) return set_error(BX_E_INVALID, "scope variable out of range");
    }
    if (!p.order.empty()) {
        std::vector<char> seen(p.n, 0);
        if ((int)p.order.size() != p.n) return set_error(BX_E_INVALID, "order: wrong length");
        for (int32_t v : p.order) {
            if (v < 0 || v >= p.n || seen[v]) return set_error(BX_E_INVALID, "order is not a permutation");
            seen[v] = 1;
        }
    }
    return BX_OK;
}

bx_status compute_order(const Problem &p, bx_order_heuristic h, std::vector<int32_t> &order,
                        std::vector<int32_t> &parent) {
    BitGraph g = primal(p);
    parent.assign(p.n, -1);
    switch (h) {
    case BX_ORDER_MIN_DEGREE: greedy_order(g, false, order); break;
    case BX_ORDER_MIN_FILL: greedy_order(g, true, order); break;
    case BX_ORDER_DFS: dfs_tree(g, order, parent); break;
    case BX_ORDER_DEGREE_SORT: {
        std::vector<int> deg = static_degrees(g);
        order.resize(p.n);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return deg[a] < deg[b]; });
        break;
    }
    default: return set_error(BX_E_INVALID, "unknown order heuristic");
    }
    return BX_OK;
}

int32_t induced_width(const Problem &p, const std::vector<int32_t> &order) {
    BitGraph g = primal(p);
    const int n = p.n;
    std::vector<int> pos(n);
    for (int i = 0; i < n; ++i) pos[order[i]] = i;
    int w = 0;
    for (int i = n - 1; i >= 0; --i) {
        int v = order[i];
        std::vector<int> earlier;
        for (int u = 0; u < n; ++u) if (g.has(v, u) && pos[u] < i) earlier.push_back(u);
        w = std::max<int>(w, (int)earlier.size());
        for (int a : earlier) for (int b : earlier) g.link(a, b);
    }
    return w;
}

// ---------------------------------------------------------------- planning
namespace {

int64_t table_entries(const std::vector<int32_t> &scope, const std::vector<int32_t> &dom) {
    int64_t s = 1;
    for (int32_t v : scope) s *= dom[v];
    return s;
}

// Greedy scope-based partition (the partition step of Alg. 2): functions in (decreasing
// arity, increasing id) order, each into the first mini-bucket whose scope
// stays within `ibound` variables, else into a new one.
std::vector<std::vector<int32_t>> greedy_partition(const PInst &I, const std::vector<int32_t> &B,
                                                   int ibound) {
    std::vector<int32_t> ids = B;
    std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
        size_t sa = I.fns[a].scope.size(), sb = I.fns[b].scope.size();
        if (sa != sb) return sa > sb;
        return a < b;
    });
    std::vector<std::vector<int32_t>> parts;
    std::vector<std::vector<char>> in;   // variable membership per part
    for (int32_t id : ids) {
        const auto &sc = I.fns[id].scope;
        size_t k = 0;
        for (; k < parts.size(); ++k) {
            int extra = 0, size = 0;
            for (char c : in[k]) size += c;
            for (int32_t v : sc) extra += !in[k][v];
            if (size + extra <= ibound) break;
        }
        if (k == parts.size()) {
            parts.emplace_back();
            in.emplace_back(I.n, 0);
        }
        parts[k].push_back(id);
        for (int32_t v : sc) in[k][v] = 1;
    }
    return parts;
}

std::vector<int32_t> union_sorted(const PInst &I, const std::vector<int32_t> &ids) {
    std::vector<char> in(I.n, 0);
    std::vector<int32_t> u;
    for (int32_t id : ids)
        for (int32_t v : I.fns[id].scope)
            if (!in[v]) { in[v] = 1; u.push_back(v); }
    std::sort(u.begin(), u.end(), [&](int a, int b) { return I.pos[a] < I.pos[b]; });
    return u;
}

// Register blocking of a tiled-path mini-bucket.  The plain row loop loads
// every lane function once per row.  A thread that computes a box of rows
// over all values of outer variables a and b instead loads a lane function
// once per value combination of the box variables it depends on:
//     loads per row = sum_f (da if f has a) (db if f has b) / (da db).
// Among b with 2 <= db <= kBlockMaxDb1 (kBlockMaxDb beside an a), and a
// absent or with 2 <= da <= kBlockMaxDa (and D <= kBlockMaxD2), such that at most one lane function depends on neither, at
// most one on b only, at most one on a only and none on both (the shape the
// blocked loop handles), the pair with the fewest loads is taken when it
// saves at least a quarter of the plain loop's; the fastest variables win
// ties.  The
// outer variables are then visited with a and b last (dims and every
// function's strides permuted alike, ostr = the output stride of each), and
// the lane functions grouped by which box variables they depend on.
void choose_blocking(DevMb &d, std::vector<DevFn> &lane, std::vector<DevFn> &uni) {
    const int nvo = d.nv - d.n_inner;
    const int nfl = (int)lane.size();
    if (d.path != 0 || d.D > kBlockMaxD || nfl < 1 || nfl > kBlockRowCol || nvo < 1 ||
        d.n_inner > kBlockMaxInner)
        return;
    double best = 0.75 * nfl;
    int ba = -1, bb = -1;
    for (int b = nvo - 1; b >= 0; --b) {
        const int db = d.dims[b];
        if (db < 2 || db > kBlockMaxDb1) continue;
        for (int k = 0; k <= nvo; ++k) {   // a: absent, then the fastest first
            const int a = k == 0 ? -1 : nvo - k;
            if (a == b) continue;
            const int da = a < 0 ? 1 : d.dims[a];
            if (a >= 0 && (da < 2 || da > kBlockMaxDa || db > kBlockMaxDb || d.D > kBlockMaxD2)) continue;
            // the blocked loop takes at most one function depending on
            // neither box variable, one on b only, one on a only, none on both
            int cls[4] = {0, 0, 0, 0};
            double c = 0;
            for (const DevFn &f : lane) {
                const bool fa = a >= 0 && f.stride[a], fb = f.stride[b] != 0;
                ++cls[(fa ? 2 : 0) + (fb ? 1 : 0)];
                c += (double)(fa ? da : 1) * (fb ? db : 1);
            }
            if (cls[0] > 1 || cls[1] > 1 || cls[2] > 1 || cls[3] > 0) continue;
            c /= (double)(da * db);
            if (c < best - 1e-9) {
                best = c;
                ba = a;
                bb = b;
            }
        }
    }
    if (bb < 0) return;
    // visiting order of the outer variables: the others in output order, then a, then b
    std::vector<int> perm;
    for (int j = 0; j < nvo; ++j)
        if (j != ba && j != bb) perm.push_back(j);
    if (ba >= 0) perm.push_back(ba);
    perm.push_back(bb);
    std::vector<int32_t> nat(nvo);
    int64_t s = 1;
    for (int j = nvo - 1; j >= 0; --j) { nat[j] = (int32_t)s; s *= d.dims[j]; }
    // lane groups: neither box variable, b only, a only, both
    std::vector<DevFn> grp[4];
    for (const DevFn &f : lane) grp[(ba >= 0 && f.stride[ba] ? 2 : 0) + (f.stride[bb] ? 1 : 0)].push_back(f);
    lane.clear();
    for (int k = 0; k < 4; ++k) lane.insert(lane.end(), grp[k].begin(), grp[k].end());
    d.g0 = (int32_t)grp[0].size();
    d.ga = d.g0 + (int32_t)grp[1].size();
    d.gb = d.ga + (int32_t)grp[2].size();
    auto permute = [&](int32_t *v) {
        std::vector<int32_t> old(v, v + nvo);
        for (int k = 0; k < nvo; ++k) v[k] = old[perm[k]];
    };
    for (DevFn &f : lane) permute(f.stride);
    for (DevFn &f : uni) permute(f.stride);
    for (int k = 0; k < nvo; ++k) d.ostr[k] = nat[perm[k]];
    d.da = ba >= 0 ? d.dims[ba] : 1;
    d.db = d.dims[bb];
    permute(d.dims);
    d.blk = 1;
}

}  // namespace

// Launch levels and groups of packed mini-buckets.  Mini-buckets are visited
// in creation order, which puts every producer before its consumer.  A
// packed mini-bucket opens a group and takes in the groups of its packed
// children, smallest first, while the group stays within the fusion limits
// (rows, rows per stage, stages); its stage is one after the deepest child
// group taken in.  A
// group is launched one level after the latest producer outside it (level 0
// when it has none); any other mini-bucket one level after its latest
// producer.  A group is one connected part of the bucket tree, computed by
// one workgroup stage by stage, so its inner hand-offs need no launch.
void schedule_levels(Plan &P) {
    const size_t n = P.mbs.size();
    std::vector<std::vector<int32_t>> kids(n), members(n);
    for (size_t g = 0; g < n; ++g) {
        const PInst &I = P.inst[P.mbs[g].inst];
        for (int32_t id : P.mbs[g].members)
            if (I.fns[id].src_mb >= 0) kids[g].push_back(I.fns[id].src_mb);
    }
    std::vector<int32_t> gid(n, -1), stage(n, 0), level(n, 0);
    std::vector<int64_t> grows(n, 0);
    std::vector<std::vector<int64_t>> srows(n);   // rows per stage of a group
    auto level_of = [&](int32_t c) { return gid[c] >= 0 ? level[gid[c]] : level[c]; };
    P.n_groups = P.n_packed = 0;
    for (size_t gi = 0; gi < n; ++gi) {
        const int32_t g = (int32_t)gi;
        if (P.dmb[g].path != 3) {
            int l = 0;
            for (int32_t c : kids[g]) l = std::max(l, level_of(c) + 1);
            level[g] = l;
            continue;
        }
        gid[g] = g;
        grows[g] = P.mbs[g].out_rows;
        members[g].assign(1, g);
        std::vector<int32_t> open;
        for (int32_t c : kids[g])
            if (gid[c] == c) open.push_back(c);   // a packed child heads its own group
        std::stable_sort(open.begin(), open.end(), [&](int32_t a, int32_t b) { return grows[a] < grows[b]; });
        std::vector<int64_t> below;               // rows per stage of the children taken in
        for (int32_t c : open) {
            // the group after taking c in: stages of c's group merge with the
            // others', g one stage after the deepest
            std::vector<int64_t> m = below;
            if (m.size() < srows[c].size()) m.resize(srows[c].size(), 0);
            for (size_t k = 0; k < srows[c].size(); ++k) m[k] += srows[c][k];
            bool ok = grows[g] + grows[c] <= P.fuse_max_rows && (int)m.size() + 1 <= P.fuse_max_stages &&
                      members[g].size() + members[c].size() <= (size_t)kPackMaxSegs;
            for (int64_t r : m) ok = ok && r <= P.fuse_max_stage_rows;
            if (!ok) continue;
            below = m;
            grows[g] += grows[c];
            for (int32_t x : members[c]) gid[x] = g;
            members[g].insert(members[g].end(), members[c].begin(), members[c].end());
            members[c].clear();
            srows[c].clear();
        }
        // stages of the members taken in keep their depth from the leaves of
        // their own groups; g comes after all of them
        stage[g] = (int32_t)below.size();
        below.push_back(P.mbs[g].out_rows);
        srows[g] = below;
        int l = 0;
        for (int32_t m : members[g])
            for (int32_t c : kids[m])
                if (gid[c] != g) l = std::max(l, level_of(c) + 1);
        level[g] = l;
    }
    int32_t max_level = -1;
    for (size_t g = 0; g < n; ++g) {
        PMb &mb = P.mbs[g];
        mb.group = gid[g];
        mb.stage = stage[g];
        mb.level = level_of((int32_t)g);
        P.dmb[g].level = mb.level;
        max_level = std::max(max_level, mb.level);
        if (gid[g] >= 0) ++P.n_packed;
        if (gid[g] == (int32_t)g) ++P.n_groups;
    }
    P.n_levels = max_level + 1;
}

// Packing on or off (when the options allow it): code paths, launch levels
// and tiles are planned again; the per-level tuning starts from the defaults.
bx_status set_packing(Plan &P, bool on) {
    P.pack_on = on && P.pack_allowed;
    bx_status s = fill_descriptors(P);
    if (s != BX_OK) return s;
    schedule_levels(P);
    P.level_goal.assign(P.n_levels, P.rows_per_tile > 0 ? P.rows_per_tile : kDefaultTilesGoal);
    P.level_stage.assign(P.n_levels, 1);
    P.level_nt.assign(P.n_levels, 0);
    P.level_xcd.assign(P.n_levels, 0);
    retile_levels(P);
    return BX_OK;
}

// Mini-bucket and function descriptors: inner/outer split, lane / outer-only
// function order, strides, code path.  Table offsets are taken as they stand
// in the plan (absolute once resolved).
bx_status fill_descriptors(Plan &P) {
    const size_t n_mb = P.mbs.size();
    P.dmb.assign(n_mb, DevMb{});
    P.dfn.clear();
    P.util_rows = P.joint_entries = P.algo_bytes = 0;
    P.max_scope = 0;
    for (size_t g = 0; g < n_mb; ++g) {
        const PMb &mb = P.mbs[g];
        const PInst &I = P.inst[mb.inst];
        DevMb d{};
        d.out_off = mb.out_off;
        d.nv = (int32_t)mb.U.size() - 1;
        d.D = I.dom[mb.var];
        d.out_rows = mb.out_rows;
        d.inst = mb.inst;
        d.level = mb.level;
        d.red = mb.red;
        for (int j = 0; j < d.nv; ++j) d.dims[j] = I.dom[mb.U[j]];
        d.f_begin = (int32_t)P.dfn.size();
        // inner variables: the longest run of fastest output variables whose
        // rows fit one workgroup pass
        int n_inner = 0;
        int64_t p_in = 1;
        while (n_inner < d.nv && p_in * d.dims[d.nv - 1 - n_inner] <= kUtilThreads) {
            p_in *= d.dims[d.nv - 1 - n_inner];
            ++n_inner;
        }
        d.n_inner = n_inner;
        d.p_in = (int32_t)p_in;
        d.q = (int32_t)(kUtilThreads / p_in);
        d.n_outer = d.out_rows / p_in;
        bool small_tables = mb.out_rows < kTileMaxTable;
        // functions: the ones touching an inner variable first
        std::vector<std::pair<int64_t, DevFn>> lane;   // (table size, descriptor)
        std::vector<DevFn> uni, ino, cst;   // outer-only; inner-only; eliminated variable alone
        int64_t in_bytes = 0;
        for (int32_t id : mb.members) {
            const PFn &f = I.fns[id];
            DevFn e{};
            e.src_mb = f.src_mb;
            e.tab_off = f.off;
            // stride of each scope variable inside f's table (last = 1)
            std::vector<int64_t> st(f.scope.size());
            int64_t s = 1;
            for (int j = (int)f.scope.size() - 1; j >= 0; --j) { st[j] = s; s *= I.dom[f.scope[j]]; }
            bool touches_inner = false;
            e.io_max = 0;
            for (int j = 0; j < d.nv; ++j) {
                int32_t u = mb.U[j];
                int32_t sv = 0;
                for (size_t q = 0; q < f.scope.size(); ++q) if (f.scope[q] == u) sv = (int32_t)st[q];
                e.stride[j] = sv;
                if (sv && j >= d.nv - n_inner) {
                    touches_inner = true;
                    e.io_max += (d.dims[j] - 1) * sv;
                }
            }
            // every row of the mini-bucket must address inside this table
            int64_t reach = d.D - 1;
            for (int j = 0; j < d.nv; ++j) reach += (int64_t)(d.dims[j] - 1) * e.stride[j];
            if (reach >= f.size || f.scope.back() != mb.var)
                return set_error(BX_E_INVALID, "internal: stride descriptor out of bounds");
            in_bytes += 4 * f.size;
            small_tables = small_tables && f.size < kTileMaxTable;
            bool touches_output = false, touches_outer = false;
            for (int j = 0; j < d.nv; ++j) {
                touches_output = touches_output || e.stride[j] != 0;
                if (j < d.nv - n_inner) touches_outer = touches_outer || e.stride[j] != 0;
            }
            if (touches_inner && touches_outer) lane.emplace_back(f.size, e);
            else if (touches_inner) ino.push_back(e);
            else if (touches_output) uni.push_back(e);
            else cst.push_back(e);
        }
        // smaller lane tables first: the device stages a prefix of the lane
        // functions in LDS when their rows fit
        std::stable_sort(lane.begin(), lane.end(),
                         [](const std::pair<int64_t, DevFn> &a, const std::pair<int64_t, DevFn> &b) {
                             return a.first < b.first;
                         });
        d.nfl = (int32_t)lane.size();
        d.nfi = (int32_t)ino.size();
        d.nfc = (int32_t)cst.size();
        d.nf = (int32_t)(lane.size() + uni.size() + ino.size() + cst.size());
        d.path = (d.D <= kTileMaxD && d.nfl <= kTileLaneFns && (int)uni.size() <= kTileOuterFns &&
                  d.nfi <= kTileConstFns && d.nfc <= kTileConstFns && d.nfl * d.D <= kTileMaxRun &&
                  small_tables)
                     ? 0 : 1;
        if (d.path == 1 && d.D > kTileMaxD && d.nf <= kLaneMaxFns) {
            // lane groups: the G in {8, 16, 32, 64} with the fewest idle lanes
            // over the ceil(D / G) passes, the larger G on ties
            d.path = 2;
            d.lanes = 8;
            double best = 0.0;
            for (int G = 8; G <= 64; G *= 2) {
                const double use = (double)d.D / (double)(G * ((d.D + G - 1) / G));
                if (use >= best - 1e-12) { best = use; d.lanes = G; }
            }
        }
        // small mini-buckets: packed several to a workgroup (and fused with
        // packed neighbours of the bucket tree, see schedule_levels)
        if (P.pack_on && mb.out_rows <= std::min<int64_t>(P.pack_max_rows, kPackRowLimit) && d.nf <= kPackMaxFns &&
            d.nv <= kPackMaxVars && d.D <= kPackMaxD) {
            bool fit = true;   // dims and strides fit 16 bits
            for (int j = 0; j < d.nv; ++j) fit = fit && d.dims[j] <= kPackMaxStride;
            for (const auto &e : lane)
                for (int j = 0; j < d.nv; ++j) fit = fit && e.second.stride[j] <= kPackMaxStride;
            for (const std::vector<DevFn> *v : {&uni, &ino, &cst})
                for (const DevFn &e : *v)
                    for (int j = 0; j < d.nv; ++j) fit = fit && e.stride[j] <= kPackMaxStride;
            if (fit) d.path = 3;
        }
        std::vector<DevFn> lanes;
        for (auto &e : lane) lanes.push_back(e.second);
        if (!(P.opt.flags & BX_FLAG_NO_BLOCKING)) choose_blocking(d, lanes, uni);
        for (auto &e : lanes) P.dfn.push_back(e);
        for (auto &e : uni) P.dfn.push_back(e);
        for (auto &e : ino) P.dfn.push_back(e);
        for (auto &e : cst) P.dfn.push_back(e);
        P.dmb[g] = d;
        P.util_rows += mb.out_rows;
        P.joint_entries += mb.out_rows * d.D;
        P.algo_bytes += in_bytes + 4 * mb.out_rows;
        P.mbs[g].algo_bytes = in_bytes + 4 * mb.out_rows;
        P.max_scope = std::max<int32_t>(P.max_scope, (int32_t)mb.U.size());
    }
    return BX_OK;
}

bx_status build_plan(const std::vector<const Problem *> &probs, const bx_options &opt, Plan &P,
                     Chooser chooser, void *chooser_ctx) {
    P.opt = opt;
    P.tune_cache = opt.tune_cache ? opt.tune_cache : "";
    P.opt.tune_cache = nullptr;     // the caller's string need not outlive the call
    P.pack_allowed = P.pack_on = !(opt.flags & BX_FLAG_NO_PACKING);
    P.pack_max_rows = opt.pack_max_rows > 0 ? opt.pack_max_rows : kPackMaxRows;
    P.fuse_max_rows = opt.fuse_max_rows > 0 ? opt.fuse_max_rows : kFuseMaxRows;
    P.fuse_max_stages = opt.fuse_max_stages > 0 ? opt.fuse_max_stages : kFuseMaxStages;
    P.fuse_max_stage_rows = opt.fuse_max_stage_rows > 0 ? opt.fuse_max_stage_rows : kFuseMaxStageRows;
    P.pack_stage_rows = opt.pack_stage_rows > 0 ? opt.pack_stage_rows : kPackStageRows;
    P.inst.clear();
    P.mbs.clear();
    if (probs.empty()) return set_error(BX_E_INVALID, "no problems");
    P.ct = probs[0]->ct;
    const bool bounded = opt.algo == BX_ALGO_MBE || opt.algo == BX_ALGO_ADPOP || opt.algo == BX_ALGO_MBE_SUM;
    const bool sum_mode = opt.algo == BX_ALGO_BE_SUM || opt.algo == BX_ALGO_MBE_SUM;
    if (sum_mode && probs[0]->ct != BX_COST_F32)
        return set_error(BX_E_UNSUPPORTED, "the sum-product variant needs float costs (BX_COST_F32)");
    P.sum_mode = sum_mode;
    const bool dpop = opt.algo == BX_ALGO_DPOP || opt.algo == BX_ALGO_ADPOP;
    if (bounded && opt.ibound < 1) return set_error(BX_E_INVALID, "ibound must be >= 1");
    const int64_t limit = opt.max_table_entries > 0 ? std::min<int64_t>(opt.max_table_entries, 2147483647LL)
                                                    : 2147483647LL;
    int64_t in_elems = 0;   // input tables (elements)
    int64_t msg_elems = 0;  // message tables (elements)
    std::vector<std::vector<int32_t>> input_src;   // per instance: per input fn, caller index

    for (size_t pi = 0; pi < probs.size(); ++pi) {
        const Problem &pr = *probs[pi];
        if (pr.ct != P.ct) return set_error(BX_E_INVALID, "problems of one plan must share a cost type");
        bx_status st = validate_problem(pr);
        if (st != BX_OK) return st;
        PInst I;
        I.n = pr.n;
        I.dom = pr.dom;
        // ---- order / pseudo-tree
        if (dpop) {
            if (!pr.parent.empty()) {
                I.parent = pr.parent;
                st = check_pseudotree(pr, I.parent);
                if (st != BX_OK) return st;
                I.order = preorder(I.parent);
            } else {
                st = compute_order(pr, BX_ORDER_DFS, I.order, I.parent);
                if (st != BX_OK) return st;
            }
        } else if (!pr.order.empty()) {
            I.order = pr.order;
        } else {
            st = compute_order(pr, opt.order, I.order, I.parent);
            if (st != BX_OK) return st;
        }
        I.pos.assign(I.n, 0);
        for (int i = 0; i < I.n; ++i) I.pos[I.order[i]] = i;
        I.bucket.assign(I.n, {});
        // ---- normalise the inputs (scope by position, eliminated variable last)
        I.m_inputs = (int32_t)pr.fns.size();
        int32_t ic = 0;
        double dc = 0.0;
        for (size_t fi = 0; fi < pr.fns.size(); ++fi) {
            const Function &f = pr.fns[fi];
            PFn g;
            g.id = (int32_t)fi;
            g.input_index = (int32_t)fi;
            g.scope = f.scope;
            std::sort(g.scope.begin(), g.scope.end(), [&](int a, int b) { return I.pos[a] < I.pos[b]; });
            g.size = table_entries(g.scope, I.dom);
            if (g.size > limit) return set_error(BX_E_TOO_LARGE, "input table larger than the size limit");
            if (g.scope.empty()) {
                if (P.ct == BX_COST_I32) {
                    int64_t s = (int64_t)ic + f.ti[0];
                    ic = s >= kInfI32 ? kInfI32 : (int32_t)s;
                } else {
                    dc += (double)f.tf[0];
                }
            } else {
                g.off = in_elems;
                in_elems += align_up(g.size, kAlignElems);
                I.bucket[g.scope.back()].push_back(g.id);
            }
            I.fns.push_back(std::move(g));
            // range of the finite costs (a feature for partition scoring)
            double lo = 0.0, hi = 0.0;
            bool any = false;
            for (size_t r = 0; r < (P.ct == BX_COST_I32 ? f.ti.size() : f.tf.size()); ++r) {
                const double x = P.ct == BX_COST_I32 ? (double)f.ti[r] : (double)f.tf[r];
                if (P.ct == BX_COST_I32 ? f.ti[r] >= kInfI32 : !std::isfinite(x)) continue;
                if (!any || x < lo) lo = x;
                if (!any || x > hi) hi = x;
                any = true;
            }
            I.fn_range.push_back(any ? hi - lo : 0.0);
        }
        I.host_const = P.ct == BX_COST_I32 ? (double)ic : dc;

        P.inst.push_back(std::move(I));
    }

    // ---- elimination (scopes only): positions n-1 .. 0 of every instance.
    // With a chooser, instances advance together: each runs until it meets a
    // bucket that needs a partition decision, then all pending decisions are
    // scored in one call and the instances resume.
    const size_t n_inst = P.inst.size();
    std::vector<std::vector<std::vector<char>>> seps(n_inst);
    if (opt.algo == BX_ALGO_DPOP)
        for (size_t pi = 0; pi < n_inst; ++pi) seps[pi] = separators(*probs[pi], P.inst[pi].parent);
    auto commit = [&](size_t pi, int32_t v, const std::vector<std::vector<int32_t>> &parts) -> bx_status {
        PInst &I = P.inst[pi];
        for (size_t k = 0; k < parts.size(); ++k) {
            PMb mb;
            mb.inst = (int32_t)pi;
            mb.var = v;
            mb.k = (int32_t)k;
            mb.members = parts[k];
            mb.red = sum_mode && k == 0;   // the first mini-bucket sums, the others minimise
            mb.U = union_sorted(I, parts[k]);
            std::vector<int32_t> out(mb.U.begin(), mb.U.end() - 1);
            mb.out_rows = table_entries(out, I.dom);
            if (mb.out_rows * I.dom[v] > limit)
                return set_error(BX_E_TOO_LARGE, "mini-bucket table of " + std::to_string(mb.out_rows * I.dom[v]) +
                                                     " entries exceeds the size limit");
            if ((int)out.size() > kMaxVars)
                return set_error(BX_E_TOO_LARGE, "mini-bucket scope has too many variables");
            if (opt.algo == BX_ALGO_DPOP) {
                std::vector<char> in(I.n, 0);
                for (int32_t u : out) in[u] = 1;
                if (in != seps[pi][v])
                    return set_error(BX_E_INVALID, "DPOP message scope of variable " + std::to_string(v) +
                                                       " differs from its separator");
            }
            mb.out_off = msg_elems;
            msg_elems += align_up(mb.out_rows, kAlignElems);
            int level = 0;
            for (int32_t id : mb.members) {
                int32_t src = I.fns[id].src_mb;
                if (src >= 0) level = std::max(level, P.mbs[src].level + 1);
            }
            mb.level = level;
            mb.dep_level = level;
            const int32_t gi = (int32_t)P.mbs.size();
            if (!out.empty()) {
                PFn g;
                g.id = (int32_t)I.fns.size();
                g.scope = out;
                g.size = mb.out_rows;
                g.off = -1;      // resolved below (message region)
                g.src_mb = gi;
                mb.out_id = g.id;
                I.bucket[out.back()].push_back(g.id);
                I.fns.push_back(std::move(g));
                I.fn_range.push_back(0.0);
            }
            I.mbs.push_back(gi);
            P.mbs.push_back(std::move(mb));
        }
        return BX_OK;
    };
    struct Pending {
        size_t inst;
        int32_t v;
        std::vector<int32_t> B;
        std::vector<Candidate> cands;
    };
    std::vector<int> cur(n_inst);
    for (size_t pi = 0; pi < n_inst; ++pi) cur[pi] = P.inst[pi].n - 1;
    P.n_decisions = P.n_nongreedy = P.n_candidates = 0;
    P.decisions.clear();
    for (;;) {
        std::vector<Pending> pend;
        for (size_t pi = 0; pi < n_inst; ++pi) {
            PInst &I = P.inst[pi];
            while (cur[pi] >= 0) {
                const int32_t v = I.order[cur[pi]];
                const std::vector<int32_t> B = I.bucket[v];
                if (B.empty()) {
                    // sum-product: each value of an unconstrained variable weighs 1
                    if (sum_mode) I.bound_const -= std::log((double)I.dom[v]);
                    --cur[pi];
                    continue;
                }
                bx_status st;
                if (!bounded || (int)union_sorted(I, B).size() <= opt.ibound) {
                    st = commit(pi, v, {B});
                } else if (!chooser) {
                    st = commit(pi, v, greedy_partition(I, B, opt.ibound));
                } else {
                    // the seed depends on the bucket only, so an instance gets the
                    // same candidates wherever it sits in a batch
                    uint64_t seed = 0x9e3779b97f4a7c15ull * (uint64_t)(v + 1);
                    for (int32_t id : B) seed = (seed ^ (uint64_t)id) * 0x100000001b3ull;
                    std::vector<Candidate> cands = candidate_partitions(I, B, opt.ibound, seed);
                    if (cands.size() > 1) {
                        pend.push_back(Pending{pi, v, B, std::move(cands)});
                        break;       // resumes at this bucket once decided
                    }
                    st = commit(pi, v, cands[0].parts);
                }
                if (st != BX_OK) return st;
                --cur[pi];
            }
        }
        if (pend.empty()) break;
        std::vector<int32_t> offsets(1, 0);
        for (const Pending &d : pend) offsets.push_back(offsets.back() + (int32_t)d.cands.size());
        std::vector<float> feats((size_t)offsets.back() * kPartFeatures);
        for (size_t k = 0; k < pend.size(); ++k) {
            const Pending &d = pend[k];
            float *f0 = feats.data() + (size_t)offsets[k] * kPartFeatures;
            for (size_t c = 0; c < d.cands.size(); ++c) {
                float *fc = f0 + c * kPartFeatures;
                partition_features(P.inst[d.inst], d.B, d.v, opt.ibound, d.cands[c], P.inst[d.inst].fn_range, fc);
                for (int i = 0; i < kPartBaseFeatures; ++i) fc[kPartBaseFeatures + i] = fc[i] - f0[i];
            }
        }
        std::vector<int32_t> choices(pend.size(), 0), dec_inst(pend.size());
        for (size_t k = 0; k < pend.size(); ++k) dec_inst[k] = (int32_t)pend[k].inst;
        bx_status cs = chooser(chooser_ctx, (int32_t)pend.size(), dec_inst.data(), offsets.data(), feats.data(),
                               choices.data());
        if (cs != BX_OK) return cs;
        for (size_t k = 0; k < pend.size(); ++k) {
            const Pending &d = pend[k];
            const int32_t c = choices[k];
            if (c < 0 || c >= (int32_t)d.cands.size())
                return set_error(BX_E_INVALID, "partition chooser returned an invalid candidate");
            ++P.n_decisions;
            P.n_nongreedy += c != 0;
            P.n_candidates += (int64_t)d.cands.size();
            P.decisions.push_back(Decision{(int32_t)d.inst, d.v, d.B, d.cands, c});
            bx_status st = commit(d.inst, d.v, d.cands[c].parts);
            if (st != BX_OK) return st;
            --cur[d.inst];
        }
    }

    // ------------------------------------------------------------ layout
    auto align_bytes = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t n_mb = P.mbs.size();
    size_t off = 0;
    P.off_counters = off;
    P.n_counters = 4 + n_mb;                 // next tile, error flag, sink of the descriptor
                                             //   warm-up, spare, done[mb]
    off = align_bytes(off + P.n_counters * sizeof(int32_t));

    // function descriptors and mini-bucket descriptors (offsets resolved
    // below; built now for the sizes and statistics)
    bx_status ds = fill_descriptors(P);
    if (ds != BX_OK) return ds;
    schedule_levels(P);

    // ---- value assignment schedule: level of v = 1 + max level of the
    // other variables of its bucket's functions (all earlier in the order)
    P.dvar.clear(); P.dvfn.clear(); P.dterm.clear(); P.docc.clear(); P.dpair.clear();
    P.vlevel_var_begin.clear(); P.vlevel_pair_begin.clear();
    P.dinst.assign(P.inst.size(), DevInst{});
    P.dconst.clear();
    P.max_value_levels = 0;
    P.total_vars = 0;
    int64_t sigma_elems = 0;
    for (size_t ii = 0; ii < P.inst.size(); ++ii) {
        const PInst &I = P.inst[ii];
        DevInst di{};
        di.n = I.n;
        di.vfn_begin = (int32_t)P.dvfn.size();
        di.term_begin = (int32_t)P.dterm.size() / 2;
        di.is_f32 = P.ct == BX_COST_F32;
        di.host_const = I.host_const;
        di.bound_const = I.bound_const;
        di.sigma_off = sigma_elems * 4;
        sigma_elems += align_up(std::max(I.n, 1), kAlignElems);
        P.total_vars += I.n;
        std::vector<int> vl(I.n, 0);
        int nl = 0;
        for (int p = 0; p < I.n; ++p) {
            int v = I.order[p];
            int l = 0;
            for (int32_t id : I.bucket[v])
                for (int32_t u : I.fns[id].scope) if (u != v) l = std::max(l, vl[u] + 1);
            vl[v] = l;
            nl = std::max(nl, l + 1);
        }
        di.lvl_begin = (int32_t)P.vlevel_var_begin.size();
        di.var_begin = (int32_t)P.dvar.size();
        di.pair_begin = (int32_t)P.dpair.size();
        int steps = 0;
        for (int l = 0; l < nl; ++l) {
            int32_t pairs_in_step = 0;
            bool open = false;
            for (int p = 0; p < I.n; ++p) {
                int v = I.order[p];
                if (vl[v] != l) continue;
                if (!open || pairs_in_step + I.dom[v] > kValuePairCap) {
                    P.vlevel_var_begin.push_back((int32_t)P.dvar.size());
                    P.vlevel_pair_begin.push_back((int32_t)P.dpair.size());
                    ++steps;
                    pairs_in_step = 0;
                    open = true;
                }
                DevVar dv{};
                dv.var = v;
                dv.D = I.dom[v];
                dv.f_begin = (int32_t)P.dvfn.size();
                for (int32_t id : I.bucket[v]) {
                    const PFn &f = I.fns[id];
                    DevVFn e{};
                    e.tab_off = f.off;
                    e.t_begin = (int32_t)P.dterm.size() / 2;
                    int64_t s = 1;
                    for (int j = (int)f.scope.size() - 1; j >= 0; --j) {
                        if (f.scope[j] != v) { P.dterm.push_back(f.scope[j]); P.dterm.push_back((int32_t)s); }
                        s *= I.dom[f.scope[j]];
                    }
                    e.nt = (int32_t)P.dterm.size() / 2 - e.t_begin;
                    // message tables are patched below: mark with src
                    if (f.src_mb >= 0) e.tab_off = -2 - f.src_mb;
                    P.dvfn.push_back(e);
                }
                dv.nf = (int32_t)P.dvfn.size() - dv.f_begin;
                dv.pair_begin = (int32_t)P.dpair.size();
                for (int x = 0; x < dv.D; ++x)
                    P.dpair.push_back(DevPair{(int32_t)P.dvar.size(), x, dv.f_begin, dv.nf});
                pairs_in_step += dv.D;
                P.dvar.push_back(dv);
            }
        }
        di.n_lvl = steps;
        di.var_n = (int32_t)P.dvar.size() - di.var_begin;
        di.pair_n = (int32_t)P.dpair.size() - di.pair_begin;
        P.max_value_levels = std::max(P.max_value_levels, steps);
        // the input functions, for the cost of the assignment
        di.ub_begin = (int32_t)P.dvfn.size();
        for (int f = 0; f < I.m_inputs; ++f) {
            const PFn &g = I.fns[f];
            if (g.scope.empty()) continue;
            DevVFn e{};
            e.tab_off = g.off;
            e.t_begin = (int32_t)P.dterm.size() / 2;
            int64_t s = 1;
            for (int j = (int)g.scope.size() - 1; j >= 0; --j) {
                P.dterm.push_back(g.scope[j]);
                P.dterm.push_back((int32_t)s);
                s *= I.dom[g.scope[j]];
            }
            e.nt = (int32_t)P.dterm.size() / 2 - e.t_begin;
            P.dvfn.push_back(e);
        }
        di.ub_n = (int32_t)P.dvfn.size() - di.ub_begin;
        di.vfn_n = (int32_t)P.dvfn.size() - di.vfn_begin;
        di.term_n = (int32_t)P.dterm.size() / 2 - di.term_begin;
        // the same terms grouped by variable: (function within the problem,
        // stride) for every function of the value and UB lists that has the
        // variable in its scope, so that a variable's value can be added into
        // those functions' offsets as soon as it is chosen
        di.occ_begin = (int32_t)P.docc.size() / 2;
        {
            std::vector<std::vector<std::pair<int32_t, int32_t>>> by_var(I.n);
            for (int32_t f = di.vfn_begin; f < di.vfn_begin + di.vfn_n; ++f) {
                const DevVFn &e = P.dvfn[f];
                for (int32_t t = e.t_begin; t < e.t_begin + e.nt; ++t)
                    by_var[P.dterm[2 * t]].push_back({f - di.vfn_begin, P.dterm[2 * t + 1]});
            }
            for (int32_t q = di.var_begin; q < di.var_begin + di.var_n; ++q) {
                DevVar &dv = P.dvar[q];
                dv.occ_begin = (int32_t)P.docc.size() / 2;
                for (const auto &o : by_var[dv.var]) {
                    P.docc.push_back(o.first);
                    P.docc.push_back(o.second);
                }
                dv.occ_n = (int32_t)P.docc.size() / 2 - dv.occ_begin;
            }
        }
        di.occ_n = (int32_t)P.docc.size() / 2 - di.occ_begin;
        if (di.occ_n != di.term_n) return set_error(BX_E_INVALID, "internal: value-phase terms of a variable without a value level");
        di.const_begin = (int32_t)P.dconst.size();
        for (int32_t g : I.mbs)
            if (P.mbs[g].out_id < 0) P.dconst.push_back(-2 - g);   // patched below
        di.const_n = (int32_t)P.dconst.size() - di.const_begin;
        P.dinst[ii] = di;
    }
    P.vlevel_var_begin.push_back((int32_t)P.dvar.size());
    P.vlevel_pair_begin.push_back((int32_t)P.dpair.size());
    if (P.dterm.empty()) P.dterm.push_back(0);
    if (P.docc.empty()) P.docc.assign(2, 0);

    // ---- tiles (rebuilt by retile).  The tile and segment regions hold the
    // largest lists of every tiling the planner or the tuner may choose, with
    // packing on and off.
    size_t max_tiles = 0, max_segs = 0;
    const int32_t goal0 = P.rows_per_tile > 0 ? P.rows_per_tile : kDefaultTilesGoal;
    const bool want = P.pack_on;
    for (int mode = 0; mode < (P.pack_allowed ? 2 : 1); ++mode) {
        if (P.pack_allowed) {
            ds = set_packing(P, mode == 0);
            if (ds != BX_OK) return ds;
        }
        // packed tiles counted at their most, one per group
        auto tiles_bound = [&]() {
            size_t packed = 0;
            for (int l = 0; l < P.n_levels; ++l) packed += P.level_tiled_begin[l] - P.level_pack_begin[l];
            return P.dtile.size() - packed + (size_t)P.n_groups;
        };
        for (int32_t goal : kTuneGoals) {
            retile(P, goal);
            max_tiles = std::max(max_tiles, tiles_bound());
        }
        retile(P, goal0);
        max_tiles = std::max(max_tiles, tiles_bound());
        max_segs = std::max(max_segs, (size_t)P.n_packed);   // every packed mini-bucket once
    }
    if (P.pack_allowed) {
        ds = set_packing(P, want);
        if (ds != BX_OK) return ds;
    }
    P.tile_cap = max_tiles;
    P.seg_cap = max_segs;

    // ---- byte layout
    auto place = [&](size_t &o, size_t bytes) { o = off; off = align_bytes(off + std::max<size_t>(bytes, 1)); };
    place(P.off_mb, P.dmb.size() * sizeof(DevMb));
    place(P.off_fn, P.dfn.size() * sizeof(DevFn));
    place(P.off_tile, max_tiles * sizeof(DevTile));
    place(P.off_seg, P.seg_cap * sizeof(DevSeg));
    place(P.off_var, P.dvar.size() * sizeof(DevVar));
    place(P.off_vfn, P.dvfn.size() * sizeof(DevVFn));
    place(P.off_term, P.dterm.size() * sizeof(int32_t));
    place(P.off_occ, P.docc.size() * sizeof(int32_t));
    place(P.off_pair, P.dpair.size() * sizeof(DevPair));
    place(P.off_vlv, P.vlevel_var_begin.size() * sizeof(int32_t));
    place(P.off_vlp, P.vlevel_pair_begin.size() * sizeof(int32_t));
    place(P.off_inst, P.dinst.size() * sizeof(DevInst));
    place(P.off_const, P.dconst.size() * sizeof(int64_t));
    place(P.off_zeros, 256);
    P.off_tables = off;
    P.tables_bytes = (size_t)in_elems * 4;
    off = align_bytes(off + std::max<size_t>(P.tables_bytes, 4));
    P.static_bytes = off;
    P.off_msgs = off;
    P.msgs_bytes = (size_t)msg_elems * 4;
    off = align_bytes(off + std::max<size_t>(P.msgs_bytes, 4));
    P.off_results = off;
    P.results_bytes = P.inst.size() * sizeof(DevResult);
    off = align_bytes(off + P.results_bytes);
    P.off_sigma = off;
    off = align_bytes(off + (size_t)sigma_elems * 4);
    P.total_bytes = off;

    // ---- resolve element offsets (from the workspace base)
    const int64_t tab0 = (int64_t)(P.off_tables / 4), msg0 = (int64_t)(P.off_msgs / 4);
    for (size_t g = 0; g < n_mb; ++g) P.mbs[g].out_off += msg0;
    for (PInst &I : P.inst)
        for (PFn &f : I.fns) {
            if (f.src_mb >= 0) f.off = P.mbs[f.src_mb].out_off;
            else if (!f.scope.empty()) f.off += tab0;
        }
    ds = fill_descriptors(P);    // now with resolved offsets
    if (ds != BX_OK) return ds;
    schedule_levels(P);
    retile(P, P.rows_per_tile > 0 ? P.rows_per_tile : kDefaultTilesGoal);
    for (size_t ii = 0; ii < P.inst.size(); ++ii) {
        DevInst &di = P.dinst[ii];
        for (int32_t k = 0; k < di.ub_n; ++k) P.dvfn[di.ub_begin + k].tab_off += tab0;
    }
    for (DevVFn &e : P.dvfn) {
        if (e.tab_off <= -2) e.tab_off = P.mbs[-2 - e.tab_off].out_off;
    }
    // value-phase input functions were stored table-relative; fix them
    for (size_t ii = 0; ii < P.inst.size(); ++ii) {
        const PInst &I = P.inst[ii];
        const DevInst &di = P.dinst[ii];
        int32_t lv_end = di.lvl_begin + di.n_lvl;
        for (int32_t s = di.lvl_begin; s < lv_end; ++s)
            for (int32_t ve = P.vlevel_var_begin[s]; ve < P.vlevel_var_begin[s + 1]; ++ve) {
                const DevVar &dv = P.dvar[ve];
                int32_t k = 0;
                for (int32_t id : I.bucket[dv.var]) {
                    if (I.fns[id].src_mb < 0) P.dvfn[dv.f_begin + k].tab_off = I.fns[id].off;
                    ++k;
                }
            }
    }
    for (int64_t &c : P.dconst) c = P.mbs[-2 - c].out_off;

    // ---- normalised input tables (host image of the table region)
    P.tables.assign(P.tables_bytes, 0);
    for (size_t pi = 0; pi < probs.size(); ++pi) {
        const Problem &pr = *probs[pi];
        const PInst &I = P.inst[pi];
        for (int f = 0; f < I.m_inputs; ++f) {
            const PFn &g = I.fns[f];
            if (g.scope.empty()) continue;
            const Function &src = pr.fns[f];
            const int a = (int)src.scope.size();
            // stride of each caller-order scope position in the normalised table
            std::vector<int64_t> ns(a, 0);
            for (int j = 0; j < a; ++j) {
                int64_t s = 1;
                for (int q = (int)g.scope.size() - 1; q >= 0 && g.scope[q] != src.scope[j]; --q) s *= I.dom[g.scope[q]];
                ns[j] = s;
            }
            std::vector<int32_t> dig(a, 0);
            int64_t dst = 0;
            uint8_t *base = P.tables.data() + (size_t)(g.off - tab0) * 4;
            for (int64_t r = 0; r < g.size; ++r) {
                if (P.ct == BX_COST_I32) reinterpret_cast<int32_t *>(base)[dst] = src.ti[r];
                else reinterpret_cast<float *>(base)[dst] = src.tf[r];
                // odometer over the caller's scope, last position fastest
                for (int j = a - 1; j >= 0; --j) {
                    dst += ns[j];
                    if (++dig[j] < I.dom[src.scope[j]]) break;
                    dst -= ns[j] * I.dom[src.scope[j]];
                    dig[j] = 0;
                }
            }
        }
    }
    P.tuned_valid = false;
    return BX_OK;
}

// Tiles: tiled-path mini-buckets are cut into runs of outer indices holding
// about `target_rows` rows (a multiple of q outer indices, at most
// kTileMaxOuter); row-path mini-buckets into runs of kRowTileRows rows;
// lane-group mini-buckets into kLanePasses passes of 256 / G rows.  Tiles are grouped by level, mini-buckets in
// creation order inside a level.
int64_t outer_per_tile(const DevMb &d, int32_t target_rows) {
    if (d.blk) {   // whole boxes, a multiple of q boxes when the tile holds q
        const int64_t box = (int64_t)d.da * d.db;
        const int64_t cap = kTileMaxOuter / box;
        int64_t nb = std::max<int64_t>(1, target_rows / (d.p_in * box));
        nb = std::min<int64_t>(nb, cap);
        if (nb >= d.q) nb = nb / d.q * d.q;
        return nb * box;
    }
    int64_t no = std::max<int64_t>(1, target_rows / d.p_in);
    no = std::min<int64_t>(no, kTileMaxOuter);
    no = std::max<int64_t>(d.q, no / d.q * d.q);
    return std::min<int64_t>(no, kTileMaxOuter);
}

// Lane functions of a staging-eligible mini-bucket ordered by the span of
// table entries one tile reads (the device stages a prefix of them in LDS):
// exact for the first tile, whose outer indices are enumerated.
static void order_lanes_for_staging(Plan &P, int32_t g, int64_t n_o) {
    const DevMb &d = P.dmb[g];
    if (d.path != 0 || d.blk || d.nfl < 2 || d.nfl > kStageMaxFns || d.D > kStageMaxD) return;
    const int nvo = d.nv - d.n_inner;
    DevFn *lane = P.dfn.data() + d.f_begin;
    std::vector<std::pair<int64_t, int>> span(d.nfl);
    for (int f = 0; f < d.nfl; ++f) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int64_t o = 0; o < n_o; ++o) {
            int64_t rem = o, off = 0;
            for (int j = nvo - 1; j >= 0; --j) {
                off += (rem % d.dims[j]) * lane[f].stride[j];
                rem /= d.dims[j];
            }
            lo = std::min(lo, off);
            hi = std::max(hi, off);
        }
        span[f] = {hi - lo + lane[f].io_max + d.D, f};
    }
    std::stable_sort(span.begin(), span.end());
    std::vector<DevFn> sorted(d.nfl);
    for (int f = 0; f < d.nfl; ++f) sorted[f] = lane[span[f].second];
    std::copy(sorted.begin(), sorted.end(), lane);
}

void retile(Plan &P, int32_t tiles_goal) {
    P.rows_per_tile = tiles_goal;
    P.level_goal.assign(P.n_levels, tiles_goal);
    retile_levels(P);
}

// Tiles with the per-level goals in P.level_goal.
void retile_levels(Plan &P) {
    if (P.level_goal.size() != (size_t)P.n_levels) P.level_goal.assign(P.n_levels, kDefaultTilesGoal);
    P.dtile.clear();
    P.level_tile_begin.assign(P.n_levels + 1, 0);
    P.level_row_begin.assign(P.n_levels, 0);
    P.level_lane_begin.assign(P.n_levels, 0);
    P.level_pack_begin.assign(P.n_levels, 0);
    P.level_tiled_begin.assign(P.n_levels, 0);
    P.dseg.clear();
    if (P.level_stage.size() != (size_t)P.n_levels) P.level_stage.assign(P.n_levels, 1);
    if (P.level_nt.size() != (size_t)P.n_levels) P.level_nt.assign(P.n_levels, 0);
    if (P.level_xcd.size() != (size_t)P.n_levels) P.level_xcd.assign(P.n_levels, 0);
    std::vector<std::vector<int32_t>> by_level(P.n_levels);
    for (size_t g = 0; g < P.mbs.size(); ++g) by_level[P.mbs[g].level].push_back((int32_t)g);
    std::vector<std::vector<int32_t>> gmem(P.mbs.size());   // members of each packed group
    for (size_t g = 0; g < P.mbs.size(); ++g)
        if (P.mbs[g].group >= 0) gmem[P.mbs[g].group].push_back((int32_t)g);
    for (int l = 0; l < P.n_levels; ++l) {
        P.level_tile_begin[l] = (int32_t)P.dtile.size();
        // mini-buckets whose input messages were written last go first: those
        // messages are the likeliest to still be in the device's caches
        // (tiles run roughly in list order)
        {
            std::vector<std::pair<int64_t, int32_t>> key;
            for (int32_t g : by_level[l]) {
                const DevMb &d = P.dmb[g];
                int64_t k = -1;
                for (int f = 0; f < d.nf; ++f) {
                    const int32_t src = P.dfn[d.f_begin + f].src_mb;   // producers of earlier levels
                    if (src >= 0 && P.mbs[src].level < l) k = std::max<int64_t>(k, P.mbs[src].done_tile);
                }
                key.emplace_back(-k, g);
            }
            std::stable_sort(key.begin(), key.end());
            for (size_t i = 0; i < key.size(); ++i) by_level[l][i] = key[i].second;
        }
        // rows per tile for this level: the level's rows spread over about
        // level_goal[l] tiles, within [kMinTileRows, kMaxTileRows]
        int64_t level_rows = 0;
        for (int32_t g : by_level[l]) level_rows += P.dmb[g].out_rows;
        const int32_t target = (int32_t)std::min<int64_t>(
            kMaxTileRows, std::max<int64_t>(kMinTileRows, level_rows / std::max(1, P.level_goal[l])));
        // packed groups launched at this level first (their roots in list
        // order), several to a tile while every stage stays within
        // pack_stage_rows rows and the tile within kPackMaxSegs mini-buckets
        P.level_pack_begin[l] = (int32_t)P.dtile.size();
        std::vector<std::vector<int32_t>> cur;   // per stage: the tile's mini-buckets
        std::vector<int64_t> cur_rows;
        int32_t cur_segs = 0;
        auto flush = [&]() {
            if (cur_segs == 0) return;
            DevTile t{};
            t.mb = -1;
            t.begin = (int64_t)P.dseg.size();
            for (size_t k = 0; k < cur.size(); ++k) {
                if (cur[k].empty()) continue;
                int32_t first = 0;
                const size_t s0 = P.dseg.size();
                for (int32_t g : cur[k]) {
                    const DevMb &d = P.dmb[g];
                    DevSeg e{};
                    e.out_off = d.out_off;
                    e.nf = d.nf;
                    e.nv = d.nv;
                    e.D = d.D;
                    e.red = d.red;
                    e.mb = g;
                    e.first = first;
                    const int sh = kPackMaxVars - d.nv;   // right-aligned slots
                    for (int j = 0; j < kPackMaxVars; ++j) e.dims[j] = 1;
                    for (int j = 0; j < d.nv; ++j) e.dims[sh + j] = (uint16_t)d.dims[j];
                    for (int f = 0; f < d.nf; ++f) {
                        const DevFn &fn = P.dfn[d.f_begin + f];
                        e.tab_off[f] = fn.tab_off;
                        for (int j = 0; j < d.nv; ++j) e.stride[f][sh + j] = (uint16_t)fn.stride[j];
                    }
                    P.dseg.push_back(e);
                    first += (int32_t)P.mbs[g].out_rows;
                }
                for (size_t q = s0; q < P.dseg.size(); ++q) {
                    P.dseg[q].stage_segs = (int32_t)(P.dseg.size() - s0);
                    P.dseg[q].stage_rows = first;
                }
            }
            t.end = (int64_t)P.dseg.size();
            const int32_t ti = (int32_t)P.dtile.size();
            P.dtile.push_back(t);
            for (auto &v : cur)
                for (int32_t g : v) P.mbs[g].done_tile = ti + 1;
            cur.clear();
            cur_rows.clear();
            cur_segs = 0;
        };
        for (int32_t r : by_level[l]) {
            if (P.mbs[r].group != r) continue;
            std::vector<std::vector<int32_t>> gs(P.mbs[r].stage + 1);
            std::vector<int64_t> grows(gs.size(), 0);
            int32_t nseg = 0;
            for (int32_t g : gmem[r]) {   // the group's members, by stage
                gs[P.mbs[g].stage].push_back(g);
                grows[P.mbs[g].stage] += P.mbs[g].out_rows;
                ++nseg;
            }
            bool fits = cur_segs + nseg <= kPackMaxSegs;
            for (size_t k = 0; fits && k < gs.size(); ++k)
                fits = (k < cur_rows.size() ? cur_rows[k] : 0) + grows[k] <= P.pack_stage_rows;
            if (!fits) flush();
            if (cur.size() < gs.size()) {
                cur.resize(gs.size());
                cur_rows.resize(gs.size(), 0);
            }
            for (size_t k = 0; k < gs.size(); ++k) {
                cur[k].insert(cur[k].end(), gs[k].begin(), gs[k].end());
                cur_rows[k] += grows[k];
            }
            cur_segs += nseg;
        }
        flush();
        // tiled-path mini-buckets next, then the row path and the lane
        // groups (one launch runs them all, each tile on its own path)
        P.level_tiled_begin[l] = (int32_t)P.dtile.size();
        for (int path = 0; path < 3; ++path) {
            if (path == 1) P.level_row_begin[l] = (int32_t)P.dtile.size();
            if (path == 2) P.level_lane_begin[l] = (int32_t)P.dtile.size();
            for (int32_t g : by_level[l]) {
                const DevMb &d = P.dmb[g];
                if (d.path != path) continue;
                PMb &mb = P.mbs[g];
                mb.first_tile = (int32_t)P.dtile.size();
                const int64_t total = d.path == 0 ? d.n_outer : d.out_rows;
                const int64_t step = d.path == 0   ? outer_per_tile(d, target)
                                     : d.path == 1 ? kRowTileRows
                                                   : (int64_t)(kUtilThreads / d.lanes) * kLanePasses;
                for (int64_t r = 0; r < total; r += step) {
                    DevTile t{};
                    t.mb = g;
                    t.begin = r;
                    t.end = std::min<int64_t>(total, r + step);
                    P.dtile.push_back(t);
                }
                mb.n_tiles = (int32_t)P.dtile.size() - mb.first_tile;
                mb.done_tile = (int32_t)P.dtile.size();
                P.dmb[g].n_tiles = mb.n_tiles;
                if (d.path == 0) order_lanes_for_staging(P, g, std::min<int64_t>(total, step));
            }
        }
    }
    P.level_tile_begin[P.n_levels] = (int32_t)P.dtile.size();
    // the per-bucket schedule runs a packed mini-bucket alone, on row tiles
    // of its own (after every level's tiles)
    for (size_t g = 0; g < P.mbs.size(); ++g) {
        if (P.dmb[g].path != 3) continue;
        PMb &mb = P.mbs[g];
        mb.first_tile = (int32_t)P.dtile.size();
        for (int64_t r = 0; r < mb.out_rows; r += kRowTileRows) {
            DevTile t{};
            t.mb = (int32_t)g;
            t.begin = r;
            t.end = std::min<int64_t>(mb.out_rows, r + kRowTileRows);
            P.dtile.push_back(t);
        }
        mb.n_tiles = (int32_t)P.dtile.size() - mb.first_tile;
        P.dmb[g].n_tiles = mb.n_tiles;
    }
}

// Simulated runtime of the distributed run (Sec. 8 measures the DCOP
// algorithms by simulated runtime): every variable is an agent whose clock
// advances by its own work, and a message reaches its receiver `latency_ms`
// after the sender's clock at sending.  UTIL phase: agent v starts when the
// messages of every producer in its bucket have arrived and then computes
// its mini-buckets one after another (their device times in mb_ms, creation
// order of the problem's mini-buckets); util_ms = the latest finish.  VALUE
// phase: agent v decides once the values of the other variables of its
// bucket's functions have arrived (local work taken as zero); value_ms = the
// latest decision, value_hops = the longest chain of VALUE messages.
bx_status simulated_runtime(const Plan &P, int32_t prob, const float *mb_ms, double latency_ms,
                            double *util_ms, double *value_ms, int32_t *value_hops) {
    const PInst &I = P.inst[prob];
    std::vector<double> work(I.n, 0.0), fin(I.n, 0.0), vfin(I.n, 0.0);
    std::vector<int32_t> hops(I.n, 0);
    for (size_t k = 0; k < I.mbs.size(); ++k) {
        const double t = mb_ms[k];
        if (!(t >= 0.0)) return set_error(BX_E_INVALID, "mini-bucket time is negative or NaN");
        work[P.mbs[I.mbs[k]].var] += t;
    }
    double u = 0.0, w = 0.0;
    int32_t h = 0;
    for (int p = I.n - 1; p >= 0; --p) {   // producers are eliminated before their consumers
        const int32_t v = I.order[p];
        double start = 0.0;
        for (int32_t id : I.bucket[v]) {
            const int32_t src = I.fns[id].src_mb;
            if (src >= 0) start = std::max(start, fin[P.mbs[src].var] + latency_ms);
        }
        fin[v] = start + work[v];
        u = std::max(u, fin[v]);
    }
    for (int p = 0; p < I.n; ++p) {        // values flow from the root down
        const int32_t v = I.order[p];
        for (int32_t id : I.bucket[v])
            for (int32_t x : I.fns[id].scope) {
                if (x == v) continue;
                if (vfin[x] + latency_ms > vfin[v]) vfin[v] = vfin[x] + latency_ms;
                hops[v] = std::max(hops[v], hops[x] + 1);
            }
        w = std::max(w, vfin[v]);
        h = std::max(h, hops[v]);
    }
    if (util_ms) *util_ms = u;
    if (value_ms) *value_ms = w;
    if (value_hops) *value_hops = h;
    return BX_OK;
}

// Self-check of the launch schedule (host only): every mini-bucket is
// computed by exactly one launch level, its rows covered once; every
// producer finishes in an earlier level, or inside the same packed tile at
// an earlier stage; packed tiles' segment headers are consistent; the tile
// and segment lists fit their workspace regions.
bx_status validate_schedule(const Plan &P) {
    auto fail = [](const std::string &m) { return set_error(BX_E_INVALID, "schedule check: " + m); };
    const size_t n = P.mbs.size();
    std::vector<int64_t> covered(n, 0);
    std::vector<int32_t> lev(n, -1), tile_of(n, -1), stage_of(n, -1);
    if (P.dtile.size() > P.tile_cap) return fail("tile list exceeds its region");
    if (P.dseg.size() > P.seg_cap) return fail("segment list exceeds its region");
    if ((int)P.level_tile_begin.size() != P.n_levels + 1) return fail("level table size");
    for (int l = 0; l < P.n_levels; ++l) {
        const int32_t t0 = P.level_tile_begin[l], t1 = P.level_tile_begin[l + 1];
        const int32_t tp = P.level_pack_begin[l], tt = P.level_tiled_begin[l];
        const int32_t tr = P.level_row_begin[l], tl = P.level_lane_begin[l];
        if (!(t0 == tp && tp <= tt && tt <= tr && tr <= tl && tl <= t1)) return fail("level ranges out of order");
        for (int32_t t = t0; t < t1; ++t) {
            const DevTile &T = P.dtile[t];
            if (t >= tt) {
                const int want = t < tr ? 0 : (t < tl ? 1 : 2);
                if (T.mb < 0 || T.mb >= (int32_t)n) return fail("tile names no mini-bucket");
                const DevMb &d = P.dmb[T.mb];
                if (d.path != want) return fail("tile on the wrong path");
                // the box shapes the blocked loop is built for
                if (d.blk && !(d.D <= kBlockMaxD && d.db >= 2 &&
                               ((d.da == 1 && d.db <= kBlockMaxDb1) ||
                                (d.da >= 2 && d.da <= kBlockMaxDa && d.db <= kBlockMaxDb && d.D <= kBlockMaxD2))))
                    return fail("register-blocked box of an unsupported shape");
                const int64_t total = d.path == 0 ? d.n_outer : d.out_rows;
                if (T.begin != covered[T.mb] || T.end <= T.begin || T.end > total) return fail("tile rows not contiguous");
                covered[T.mb] = T.end;
                if (lev[T.mb] >= 0 && lev[T.mb] != l) return fail("mini-bucket split over levels");
                lev[T.mb] = l;
                continue;
            }
            if (T.mb != -1 || T.begin < 0 || T.end > (int64_t)P.dseg.size() || T.begin >= T.end ||
                T.end - T.begin > kPackMaxSegs)
                return fail("packed tile header");
            int st = 0;
            for (int64_t s0 = T.begin; s0 < T.end; ++st) {
                const DevSeg &h = P.dseg[s0];
                if (h.first != 0 || h.stage_segs < 1 || s0 + h.stage_segs > T.end) return fail("stage header");
                int32_t first = 0;
                for (int64_t q = s0; q < s0 + h.stage_segs; ++q) {
                    const DevSeg &g = P.dseg[q];
                    if (g.first != first || g.stage_segs != h.stage_segs || g.stage_rows != h.stage_rows)
                        return fail("segment offsets");
                    if (g.mb < 0 || g.mb >= (int32_t)n || P.dmb[g.mb].path != 3) return fail("segment mini-bucket");
                    if (tile_of[g.mb] >= 0) return fail("packed mini-bucket placed twice");
                    tile_of[g.mb] = t;
                    stage_of[g.mb] = st;
                    lev[g.mb] = l;
                    covered[g.mb] = P.mbs[g.mb].out_rows;
                    first += (int32_t)P.mbs[g.mb].out_rows;
                }
                if (first != h.stage_rows) return fail("stage rows");
                s0 += h.stage_segs;
            }
        }
    }
    for (size_t g = 0; g < n; ++g) {
        const DevMb &d = P.dmb[g];
        const int64_t total = d.path == 0 ? d.n_outer : d.out_rows;
        if (lev[g] < 0 || covered[g] != total) return fail("mini-bucket " + std::to_string(g) + " not covered");
        const PInst &I = P.inst[P.mbs[g].inst];
        for (int32_t id : P.mbs[g].members) {
            const int32_t c = I.fns[id].src_mb;
            if (c < 0) continue;
            const bool same_tile = tile_of[g] >= 0 && tile_of[c] == tile_of[g];
            if (same_tile ? stage_of[c] >= stage_of[g] : lev[c] >= lev[g])
                return fail("mini-bucket " + std::to_string(g) + " runs before its producer " + std::to_string(c));
        }
        // the per-bucket schedule's own tiles of a mini-bucket
        const PMb &mb = P.mbs[g];
        int64_t pos = 0;
        for (int32_t t = mb.first_tile; t < mb.first_tile + mb.n_tiles; ++t) {
            const DevTile &T = P.dtile[t];
            if (T.mb != (int32_t)g || T.begin != pos) return fail("per-bucket tiles");
            pos = T.end;
        }
        if (mb.n_tiles > 0 && pos != total) return fail("per-bucket tiles do not cover the rows");
    }
    return BX_OK;
}

}  // namespace bx
