// Candidate mini-bucket partitions of an over-full bucket and their features.
//
// The partition step of Alg. 2 only asks for *a* partition of the bucket whose parts have
// at most `ibound` variables; every such partition gives a valid lower bound
// (Sec. 2.2).  The greedy rule (decreasing arity, first fit) is candidate 0;
// the others are alternative valid partitions that a learned scorer may
// prefer.  Features describe a candidate by scope sizes, how many variables
// it splits across parts, table sizes, and how much input cost variation it
// separates.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>

#include "bx_internal.h"

namespace bx {

namespace {

struct Part {
    std::vector<int32_t> ids;
    std::vector<char> in;   // variable membership
    int size = 0;
};

int extra_vars(const Part &p, const std::vector<int32_t> &scope) {
    int e = 0;
    for (int32_t u : scope) e += !p.in[u];
    return e;
}

void add_to(Part &p, int32_t id, const std::vector<int32_t> &scope) {
    p.ids.push_back(id);
    for (int32_t u : scope)
        if (!p.in[u]) { p.in[u] = 1; ++p.size; }
}

// first fit (best_fit = false) or fewest new variables (best_fit = true) over
// the functions in the given order
std::vector<std::vector<int32_t>> fit(const PInst &I, const std::vector<int32_t> &order, int ibound,
                                      bool best_fit) {
    std::vector<Part> parts;
    for (int32_t id : order) {
        const auto &sc = I.fns[id].scope;
        int pick = -1, pick_extra = 1 << 30;
        for (size_t k = 0; k < parts.size(); ++k) {
            const int e = extra_vars(parts[k], sc);
            if (parts[k].size + e > ibound) continue;
            if (!best_fit) { pick = (int)k; break; }
            if (e < pick_extra) { pick = (int)k; pick_extra = e; }
        }
        if (pick < 0) {
            parts.emplace_back();
            parts.back().in.assign(I.n, 0);
            pick = (int)parts.size() - 1;
        }
        add_to(parts[pick], id, sc);
    }
    std::vector<std::vector<int32_t>> out;
    for (auto &p : parts) out.push_back(p.ids);
    return out;
}

// grow one part at a time from the largest remaining function, adding the
// fitting function that shares most variables with the part
std::vector<std::vector<int32_t>> grow(const PInst &I, std::vector<int32_t> rest, int ibound) {
    std::stable_sort(rest.begin(), rest.end(), [&](int32_t a, int32_t b) {
        return I.fns[a].scope.size() > I.fns[b].scope.size();
    });
    std::vector<std::vector<int32_t>> out;
    while (!rest.empty()) {
        Part p;
        p.in.assign(I.n, 0);
        add_to(p, rest.front(), I.fns[rest.front()].scope);
        rest.erase(rest.begin());
        for (;;) {
            int best = -1, best_share = -1;
            for (size_t i = 0; i < rest.size(); ++i) {
                const auto &sc = I.fns[rest[i]].scope;
                const int e = extra_vars(p, sc);
                if (p.size + e > ibound) continue;
                const int share = (int)sc.size() - e;
                if (share > best_share) { best = (int)i; best_share = share; }
            }
            if (best < 0) break;
            add_to(p, rest[best], I.fns[rest[best]].scope);
            rest.erase(rest.begin() + best);
        }
        out.push_back(p.ids);
    }
    return out;
}

std::vector<std::vector<int32_t>> canonical(std::vector<std::vector<int32_t>> parts) {
    for (auto &p : parts) std::sort(p.begin(), p.end());
    std::sort(parts.begin(), parts.end());
    return parts;
}

uint64_t mix(uint64_t x) {   // splitmix64 step
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

}  // namespace

std::vector<Candidate> candidate_partitions(const PInst &I, const std::vector<int32_t> &B, int ibound,
                                            uint64_t seed) {
    std::vector<Candidate> out;
    std::vector<std::vector<std::vector<int32_t>>> seen;
    auto push = [&](std::vector<std::vector<int32_t>> parts, int gen) {
        auto c = canonical(parts);
        for (const auto &s : seen)
            if (s == c) return;
        seen.push_back(c);
        out.push_back(Candidate{std::move(parts), gen});
    };
    std::vector<int32_t> by_arity = B;
    std::stable_sort(by_arity.begin(), by_arity.end(), [&](int32_t a, int32_t b) {
        const size_t sa = I.fns[a].scope.size(), sb = I.fns[b].scope.size();
        if (sa != sb) return sa > sb;
        return a < b;
    });
    push(fit(I, by_arity, ibound, false), 0);        // the greedy rule
    push(fit(I, by_arity, ibound, true), 1);         // fewest new variables
    push(grow(I, B, ibound), 2);                     // overlap growth
    // functions ordered by their latest variable other than the bucket's
    std::vector<int32_t> by_pos = B;
    auto second = [&](int32_t id) {
        const auto &sc = I.fns[id].scope;
        return sc.size() >= 2 ? I.pos[sc[sc.size() - 2]] : -1;
    };
    std::stable_sort(by_pos.begin(), by_pos.end(), [&](int32_t a, int32_t b) { return second(a) > second(b); });
    push(fit(I, by_pos, ibound, false), 3);
    // two seeded shuffles (first fit, fewest new variables)
    for (int r = 0; r < 2; ++r) {
        std::vector<int32_t> sh = B;
        uint64_t s = seed * 1315423911ull + (uint64_t)r;
        for (size_t i = sh.size(); i > 1; --i) {
            s = mix(s);
            std::swap(sh[i - 1], sh[s % i]);
        }
        push(fit(I, sh, ibound, r == 1), 4 + r);
    }
    return out;
}

void partition_features(const PInst &I, const std::vector<int32_t> &B, int32_t v, int ibound,
                        const Candidate &c, const std::vector<double> &fn_range, float *f) {
    const int nb = (int)B.size();
    const int m = (int)c.parts.size();
    std::vector<int> cnt(I.n, 0);
    int dmax = 2;
    for (int32_t id : B)
        for (int32_t u : I.fns[id].scope) dmax = std::max(dmax, I.dom[u]);
    std::vector<int> sizes;
    std::vector<double> logs;
    int singletons = 0, max_fns = 0;
    std::vector<int> part_of(I.fns.size(), -1);
    for (int k = 0; k < m; ++k) {
        std::vector<char> in(I.n, 0);
        int s = 0;
        double lg = 0.0;
        for (int32_t id : c.parts[k]) {
            part_of[id] = k;
            for (int32_t u : I.fns[id].scope)
                if (!in[u]) { in[u] = 1; ++s; lg += std::log2((double)I.dom[u]); ++cnt[u]; }
        }
        sizes.push_back(s);
        logs.push_back(lg);
        singletons += c.parts[k].size() == 1;
        max_fns = std::max<int>(max_fns, (int)c.parts[k].size());
    }
    int nU = 0, split = 0, dup = 0;
    for (int u = 0; u < I.n; ++u) {
        if (!cnt[u]) continue;
        ++nU;
        if (u != v) {
            split += cnt[u] >= 2;
            dup += cnt[u] - 1;
        }
    }
    const int m_min = std::max(1, (nU - 1 + std::max(1, ibound - 1) - 1) / std::max(1, ibound - 1));
    const double lmax = ibound * std::log2((double)dmax);
    int msgs = 0;
    for (int32_t id : B) msgs += I.fns[id].src_mb >= 0;
    // input cost variation separated by the partition: pairs of functions in
    // different parts that share a variable other than the bucket's
    double total_range = 0.0, cut = 0.0;
    for (int32_t id : B) total_range += fn_range[id];
    for (int a = 0; a < nb; ++a)
        for (int b = a + 1; b < nb; ++b) {
            const int32_t fa = B[a], fb = B[b];
            if (part_of[fa] == part_of[fb]) continue;
            bool share = false;
            for (int32_t u : I.fns[fa].scope)
                if (u != v && std::find(I.fns[fb].scope.begin(), I.fns[fb].scope.end(), u) != I.fns[fb].scope.end()) {
                    share = true;
                    break;
                }
            if (share) cut += 0.5 * (fn_range[fa] + fn_range[fb]);
        }
    const double mean_size = std::accumulate(sizes.begin(), sizes.end(), 0.0) / m;
    const double mean_log = std::accumulate(logs.begin(), logs.end(), 0.0) / m;
    f[0] = (float)m / nb;
    f[1] = (float)m / m_min;
    f[2] = (float)nU / ibound;
    f[3] = (float)*std::max_element(sizes.begin(), sizes.end()) / ibound;
    f[4] = (float)(mean_size / ibound);
    f[5] = (float)*std::min_element(sizes.begin(), sizes.end()) / ibound;
    f[6] = nU > 1 ? (float)split / (nU - 1) : 0.f;
    f[7] = nU > 1 ? (float)dup / (nU - 1) : 0.f;
    f[8] = (float)(mean_log / lmax);
    f[9] = (float)(*std::max_element(logs.begin(), logs.end()) / lmax);
    f[10] = (float)singletons / m;
    f[11] = (float)max_fns / nb;
    f[12] = (float)msgs / nb;
    f[13] = (float)I.pos[v] / std::max(1, I.n - 1);
    f[14] = total_range > 0.0 ? (float)(cut / total_range / std::max(1, nb - 1)) : 0.f;
    f[15] = (float)c.generator / 5.f;
}

}  // namespace bx
