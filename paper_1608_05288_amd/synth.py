"""Seeded synthetic instance generators.

This module only draws random graphs and random cost / probability tables.
It performs none of the elimination arithmetic (no ordering, no bucket
construction, no aggregation or projection); any structural acceptance
test (for example a bound on the separator size of a pseudo-tree) is
passed in by the caller as a predicate, so that the CPU checker and the
device library each apply their own.

The graph families follow the experimental section of the paper
(Sec. 8.1, "Binary Random Networks"): random graphs with a fixed edge
count, rectangular grids with 4-neighbourhoods, and Barabasi-Albert
scale-free graphs; costs are random integers (the paper uses [0, 100] and
a tightness p2 giving the share of infinite entries).  Belief networks for
MPE (Sec. 3) get conditional probability tables whose rows are drawn from
a flat Dirichlet distribution.

Table layout everywhere: a table over scope (s_0, ..., s_{a-1}) is a flat
row-major array, s_0 most significant, s_{a-1} varying fastest.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Callable, List, Optional, Sequence

import numpy as np

INF_I32 = np.int32(2**31 - 1)


@dataclasses.dataclass
class Instance:
    """A discrete optimisation instance <X, D, C>.

    kind == "cost_i32": tables hold int32 costs in [0, INF_I32], INF_I32 = infinity.
    kind == "prob_f64": tables hold float64 probabilities (an MPE instance);
                        the cost of an entry is -ln(p).
    """
    domains: np.ndarray            # int32[n]
    scopes: List[np.ndarray]       # int32[arity] per function
    tables: List[np.ndarray]       # flat, prod(domains[scope]) entries
    kind: str = "cost_i32"
    name: str = ""
    seed: int = 0
    parents: Optional[np.ndarray] = None   # pseudo-tree parent array when supplied

    @property
    def n(self) -> int:
        return int(self.domains.shape[0])

    @property
    def m(self) -> int:
        return len(self.scopes)

    def edges(self):
        """Distinct variable pairs that share a scope (the primal graph)."""
        out = set()
        for s in self.scopes:
            s = [int(v) for v in s]
            for i in range(len(s)):
                for j in range(i + 1, len(s)):
                    a, b = min(s[i], s[j]), max(s[i], s[j])
                    out.add((a, b))
        return sorted(out)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _connected(n: int, edges: Sequence) -> bool:
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = [False] * n
    stack = [0]
    seen[0] = True
    while stack:
        u = stack.pop()
        for w in adj[u]:
            if not seen[w]:
                seen[w] = True
                stack.append(w)
    return all(seen)


def gnm_edges(rng: np.random.Generator, n: int, m: int, connected: bool = True,
              max_tries: int = 10000):
    """G(n, M): M distinct undirected edges drawn uniformly; redrawn until
    connected when asked (the paper keeps only connected graphs, Sec. 8.1)."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    if m > len(pairs):
        raise ValueError("too many edges")
    for _ in range(max_tries):
        pick = rng.choice(len(pairs), size=m, replace=False)
        edges = sorted(pairs[k] for k in pick)
        if not connected or _connected(n, edges):
            return edges
    raise RuntimeError("could not draw a connected graph")


def grid_edges(rows: int, cols: int):
    """4-neighbour grid (Sec. 8.1, grid topology); variable id = r * cols + c."""
    edges = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                edges.append((v, v + 1))
            if r + 1 < rows:
                edges.append((v, v + cols))
    return edges


def barabasi_albert_edges(rng: np.random.Generator, n: int):
    """Scale-free graph as described in Sec. 8.1: start from a connected
    2-node network and attach every new node to two existing nodes chosen
    with probability proportional to their degree; 2(n-2)+1 edges."""
    edges = [(0, 1)]
    deg = np.zeros(n, dtype=np.int64)
    deg[0] = deg[1] = 1
    for v in range(2, n):
        p = deg[:v] / deg[:v].sum()
        pick = rng.choice(v, size=min(2, v), replace=False, p=p)
        for u in sorted(int(u) for u in pick):
            edges.append((u, v))
            deg[u] += 1
            deg[v] += 1
    return sorted(edges)


def _cost_table(rng, size: int, lo: int, hi: int, tightness: float) -> np.ndarray:
    t = rng.integers(lo, hi + 1, size=size, dtype=np.int64).astype(np.int32)
    if tightness > 0.0:
        mask = rng.random(size) < tightness
        t[mask] = INF_I32
    return t


def wcsp_from_edges(rng, domains: np.ndarray, edges, cost_lo: int, cost_hi: int,
                    unary: bool = True, tightness: float = 0.0,
                    unary_tightness: float = 0.0) -> Instance:
    """Binary WCSP on the given graph: one cost table per edge (scope (a, b),
    a < b) and, when asked, one unary table per variable."""
    domains = np.asarray(domains, dtype=np.int32)
    scopes, tables = [], []
    if unary:
        for v in range(domains.shape[0]):
            scopes.append(np.array([v], dtype=np.int32))
            tables.append(_cost_table(rng, int(domains[v]), cost_lo, cost_hi,
                                      unary_tightness))
    for a, b in edges:
        scopes.append(np.array([a, b], dtype=np.int32))
        tables.append(_cost_table(rng, int(domains[a]) * int(domains[b]),
                                  cost_lo, cost_hi, tightness))
    return Instance(domains=domains, scopes=scopes, tables=tables, kind="cost_i32")


# ---------------------------------------------------------------------------
# Workload families
# ---------------------------------------------------------------------------

def random_wcsp(seed: int, n: int = 12, m_edges: int = 20, d: int = 3,
                cost_hi: int = 100, tightness: float = 0.0, unary: bool = True,
                connected: bool = True) -> Instance:
    """Random binary WCSP on G(n, M) with uniform domain d and integer costs
    in [0, cost_hi] (default: 12 variables, 20 constraints, domain 3)."""
    rng = _rng(seed)
    edges = gnm_edges(rng, n, m_edges, connected=connected)
    inst = wcsp_from_edges(rng, np.full(n, d, np.int32), edges, 0, cost_hi,
                           unary=unary, tightness=tightness)
    inst.name, inst.seed = f"random_n{n}_m{m_edges}_d{d}", seed
    return inst


def grid_wcsp(seed: int, rows: int = 20, cols: int = 20, d: int = 4,
              cost_hi: int = 1000, tightness: float = 0.0) -> Instance:
    """Grid WCSP: unary costs on every cell and binary costs on every
    4-neighbour edge (default 20x20, domain 4, costs in [0, 1000])."""
    rng = _rng(seed)
    inst = wcsp_from_edges(rng, np.full(rows * cols, d, np.int32),
                           grid_edges(rows, cols), 0, cost_hi, unary=True,
                           tightness=tightness)
    inst.name, inst.seed = f"grid{rows}x{cols}_d{d}", seed
    return inst


def scale_free_wcsp(seed: int, n: int = 20, d: int = 5, cost_hi: int = 100,
                    tightness: float = 0.0) -> Instance:
    rng = _rng(seed)
    inst = wcsp_from_edges(rng, np.full(n, d, np.int32),
                           barabasi_albert_edges(rng, n), 0, cost_hi,
                           unary=False, tightness=tightness)
    inst.name, inst.seed = f"scalefree_n{n}_d{d}", seed
    return inst


def dcop_candidate(seed: int, n: int = 25, density: float = 0.3, d: int = 5,
                   cost_hi: int = 100) -> Instance:
    """Random DCOP: one agent per variable, floor(n(n-1)p/2) binary
    constraints on a connected random graph, domain d, costs in [0, cost_hi].
    (The paper prints the edge count as floor(n(n-1)p1); with p1 > 0.5 that
    exceeds the number of vertex pairs, so the undirected count is used.)"""
    m = int(np.floor(n * (n - 1) * density / 2.0))
    rng = _rng(seed)
    edges = gnm_edges(rng, n, m, connected=True)
    inst = wcsp_from_edges(rng, np.full(n, d, np.int32), edges, 0, cost_hi,
                           unary=False)
    inst.name, inst.seed = f"dcop_n{n}_p{density}_d{d}", seed
    return inst


def accepted(make: Callable[[int], Instance], count: int, seed0: int,
             accept: Optional[Callable[[Instance], bool]] = None,
             max_draws: int = 1_000_000) -> List[Instance]:
    """Rejection sampling over consecutive seeds seed0, seed0+1, ...: keep the
    first `count` instances the caller's predicate accepts."""
    out = []
    s = seed0
    while len(out) < count:
        if s - seed0 > max_draws:
            raise RuntimeError("acceptance rate too low")
        inst = make(s)
        if accept is None or accept(inst):
            out.append(inst)
        s += 1
    return out


def bayes_net(seed: int, n: int = 100, n_parents: int = 3, d: int = 2,
              alpha: float = 1.0) -> Instance:
    """Random belief network for MPE: variables visited in a random
    topological order; each takes `n_parents` distinct parents drawn uniformly
    from the variables before it (fewer for the first ones).  The CPT of x has
    scope (parents in increasing id order, x) and each of its rows is a
    Dirichlet(alpha, ..., alpha) draw over D_x."""
    rng = _rng(seed)
    topo = rng.permutation(n)
    scopes, tables = [], []
    for k in range(n):
        x = int(topo[k])
        earlier = topo[:k]
        npar = min(n_parents, k)
        pa = sorted(int(v) for v in rng.choice(earlier, size=npar, replace=False)) if npar else []
        scope = np.array(pa + [x], dtype=np.int32)
        rows = d ** npar
        cpt = rng.dirichlet(np.full(d, alpha), size=rows).reshape(-1)
        scopes.append(scope)
        tables.append(cpt.astype(np.float64))
    inst = Instance(domains=np.full(n, d, np.int32), scopes=scopes, tables=tables,
                    kind="prob_f64", name=f"bn_n{n}_p{n_parents}", seed=seed)
    return inst


def batch_candidate(seed: int, n_lo: int = 30, n_hi: int = 80, r_lo: float = 1.5,
                    r_hi: float = 3.0, d_choices=(2, 3, 4), cost_hi: int = 100) -> Instance:
    """One member of the uneven batched family: n ~ U{n_lo..n_hi},
    G(n, floor(r n)) with r ~ U(r_lo, r_hi), per-variable domain drawn from
    d_choices, unary + binary integer costs in [0, cost_hi]."""
    rng = _rng(seed)
    n = int(rng.integers(n_lo, n_hi + 1))
    r = float(rng.uniform(r_lo, r_hi))
    m = min(int(np.floor(r * n)), n * (n - 1) // 2)
    doms = rng.choice(np.asarray(d_choices, np.int32), size=n).astype(np.int32)
    edges = gnm_edges(rng, n, m, connected=True)
    inst = wcsp_from_edges(rng, doms, edges, 0, cost_hi, unary=True)
    inst.name, inst.seed = f"batch_n{n}_m{m}", seed
    return inst


def tiny_random(seed: int, n_lo: int = 1, n_hi: int = 8, d_lo: int = 1, d_hi: int = 3,
                max_arity: int = 3, m_lo: int = 0, m_hi: int = 10,
                tightness: float = 0.5, cost_hi: int = 100,
                allow_empty_scope: bool = True) -> Instance:
    """Tiny random instance with mixed arities (0..max_arity), optional
    infinite entries: used to compare elimination with exhaustive search."""
    rng = _rng(seed)
    n = int(rng.integers(n_lo, n_hi + 1))
    doms = rng.integers(d_lo, d_hi + 1, size=n).astype(np.int32)
    m = int(rng.integers(m_lo, m_hi + 1))
    scopes, tables = [], []
    for _ in range(m):
        lo = 0 if allow_empty_scope else 1
        a = int(rng.integers(lo, min(max_arity, n) + 1))
        scope = rng.permutation(n)[:a].astype(np.int32)   # arbitrary variable order
        size = int(np.prod(doms[scope])) if a else 1
        scopes.append(scope)
        tables.append(_cost_table(rng, size, 0, cost_hi, tightness))
    return Instance(domains=doms, scopes=scopes, tables=tables, kind="cost_i32",
                    name="tiny", seed=seed)


def tiny_bayes_net(seed: int, n: int = 7, n_parents: int = 2, d_hi: int = 3) -> Instance:
    rng = _rng(seed)
    doms = rng.integers(2, d_hi + 1, size=n).astype(np.int32)
    topo = rng.permutation(n)
    scopes, tables = [], []
    for k in range(n):
        x = int(topo[k])
        npar = min(n_parents, k)
        pa = [int(v) for v in rng.choice(topo[:k], size=npar, replace=False)] if npar else []
        scope = np.array(pa + [x], dtype=np.int32)    # parents in drawn order, child last
        rows = int(np.prod(doms[pa])) if pa else 1
        cpt = rng.dirichlet(np.ones(int(doms[x])), size=rows).reshape(-1)
        scopes.append(scope)
        tables.append(cpt)
    return Instance(domains=doms, scopes=scopes, tables=tables, kind="prob_f64",
                    name="tiny_bn", seed=seed)


def tiny_factor_graph(seed: int, n_lo: int = 2, n_hi: int = 8, d_lo: int = 1, d_hi: int = 3,
                      max_arity: int = 3, m_lo: int = 1, m_hi: int = 10, zero_frac: float = 0.1) -> Instance:
    """Tiny random factor graph with non-negative factors (a share of them
    zero) in (0, 1]: unnormalised weights, kind "prob_f64" (cost -ln w), for the
    sum-product variant against exhaustive enumeration."""
    rng = _rng(seed)
    n = int(rng.integers(n_lo, n_hi + 1))
    doms = rng.integers(d_lo, d_hi + 1, size=n).astype(np.int32)
    m = int(rng.integers(m_lo, m_hi + 1))
    scopes, tables = [], []
    for _ in range(m):
        a = int(rng.integers(0, min(max_arity, n) + 1))
        scope = rng.permutation(n)[:a].astype(np.int32)
        size = int(np.prod(doms[scope])) if a else 1
        w = rng.uniform(0.05, 1.0, size)
        w[rng.random(size) < zero_frac] = 0.0
        scopes.append(scope)
        tables.append(w)
    return Instance(domains=doms, scopes=scopes, tables=tables, kind="prob_f64", name="tiny_fg", seed=seed)


def with_evidence(inst: Instance, evidence: Dict[int, int]) -> Instance:
    """A copy of a belief network with the observed values as indicator
    factors (weight 1 at the observed value, 0 elsewhere)."""
    scopes = list(inst.scopes)
    tables = list(inst.tables)
    for v, x in sorted(evidence.items()):
        t = np.zeros(int(inst.domains[v]), np.float64)
        t[int(x)] = 1.0
        scopes.append(np.array([v], np.int32))
        tables.append(t)
    return dataclasses.replace(inst, scopes=scopes, tables=tables, name=inst.name + "_ev")


def permute_scope(inst: Instance, fi: int, perm: Sequence[int]) -> Instance:
    """Return a copy of `inst` in which function fi's scope is listed in the
    order perm (a permutation of its positions) and its table re-laid out to
    match; the function itself is unchanged.  Used to check that callers may
    give scopes in any order."""
    scopes = [s.copy() for s in inst.scopes]
    tables = [t.copy() for t in inst.tables]
    s = scopes[fi]
    shape = tuple(int(inst.domains[v]) for v in s)
    t = tables[fi].reshape(shape) if len(shape) else tables[fi]
    perm = list(perm)
    scopes[fi] = s[perm]
    tables[fi] = np.ascontiguousarray(np.transpose(t, perm)).reshape(-1) if len(shape) else t
    return dataclasses.replace(inst, scopes=scopes, tables=tables)
