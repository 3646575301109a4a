"""Pins of the oracle's explicit-partition branch and of two tie rules.

The partition step of Alg. 2 admits any split of a bucket into parts whose
union scopes hold at most i-bound variables; a function wider than the bound
stands alone (reading R3).  The oracle's explicit branch (`parts=` in
oracle.solve) is checked here against facts fixed outside it:
  - the paper's Sec. 2.2 example, its bucket B4 given as three singletons at
    the bound the paper calls z = 1 (i-bound 2), reproduces the example's
    buckets and message scopes (tests/golden/paper_example_structure.json);
  - any valid partition gives LB <= OPT <= UB = cost(assignment) (Sec. 2.2),
    with OPT by exhaustive search;
  - the greedy rule's own partition, given explicitly, changes nothing.
The value tie rule (R4: smallest value) and the min-fill tie order (R11:
fewest fill edges, then fewest neighbours, then lowest id) are pinned by
hand-worked cases.
"""
import json
import os

import numpy as np
import pytest

from paper_1608_05288_amd import synth
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _buckets(res):
    out = {}
    for mb in res.minibuckets:
        out.setdefault(str(mb.var), []).append(mb.members)
    return out


def _greedy_parts(res):
    """{var: [members of mini-bucket 0, 1, ...]} as the oracle ran them."""
    parts = {}
    for mb in res.minibuckets:
        parts.setdefault(mb.var, []).append(list(mb.members))
    return parts


def _same(a, b):
    assert a.lb == b.lb and a.ub == b.ub
    assert a.assignment.tolist() == b.assignment.tolist()
    assert len(a.minibuckets) == len(b.minibuckets)
    for x, y in zip(a.minibuckets, b.minibuckets):
        assert (x.var, x.k, x.members, x.out_id) == (y.var, y.k, y.members, y.out_id)
        assert x.out_scope.tolist() == y.out_scope.tolist()
        assert np.array_equal(x.table, y.table)


def test_paper_mbe_example_as_explicit_singletons(oracle_mod):
    g = _golden("paper_example_structure.json")
    rng = np.random.default_rng(5)
    inst = synth.Instance(domains=np.full(4, 2, np.int32),
                          scopes=[np.array(s, np.int32) for s in g["functions"]],
                          tables=[rng.integers(0, 10, size=4).astype(np.int32) for _ in g["functions"]])
    # B4 = {f14, f24, f34} (ids 1, 3, 4) split into singletons, as Sec. 2.2 does
    res = oracle_mod.solve(inst, np.array(g["order"]), g["mbe_ibound"], parts={3: [[1], [3], [4]]})
    assert _buckets(res) == g["mbe_buckets"]
    scopes = {str(mb.out_id): mb.out_scope.tolist() for mb in res.minibuckets if mb.out_id >= 0}
    assert scopes == g["mbe_message_scopes"]
    opt, _ = brute.optimum(inst)
    assert res.lb <= opt <= res.ub


@pytest.mark.parametrize("ibound", [1, 2, 3])
def test_explicit_greedy_partition_changes_nothing(oracle_mod, ibound):
    over_bound_singletons = 0
    for seed in range(100):
        inst = synth.tiny_random(20_000 + 31 * ibound + seed, n_lo=3, n_hi=8, d_lo=1, d_hi=3,
                                 max_arity=3, m_lo=2, m_hi=12, tightness=0.3)
        o, _ = oracle_mod.order(inst, "min-fill")
        greedy = oracle_mod.solve(inst, o, ibound)
        parts = _greedy_parts(greedy)
        for v, plist in parts.items():
            for p in plist:
                if len(p) == 1:
                    f = p[0]
                    arity = len(inst.scopes[f]) if f < inst.m else None
                    over_bound_singletons += arity is not None and arity > ibound
        given = oracle_mod.solve(inst, o, ibound, parts=parts)
        _same(given, greedy)
    if ibound < 3:
        assert over_bound_singletons > 0      # the case R3 singles out is exercised


def _random_valid_split(rng, fns, scope_of, ibound):
    """A random partition of fns whose multi-function parts fit the bound."""
    for _ in range(50):
        k = int(rng.integers(1, len(fns) + 1))
        lab = rng.integers(0, k, size=len(fns))
        parts = [[f for f, l in zip(fns, lab) if l == j] for j in range(k)]
        parts = [p for p in parts if p]
        ok = all(len(p) == 1 or len(set().union(*[set(scope_of(f)) for f in p])) <= ibound
                 for p in parts)
        if ok:
            return parts
    return [[f] for f in fns]


def test_random_valid_partitions_bracket_optimum(oracle_mod):
    """Buckets are split at random, one bucket at a time in elimination
    order (a bucket's contents are known once the buckets eliminated before
    it are fixed); every result must satisfy LB <= OPT <= UB = cost."""
    rng = np.random.default_rng(11)
    checked = 0
    for seed in range(60):
        inst = synth.tiny_random(30_000 + seed, n_lo=3, n_hi=7, d_lo=1, d_hi=3, max_arity=3,
                                 m_lo=3, m_hi=10, tightness=0.2)
        ibound = int(rng.integers(1, 4))
        o, _ = oracle_mod.order(inst, "min-fill")
        opt, _ = brute.optimum(inst)
        spec = {}
        for p in range(inst.n - 1, -1, -1):
            v = int(o[p])
            cur = oracle_mod.solve(inst, o, ibound, parts=spec)
            fns = [f for mb in cur.minibuckets if mb.var == v for f in mb.members]
            if len(fns) < 2:
                continue
            scope_of = {}
            for f in range(inst.m):
                scope_of[f] = [int(u) for u in inst.scopes[f]]
            for mb in cur.minibuckets:
                if mb.out_id >= 0:
                    scope_of[mb.out_id] = [int(u) for u in mb.out_scope]
            spec[v] = _random_valid_split(rng, fns, lambda f: scope_of[f], ibound)
        res = oracle_mod.solve(inst, o, ibound, parts=spec)
        assert res.lb <= opt <= res.ub, (seed, res.lb, opt, res.ub)
        assert brute.cost_of(inst, res.assignment) == res.ub
        checked += 1
    assert checked == 60


def test_explicit_partition_rejections(oracle_mod):
    # x0..x3 binary; f0 {x0,x1,x2}, f1 {x0,x3}, f2 {x0}; x0 eliminated first
    inst = synth.Instance(domains=np.full(4, 2, np.int32),
                          scopes=[np.array([0, 1, 2], np.int32), np.array([0, 3], np.int32),
                                  np.array([0], np.int32)],
                          tables=[np.arange(8, dtype=np.int32), np.arange(4, dtype=np.int32),
                                  np.array([3, 1], np.int32)])
    order = np.array([1, 2, 3, 0])
    # an arity-3 function alone at i-bound 2 is a valid part (R3)
    res = oracle_mod.solve(inst, order, 2, parts={0: [[0], [1, 2]]})
    assert [mb.members for mb in res.minibuckets if mb.var == 0] == [[0], [1, 2]]
    with pytest.raises(ValueError):          # two functions over the bound together
        oracle_mod.solve(inst, order, 2, parts={0: [[0, 2], [1]]})
    with pytest.raises(ValueError):          # a function of the bucket left out
        oracle_mod.solve(inst, order, 2, parts={0: [[0], [1]]})
    with pytest.raises(ValueError):          # a function listed twice
        oracle_mod.solve(inst, order, 2, parts={0: [[0], [1, 2], [2]]})


# --------------------------------------------------------------------------
# R4: value ties go to the smallest value (hand-worked)
# --------------------------------------------------------------------------
def test_value_tie_rule_hand_worked(oracle_mod):
    # x0 in {0,1,2}, x1 in {0,1}; f(x0) = [5, 2, 2]; g(x0, x1) row-major
    # over (x0, x1) = [0,0, 1,0, 0,1].  Order [x0, x1]: x1 eliminated first,
    # h(x0) = min_x1 g = [0, 0, 0]; x0 minimises f + h = [5, 2, 2] -> tie at
    # 1 and 2 -> x0 = 1; then x1 minimises g(1, x1) = [1, 0] -> x1 = 1.
    inst = synth.Instance(domains=np.array([3, 2], np.int32),
                          scopes=[np.array([0], np.int32), np.array([0, 1], np.int32)],
                          tables=[np.array([5, 2, 2], np.int32), np.array([0, 0, 1, 0, 0, 1], np.int32)])
    res = oracle_mod.solve(inst, np.array([0, 1]), 0)
    assert res.assignment.tolist() == [1, 1]
    assert res.lb == res.ub == 2
    # a full tie on x1 at x0 = 0: g(0, x1) = [0, 0] -> x1 = 0
    inst2 = synth.Instance(domains=np.array([3, 2], np.int32),
                           scopes=[np.array([0], np.int32), np.array([0, 1], np.int32)],
                           tables=[np.array([1, 2, 2], np.int32), np.array([0, 0, 1, 0, 0, 1], np.int32)])
    res2 = oracle_mod.solve(inst2, np.array([0, 1]), 0)
    assert res2.assignment.tolist() == [0, 0]


# --------------------------------------------------------------------------
# R11: min-fill ties -> fewest neighbours -> lowest id (hand-worked)
# --------------------------------------------------------------------------
def _graph(n, edges):
    return synth.Instance(domains=np.full(n, 2, np.int32),
                          scopes=[np.array(e, np.int32) for e in edges],
                          tables=[np.zeros(4, np.int32) for _ in edges])


MIN_FILL_CASES = [
    # triangle 0-1-2 with a pendant 3 on 0.  Fill: v1 0, v2 0, v3 0, v0 2 ->
    # among fill 0 the fewest neighbours is v3 (1) -> eliminated first
    # (position 3).  Then the triangle: all fill 0, degree 2 -> lowest id 0,
    # then 1 (degree 1, tie with 2 -> lowest id), then 2.
    (4, [(0, 1), (1, 2), (0, 2), (0, 3)], [2, 1, 0, 3]),
    # path 0-1-2-3 with a pendant 4 on 1.  Fill 0 and degree 1: v0, v3, v4
    # -> v0; then v3 (fill 0, degree 1; v4 ties -> lower id 3); then v2
    # (fill 0, degree 1, ties v4 -> id 2); then v1 and v4 (degree 1) -> v1;
    # v4 last.
    (5, [(0, 1), (1, 2), (2, 3), (1, 4)], [4, 1, 2, 3, 0]),
]


@pytest.mark.parametrize("n,edges,expect", MIN_FILL_CASES)
def test_min_fill_tie_order_hand_worked(oracle_mod, n, edges, expect):
    o, _ = oracle_mod.order(_graph(n, edges), "min-fill")
    assert o.tolist() == expect
