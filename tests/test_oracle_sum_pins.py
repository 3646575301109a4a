"""Pins of the oracle's sum-product variant (the extension the paper names as
future work in Sec. 10: weighted counting / partition function /
probability of evidence).

Eliminating x sums exp(-cost) over its values instead of minimising the
cost, so Bucket Elimination returns -ln Z, Z = sum over all assignments of
the product of the factors.  Pinned here against what the mathematics fixes:
a hand-worked two-variable case; a belief network without evidence has
Z = 1 (every CPT sums to one over its child); with evidence Z = P(evidence)
by exhaustive enumeration in probability space; random factor graphs with
zero weights against exhaustive enumeration; and the mini-bucket variant
(first mini-bucket sums, the others take the maximum weight, R18) bounds
-ln Z from below, with the cost of its assignment above, and equals BE
table for table when the bound covers every bucket.
"""
import math

import numpy as np
import pytest

from paper_1608_05288_amd import synth
from oracle import brute


def _order(oracle_mod, inst, h="min-fill"):
    return oracle_mod.order(inst, h)[0]


def test_two_variable_hand_worked(oracle_mod):
    # phi(x0, x1) = [[1, 2], [3, 4]]: Z = 10; with a unary phi(x0) = [2, 1]:
    # Z = 2*(1+2) + 1*(3+4) = 13
    inst = synth.Instance(domains=np.array([2, 2], np.int32),
                          scopes=[np.array([0, 1], np.int32)],
                          tables=[np.array([1.0, 2.0, 3.0, 4.0])], kind="prob_f64")
    for order in ([0, 1], [1, 0]):
        r = oracle_mod.solve(inst, np.array(order, np.int32), 0, semiring="sum")
        assert r.lb == pytest.approx(-math.log(10.0), rel=1e-14)
    inst2 = synth.Instance(domains=np.array([2, 2], np.int32),
                           scopes=[np.array([0, 1], np.int32), np.array([0], np.int32)],
                           tables=[np.array([1.0, 2.0, 3.0, 4.0]), np.array([2.0, 1.0])], kind="prob_f64")
    r = oracle_mod.solve(inst2, np.array([0, 1], np.int32), 0, semiring="sum")
    assert r.lb == pytest.approx(-math.log(13.0), rel=1e-14)
    # eliminating x1 first: the message to x0 is -ln(1 + 2), -ln(3 + 4)
    t = r.minibuckets[0].table
    assert t == pytest.approx([-math.log(3.0), -math.log(7.0)], rel=1e-14)


def test_mini_bucket_hand_worked(oracle_mod):
    # phi02 and phi12 share x2 only; i-bound 2 splits x2's bucket in two:
    # {phi02} sums over x2, {phi12} takes the max over x2, so
    # Z_mbe = (sum_{x0,x2} phi02) * (sum_x1 max_x2 phi12)
    p02 = np.array([1.0, 2.0, 3.0, 4.0])
    p12 = np.array([0.5, 2.0, 3.0, 1.0])
    inst = synth.Instance(domains=np.array([2, 2, 2], np.int32),
                          scopes=[np.array([0, 2], np.int32), np.array([1, 2], np.int32)],
                          tables=[p02, p12], kind="prob_f64")
    r = oracle_mod.solve(inst, np.array([0, 1, 2], np.int32), 2, semiring="sum")
    z_mbe = p02.sum() * (max(0.5, 2.0) + max(3.0, 1.0))
    assert r.lb == pytest.approx(-math.log(z_mbe), rel=1e-14)
    z = sum(p02[2 * a + c] * p12[2 * b + c] for a in range(2) for b in range(2) for c in range(2))
    assert r.lb <= -math.log(z) <= r.ub


@pytest.mark.parametrize("seed", range(12))
def test_belief_network_sums_to_one(oracle_mod, seed):
    """No evidence: Z = 1, so BE gives -ln Z = 0 (every elimination of a
    child sums its CPT to one)."""
    inst = synth.tiny_bayes_net(seed, n=7, n_parents=2, d_hi=3)
    for h in ("min-fill", "min-degree"):
        r = oracle_mod.solve(inst, _order(oracle_mod, inst, h), 0, semiring="sum")
        assert abs(r.lb) <= 1e-12


@pytest.mark.parametrize("seed", range(12))
def test_probability_of_evidence(oracle_mod, seed):
    inst = synth.tiny_bayes_net(100 + seed, n=8, n_parents=2, d_hi=3)
    rng = np.random.default_rng(seed)
    ev = {int(v): int(rng.integers(0, inst.domains[v])) for v in rng.choice(inst.n, 3, replace=False)}
    inst = synth.with_evidence(inst, ev)
    want = brute.log_partition(inst)
    r = oracle_mod.solve(inst, _order(oracle_mod, inst), 0, semiring="sum")
    assert r.lb == pytest.approx(want, rel=1e-11, abs=1e-12)
    assert want > 0.0     # P(evidence) < 1


@pytest.mark.parametrize("seed", range(60))
def test_factor_graphs_against_enumeration(oracle_mod, seed):
    inst = synth.tiny_factor_graph(seed)
    want = brute.log_partition(inst)
    for h in ("min-fill", "min-degree", "degree-sort"):
        r = oracle_mod.solve(inst, _order(oracle_mod, inst, h), 0, semiring="sum")
        if math.isinf(want):
            assert math.isinf(r.lb) and r.lb > 0
        else:
            assert r.lb == pytest.approx(want, rel=1e-11, abs=1e-11)


@pytest.mark.parametrize("seed", range(60))
def test_mini_buckets_bound_log_partition(oracle_mod, seed):
    inst = synth.tiny_factor_graph(1000 + seed, n_lo=4, n_hi=8, d_lo=2, zero_frac=0.0)
    want = brute.log_partition(inst)
    o = _order(oracle_mod, inst)
    be = oracle_mod.solve(inst, o, 0, semiring="sum")
    for ib in (1, 2, 3):
        r = oracle_mod.solve(inst, o, ib, semiring="sum")
        assert r.lb <= want + 1e-9 * max(1.0, abs(want))
        assert want <= r.ub + 1e-9 * max(1.0, abs(want))
        # the assignment's cost is -ln of its weight
        w = 1.0
        for s, t in zip(inst.scopes, inst.tables):
            w *= float(np.asarray(t)[brute.entry_index(inst.domains, s, r.assignment[None, :].astype(np.int64))[0]])
        assert r.ub == pytest.approx(-math.log(w), rel=1e-12, abs=1e-12)
    big = oracle_mod.solve(inst, o, be.max_union, semiring="sum")
    assert len(big.minibuckets) == len(be.minibuckets)
    for a, b in zip(big.minibuckets, be.minibuckets):
        assert np.array_equal(a.table, b.table)


def test_sum_needs_double_costs(oracle_mod):
    inst = synth.random_wcsp(0)
    with pytest.raises(ValueError):
        oracle_mod.solve(inst, _order(oracle_mod, inst), 0, semiring="sum")
