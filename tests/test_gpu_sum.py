"""The sum-product variant (Sec. 10's extension: partition function,
probability of evidence) on the device against the FP64 oracle.

Tolerance, derived from the FP32 arithmetic (u = 2^-24): an input cost is
rounded once (error u|c|); a sum of k costs adds at most (k-1) u sum|c|; the
minimum adds nothing; a summing elimination m - ln sum_x exp(m - a_x) is
1-Lipschitz in its inputs and adds at most (D + 1 + ln D + |g|) u (the D
exponentials and their sum, the logarithm, the final subtraction).  These
add up along the bucket tree: `_error_bounds` evaluates the recursion on the
oracle's own tables, and tables, bounds and assignment costs must lie within
twice that bound (the factor covers second-order terms).
"""
import math

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth
from oracle import brute

U = 2.0 ** -24


def _costs(inst, t):
    t = np.asarray(t, np.float64)
    if inst.kind == "prob_f64":
        with np.errstate(divide="ignore"):
            return -np.log(t)
    return t


def _absmax(a):
    a = np.abs(np.asarray(a, np.float64))
    a = a[np.isfinite(a)]
    return float(a.max()) if a.size else 0.0


def _error_bounds(inst, res, sum_mode=True):
    cmax = {i: _absmax(_costs(inst, t)) for i, t in enumerate(inst.tables)}
    err = {i: U * cmax[i] for i in range(inst.m)}
    bound = sum(err[i] for i, s in enumerate(inst.scopes) if len(s) == 0)
    per_mb = []
    for mb in res.minibuckets:
        k = len(mb.members)
        e = sum(err[f] for f in mb.members) + (k - 1) * U * sum(cmax[f] for f in mb.members)
        gmax = _absmax(mb.table)
        if sum_mode and mb.k == 0:
            D = int(inst.domains[mb.var])
            e += U * (D + 1 + math.log(D) + gmax)
        per_mb.append(e)
        if mb.out_id >= 0:
            err[mb.out_id] = e
            cmax[mb.out_id] = gmax
        else:
            bound += e
    return per_mb, bound + (U * abs(res.lb) if math.isfinite(res.lb) else 0.0)


def _plan(insts, algo, ibound=0, packing=True):
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo=algo, ibound=ibound, packing=packing)
    plan.validate()
    plan.upload()
    plan.execute()
    return plan


def _check(oracle_mod, plan, k, inst, ibound, tables=True):
    res = oracle_mod.solve(inst, plan.order(k), ibound, keep_tables=True, semiring="sum")
    per_mb, tol = _error_bounds(inst, res)
    b, u, a = plan.results(k)
    if math.isinf(res.lb):
        assert math.isinf(b) and b > 0
    else:
        assert abs(b - res.lb) <= 2 * tol + 1e-30, (k, b, res.lb, tol)
    if tables:
        for i, (mb, want) in enumerate(zip(plan.minibuckets(k), res.minibuckets)):
            got = plan.util_table(k, i, mb.out_rows).astype(np.float64)
            fin = np.isfinite(want.table)
            assert np.array_equal(np.isfinite(got), fin), (k, i)
            assert np.all(np.abs(got[fin] - want.table[fin]) <= 2 * per_mb[i] + 1e-30), (k, i)
    # the device's own assignment: its cost (recomputed in FP64) bounds -ln Z
    # from above
    w = 0.0
    for s, t in zip(inst.scopes, inst.tables):
        w += float(_costs(inst, t)[brute.entry_index(inst.domains, s, a[None, :].astype(np.int64))[0]])
    if math.isfinite(res.lb):
        assert w >= res.lb - 2 * tol
    return res


def test_factor_graphs_be_sum(oracle_mod):
    """Tiny factor graphs with zero weights: BE-sum against the oracle
    (tables, -ln Z) and against exhaustive enumeration."""
    insts = [synth.tiny_factor_graph(s) for s in range(80)]
    plan = _plan(insts, "be-sum")
    for k, inst in enumerate(insts):
        res = _check(oracle_mod, plan, k, inst, 0)
        want = brute.log_partition(inst)
        assert (math.isinf(want) and math.isinf(res.lb)) or res.lb == pytest.approx(want, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("ibound", [1, 2, 3])
def test_factor_graphs_mbe_sum(oracle_mod, ibound):
    insts = [synth.tiny_factor_graph(500 + s, n_lo=4, d_lo=2, zero_frac=0.0) for s in range(60)]
    plan = _plan(insts, "mbe-sum", ibound)
    for k, inst in enumerate(insts):
        res = _check(oracle_mod, plan, k, inst, ibound)
        assert res.lb <= brute.log_partition(inst) + 1e-9


def test_probability_of_evidence(oracle_mod):
    """Belief networks of 16 variables with 4 observed: -ln P(evidence)."""
    insts = []
    for s in range(6):
        bn = synth.tiny_bayes_net(700 + s, n=16, n_parents=2, d_hi=3)
        rng = np.random.default_rng(s)
        ev = {int(v): int(rng.integers(0, bn.domains[v])) for v in rng.choice(bn.n, 4, replace=False)}
        insts.append(synth.with_evidence(bn, ev))
    plan = _plan(insts, "be-sum")
    for k, inst in enumerate(insts):
        res = _check(oracle_mod, plan, k, inst, 0)
        assert res.lb == pytest.approx(brute.log_partition(inst), rel=1e-9, abs=1e-9)


def test_belief_network_100_mbe_sum_i20(oracle_mod):
    """The MPE workload's networks (100 binary variables, 3 parents) at
    i-bound 20: every table within the derived bound of the oracle's, and the
    bound below -ln Z = 0 (no evidence: Z = 1)."""
    nets = [synth.bayes_net(s) for s in range(3)]
    plan = _plan(nets, "mbe-sum", 20)
    for k, inst in enumerate(nets):
        res = _check(oracle_mod, plan, k, inst, 20)
        assert plan.results(k)[0] <= 1e-3


def test_every_path_and_packing_off(oracle_mod):
    """Large domains (lane groups), a float grid (tiled and register-blocked
    rows) and the unpacked schedule."""
    big = []
    for s in range(3):
        rng = np.random.default_rng(900 + s)
        doms = rng.integers(9, 18, size=6).astype(np.int32)
        scopes, tables = [], []
        for (a, b) in synth.gnm_edges(rng, 6, 8):
            scopes.append(np.array([a, b], np.int32))
            tables.append(rng.uniform(0.05, 1.0, int(doms[a] * doms[b])))
        big.append(synth.Instance(domains=doms, scopes=scopes, tables=tables, kind="prob_f64"))
    grid = synth.grid_wcsp(3, rows=8, cols=8)
    fgrid = synth.Instance(domains=grid.domains, scopes=grid.scopes,
                           tables=[np.exp(-np.asarray(t, np.float64) / 400.0) for t in grid.tables],
                           kind="prob_f64")
    for packing in (True, False):
        plan = _plan(big, "be-sum", packing=packing)
        if not packing:
            assert sum(plan.level_info(l).n_lane_tiles for l in range(plan.stats().n_levels)) > 0
        for k, inst in enumerate(big):
            _check(oracle_mod, plan, k, inst, 0)
        plan = _plan([fgrid], "mbe-sum", 7, packing=packing)
        _check(oracle_mod, plan, 0, fgrid, 7)


def test_domain5_blocked_rows(oracle_mod):
    """Domain-5 problems (random DCOPs of 18 agents, costs turned into
    weights exp(-c / 50)) whose larger mini-buckets take the register-blocked
    loop with one box variable of domain 5 and D = 5: summing eliminations
    against the oracle's tables and -ln Z, and the same problems minimised
    (MPE) against the oracle's bound."""
    insts = []
    for s in range(3):
        inst = synth.dcop_candidate(40 + s, n=18, density=0.3, d=5)
        insts.append(synth.Instance(domains=inst.domains, scopes=inst.scopes,
                                    tables=[np.exp(-np.asarray(t, np.float64) / 50.0) for t in inst.tables],
                                    kind="prob_f64"))
    plan = _plan(insts, "be-sum")
    assert sum(plan.level_info(l).n_blocked for l in range(plan.stats().n_levels)) > 0
    for k, inst in enumerate(insts):
        _check(oracle_mod, plan, k, inst, 0)
    plan = _plan(insts, "be")
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), 0, keep_tables=True)
        _, tol = _error_bounds(inst, res, sum_mode=False)
        assert abs(plan.results(k)[0] - res.lb) <= 2 * tol + 1e-30
