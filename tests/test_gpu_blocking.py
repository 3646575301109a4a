"""Register blocking of the tiled UTIL path against the oracle and against
the one-row-per-slot loop.

A blocked mini-bucket computes, per thread, every row of a box of outer
variables and loads each lane table once per value combination of the box
variables it depends on; the rows are the same rows of Eq. (3), so integer
tables must be identical bit for bit to the oracle's and to the unblocked
plan's, float tables within the FP32 tolerance.
"""
import re

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth


def _blocked(plan):
    return int(re.search(r"blocked_minibuckets=(\d+)", plan.describe()).group(1))


def _plan(insts, ibound, blocking=True, tune=False):
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=ibound,
                   blocking=blocking)
    plan.upload()
    if tune:
        plan.autotune(reps=1)
    plan.execute()
    return plan


def _tables(plan, k):
    return [plan.util_table(k, i, mb.out_rows) for i, mb in enumerate(plan.minibuckets(k))]


CASES = [
    ("grid8_d4_i9", lambda: [synth.grid_wcsp(5, rows=8, cols=8)], 9),
    ("grid10_d3_i10", lambda: [synth.grid_wcsp(6, rows=10, cols=10, d=3)], 10),
    ("uneven_i8", lambda: [synth.batch_candidate(s) for s in range(12)], 8),
    ("uneven_i7", lambda: [synth.batch_candidate(100 + s) for s in range(12)], 7),
]


@pytest.mark.parametrize("name,make,ibound", CASES, ids=[c[0] for c in CASES])
def test_blocked_tables_match_oracle(oracle_mod, name, make, ibound):
    insts = make()
    plan = _plan(insts, ibound, tune=True)
    assert _blocked(plan) > 0, plan.describe()
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), ibound)
        b, u, a = plan.results(k)
        assert (b, u) == (res.lb, res.ub)
        assert a.tolist() == res.assignment.tolist()
        for i, (got, want) in enumerate(zip(_tables(plan, k), res.minibuckets)):
            assert np.array_equal(got, want.table), (name, k, i)


def test_blocking_on_off_identical_int():
    insts = [synth.grid_wcsp(7, rows=9, cols=9)] + [synth.batch_candidate(200 + s) for s in range(6)]
    on = _plan(insts, 9)
    off = _plan(insts, 9, blocking=False)
    assert _blocked(on) > 0 and _blocked(off) == 0
    for k in range(len(insts)):
        assert on.results(k)[:2] == off.results(k)[:2]
        for i, (x, y) in enumerate(zip(_tables(on, k), _tables(off, k))):
            assert np.array_equal(x, y), (k, i)


def test_blocked_float_mpe(oracle_mod):
    # binary belief networks: -ln p in FP32 on the device, FP64 in the oracle
    insts = [synth.bayes_net(s, n=40) for s in range(3)]
    plan = _plan(insts, 12)
    off = _plan(insts, 12, blocking=False)
    assert _blocked(plan) > 0, plan.describe()
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), 12)
        b = plan.results(k)[0]
        assert abs(b - res.lb) <= 1e-5 * abs(res.lb)
        for got, want, other in zip(_tables(plan, k), res.minibuckets, _tables(off, k)):
            np.testing.assert_allclose(got.astype(np.float64), want.table, rtol=1e-5, atol=0)
            np.testing.assert_allclose(got, other, rtol=1e-6, atol=0)


FORCED = [("force_nt", bx.FLAG_FORCE_NT), ("stage_always", bx.FLAG_STAGE_ALWAYS),
          ("stage_never", bx.FLAG_STAGE_NEVER), ("nt_and_stage", bx.FLAG_FORCE_NT | bx.FLAG_STAGE_ALWAYS),
          ("xcd_order", bx.FLAG_XCD_ORDER),
          ("xcd_nt_stage", bx.FLAG_XCD_ORDER | bx.FLAG_FORCE_NT | bx.FLAG_STAGE_ALWAYS)]
FORCED_CASES = [("grid20_i12", lambda: [synth.grid_wcsp(0)], 12),
                ("uneven_i10", lambda: [synth.batch_candidate(s) for s in range(24)], 10)]


@pytest.mark.parametrize("fname,flags", FORCED, ids=[f[0] for f in FORCED])
@pytest.mark.parametrize("name,make,ibound", FORCED_CASES, ids=[c[0] for c in FORCED_CASES])
def test_forced_store_and_staging_variants_match_oracle(oracle_mod, fname, flags, name, make, ibound):
    """Every level run with the non-temporal store build and/or the staging
    kernel forced on (or staging off), or its tiles taken XCD by XCD: bounds,
    assignments and every UTIL table bit for bit against the oracle."""
    insts = make()
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=ibound, flags=flags)
    plan.upload()
    plan.execute()
    for lv in range(plan.stats().n_levels):
        li = plan.level_info(lv)
        if flags & bx.FLAG_FORCE_NT:
            assert li.nontemporal == 1
        if flags & bx.FLAG_STAGE_ALWAYS:
            assert li.staged == 1
        elif flags & bx.FLAG_STAGE_NEVER:
            assert li.staged == 0
    if flags & bx.FLAG_XCD_ORDER:
        assert f"xcd_levels={plan.stats().n_levels} " in plan.describe()
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), ibound)
        b, u, a = plan.results(k)
        assert (b, u) == (res.lb, res.ub)
        assert a.tolist() == res.assignment.tolist()
        for i, (got, want) in enumerate(zip(_tables(plan, k), res.minibuckets)):
            assert np.array_equal(got, want.table), (fname, name, k, i)
