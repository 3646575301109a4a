"""Packed small mini-buckets against the oracle and against the unpacked plan.

Small mini-buckets run several to a workgroup, one row per thread, and a
connected part of the bucket tree made of them runs in one workgroup stage by
stage (children before parents, a workgroup barrier between stages).  The
rows are the same rows of Eq. (3), so integer tables equal the oracle's bit
for bit under the level schedule, the per-bucket schedule and hipGraph
replay, and equal the unpacked plan's; float tables stay within the FP32
tolerance.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth


def _plan(insts, algo, ibound, packing=True, schedule=None):
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo=algo, ibound=ibound, packing=packing)
    plan.validate()
    plan.upload()
    plan.execute(schedule=schedule)
    return plan


def _packed(plan):
    return sum(plan.level_info(l).n_packed for l in range(plan.stats().n_levels))


def _check(oracle_mod, plan, insts, ibound, exact=True):
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), ibound)
        b, u, a = plan.results(k)
        if exact:
            assert (b, u) == (res.lb, res.ub), (k, b, res.lb, u, res.ub)
            assert a.tolist() == res.assignment.tolist()
        else:
            assert abs(b - res.lb) <= 1e-5 * abs(res.lb) + 1e-6
        for i, (mb, want) in enumerate(zip(plan.minibuckets(k), res.minibuckets)):
            got = plan.util_table(k, i, mb.out_rows)
            if exact:
                assert np.array_equal(got, want.table), (k, i)
            else:
                np.testing.assert_allclose(got.astype(np.float64), want.table, rtol=1e-5, atol=1e-6)


CASES = [
    ("uneven_i10", lambda: [synth.batch_candidate(300 + s) for s in range(24)], "mbe", 10),
    ("uneven_i6", lambda: [synth.batch_candidate(400 + s) for s in range(24)], "mbe", 6),
    ("grid10_i8", lambda: [synth.grid_wcsp(11, rows=10, cols=10)], "mbe", 8),
    ("tiny_inf_i2", lambda: [synth.tiny_random(500 + s) for s in range(60)], "mbe", 2),
    ("dcop14", lambda: [synth.dcop_candidate(s, n=14, density=0.3, d=3) for s in range(6)], "dpop", 0),
]


@pytest.mark.parametrize("name,make,algo,ibound", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("schedule", [None, "per-bucket"])
def test_packed_tables_match_oracle(oracle_mod, name, make, algo, ibound, schedule):
    insts = make()
    plan = _plan(insts, algo, ibound, schedule=schedule)
    assert _packed(plan) > 0
    _check(oracle_mod, plan, insts, ibound)


def test_packing_on_off_identical_and_graph_replay(oracle_mod):
    import torch
    insts = [synth.batch_candidate(600 + s) for s in range(16)] + [synth.grid_wcsp(12, rows=8, cols=8)]
    on = _plan(insts, "mbe", 9)
    off = _plan(insts, "mbe", 9, packing=False)
    assert _packed(on) > 0 and _packed(off) == 0
    assert on.stats().n_levels < off.stats().n_levels
    ref = [[on.util_table(k, i, mb.out_rows).copy() for i, mb in enumerate(on.minibuckets(k))]
           for k in range(len(insts))]
    for k in range(len(insts)):
        assert on.results(k)[0] == off.results(k)[0]
        for i, mb in enumerate(off.minibuckets(k)):
            assert np.array_equal(ref[k][i], off.util_table(k, i, mb.out_rows)), (k, i)
    # graph replays over a poisoned workspace (inputs uploaded again), with
    # eager work between them, reproduce every table
    stream = torch.cuda.Stream()
    on.graph_create("auto", stream)
    for rep in range(3):
        on.workspace.fill_(0xFF)
        torch.cuda.synchronize()
        on.upload(stream)
        on.graph_launch(stream)
        stream.synchronize()
        torch.ones(1 << 20, device="cuda").sum().item()
        for k in range(len(insts)):
            for i, mb in enumerate(on.minibuckets(k)):
                assert np.array_equal(ref[k][i], on.util_table(k, i, mb.out_rows)), (rep, k, i)


def test_packed_rows_up_to_the_cap(oracle_mod):
    # mini-buckets of up to 65536 rows packed (the most a packed mini-bucket
    # may hold): the row decode of the packed path over its whole range
    insts = [synth.grid_wcsp(13, rows=10, cols=10)]
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=9,
                   pack=dict(pack_max_rows=1 << 20, fuse_max_stages=1))
    plan.validate()
    big = [mb.out_rows for mb in plan.minibuckets(0)]
    assert max(big) == 1 << 16
    plan.upload()
    plan.execute()
    assert _packed(plan) > 0
    _check(oracle_mod, plan, insts, 9)


def test_packed_float_mpe(oracle_mod):
    nets = [synth.bayes_net(s, n=30) for s in range(4)]
    plan = _plan(nets, "mbe", 8)
    assert _packed(plan) > 0
    _check(oracle_mod, plan, nets, 8, exact=False)
