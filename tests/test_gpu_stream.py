"""Streamed execution: every table in pinned host memory, each mini-bucket's
inputs copied in and its output computed in chunks copied out while the next
chunk runs (Sec. 6.3's concurrent transfer and execution, taken to the whole
table set).  Integer tables and bounds equal the oracle's bit for bit; float
ones stay within the FP32 tolerance; the device workspace is a small part
of what the resident plan needs."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth


def _plan(insts, algo, ibound):
    return bx.Plan([bx.Problem.from_instance(i) for i in insts], algo=algo, ibound=ibound, blocking=False)


def _check(oracle_mod, plan, insts, ibound, bounds, exact=True, semiring="min"):
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), ibound, semiring=semiring)
        if exact:
            assert bounds[k] == res.lb, (k, bounds[k], res.lb)
        else:
            assert abs(bounds[k] - res.lb) <= 1e-5 * max(1.0, abs(res.lb))
        for i, (mb, want) in enumerate(zip(plan.minibuckets(k), res.minibuckets)):
            if len(mb.out_scope) == 0:
                continue        # scalar outputs stay on the device (in the bound)
            got = plan.stream_table(k, i, mb.out_rows)
            if exact:
                assert np.array_equal(got, want.table), (k, i)
            else:
                np.testing.assert_allclose(got.astype(np.float64), want.table, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("chunk", [256, 4096])
def test_streamed_grid_and_batch(oracle_mod, chunk):
    insts = [synth.grid_wcsp(21, rows=8, cols=8)] + [synth.batch_candidate(700 + s) for s in range(12)]
    plan = _plan(insts, "mbe", 8)
    d, h = plan.stream_bytes(chunk)
    assert d < plan.workspace_bytes()
    bounds = plan.execute_streamed(chunk)
    _check(oracle_mod, plan, insts, 8, bounds)
    # the resident execute of the same plan agrees
    plan.upload()
    plan.execute()
    for k in range(len(insts)):
        assert plan.results(k)[0] == bounds[k]


def test_streamed_float_min_and_sum(oracle_mod):
    nets = [synth.bayes_net(s, n=40) for s in range(3)]
    plan = _plan(nets, "mbe", 10)
    _check(oracle_mod, plan, nets, 10, plan.execute_streamed(1024), exact=False)
    plan = _plan(nets, "mbe-sum", 10)
    _check(oracle_mod, plan, nets, 10, plan.execute_streamed(1024), exact=False, semiring="sum")


def test_streamed_full_grid_small_workspace(oracle_mod):
    """The 20x20 grid at i-bound 12 (1.1 GB of tables) through a device
    workspace of a few tens of MB."""
    inst = synth.grid_wcsp(0)
    plan = _plan([inst], "mbe", 12)
    chunk = 1 << 20
    d, h = plan.stream_bytes(chunk)
    assert d * 10 < plan.workspace_bytes()
    bounds = plan.execute_streamed(chunk)
    _check(oracle_mod, plan, [inst], 12, bounds)
