"""Value kernel: each of its staging cases against the oracle.  The kernel
copies an instance's value-level data (level bounds, variable and
candidate-value descriptors) and its function data (function descriptors and
each variable's occurrences in them) into one 140 KB LDS arena when they fit,
and reads from HBM what does not; these instances are sized so that each
case runs: both staged (also with about 110 occurrences per variable), only
the function data (1500 variables of domain 8: 12000 candidate values), only
the level data (30 variables, 4000 functions), and neither (600 variables of
domain 16, 3000 functions).  Bound, cost of the assignment and the
assignment itself are compared bit for bit (integer costs)."""
import numpy as np
import pytest

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth

pytestmark = pytest.mark.gpu


def _edges(rng, n_pick, count, distinct):
    out, seen = [], set()
    while len(out) < count:
        a, b = sorted(rng.integers(0, n_pick, size=2).tolist())
        if a == b or (distinct and (a, b) in seen):
            continue
        seen.add((a, b))
        out.append((a, b))
    return out


def _level_data_too_big(seed):
    # 1500 variables of domain 8; 150 constraints among the first 100
    rng = synth._rng(seed)
    return synth.wcsp_from_edges(rng, np.full(1500, 8, np.int32), _edges(rng, 100, 150, True), 0, 100,
                                 unary=False)


def _function_data_too_big(seed):
    # 30 variables of domain 3; 4000 binary constraints (pairs repeat) and unary costs
    rng = synth._rng(seed)
    return synth.wcsp_from_edges(rng, np.full(30, 3, np.int32), _edges(rng, 30, 4000, False), 0, 100,
                                 unary=True)


def _neither_fits(seed):
    # 600 variables of domain 16; 3000 binary constraints and unary costs
    rng = synth._rng(seed)
    return synth.wcsp_from_edges(rng, np.full(600, 16, np.int32), _edges(rng, 600, 3000, False), 0, 100,
                                 unary=True)


def _many_occurrences(seed):
    # 30 variables of domain 2; 1000 binary constraints (pairs repeat): every
    # variable in about 110 functions (value and cost lists), so the lanes of
    # a variable take its occurrences in several rounds; the function data
    # still fits the arena
    rng = synth._rng(seed)
    return synth.wcsp_from_edges(rng, np.full(30, 2, np.int32), _edges(rng, 30, 1000, False), 0, 100,
                                 unary=True)


CASES = [("both_staged", lambda s: synth.grid_wcsp(s, rows=12, cols=12), 8),
         ("many_occurrences", _many_occurrences, 3),
         ("function_data_only", _level_data_too_big, 4),
         ("level_data_only", _function_data_too_big, 3),
         ("neither", _neither_fits, 2)]


@pytest.mark.parametrize("name,make,ibound", CASES, ids=[c[0] for c in CASES])
def test_value_kernel_staging_cases(oracle_mod, name, make, ibound):
    insts = [make(0), make(1)]
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=ibound)
    plan.upload()
    plan.execute()
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), ibound)
        b, u, a = plan.results(k)
        assert (b, u) == (res.lb, res.ub), (name, k)
        assert a.tolist() == res.assignment.tolist(), (name, k)
