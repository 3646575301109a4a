"""Branch and bound with the mini-bucket bound recomputed at every node (the
use Sec. 10 proposes), every expansion bounding all children in one batched
device pass: the optimum against exhaustive search."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth
from oracle import brute


@pytest.mark.parametrize("ibound", [2, 3])
def test_random_wcsp_optimum(ibound):
    """12 variables, domain 3, 20 constraints + unary (brute force 3^12):
    the search proves the optimum, and its assignment reaches it."""
    searched = 0
    for seed in range(8):
        inst = synth.random_wcsp(seed)
        opt, _ = brute.optimum(inst)
        v, a, st = bx.bnb_solve(bx.Problem.from_instance(inst), ibound=ibound)
        assert st["proved"]
        assert v == opt, (seed, v, opt)
        assert brute.cost_of(inst, a) == opt
        searched += st["nodes"] > 0
        assert st["passes"] >= 1 + st["nodes"]
    assert searched > 0      # the bound alone did not settle every instance


def test_tiny_with_infinities():
    for seed in range(40):
        inst = synth.tiny_random(300 + seed, n_lo=3, n_hi=8, d_lo=1, d_hi=3)
        opt, _ = brute.optimum(inst)
        v, a, st = bx.bnb_solve(bx.Problem.from_instance(inst), ibound=2)
        assert st["proved"] and v == opt, (seed, v, opt)
        assert brute.cost_of(inst, a) == opt


def test_exact_bound_needs_no_search_and_node_limit():
    inst = synth.random_wcsp(3)
    opt, _ = brute.optimum(inst)
    v, a, st = bx.bnb_solve(bx.Problem.from_instance(inst), algo="be")
    assert v == opt and st["nodes"] == 0 and st["proved"]
    # one expansion only: an upper bound, not proved (when a search was needed)
    v1, a1, st1 = bx.bnb_solve(bx.Problem.from_instance(inst), ibound=2, max_nodes=1)
    assert v1 >= opt and brute.cost_of(inst, a1) == v1
    assert st1["nodes"] <= 1
