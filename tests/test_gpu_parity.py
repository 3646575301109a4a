"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer work is compared bit for bit: the bound, the cost of the assignment,
the assignment (both sides break value ties towards the smallest value) and
every UTIL table.  Float (MPE, -ln p) work is compared within 1e-5 relative
on the bound, the tolerance stated for FP32 against the FP64 oracle.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth
from oracle import brute


def _run(insts, algo, ibound, order="min-fill", schedule=None, packing=True):
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo=algo, ibound=ibound, order=order,
                   packing=packing)
    plan.upload()
    plan.execute(schedule=schedule)
    return plan


def _check_tables(plan, prob, res, exact=True, rtol=0.0):
    mbs = plan.minibuckets(prob)
    assert len(mbs) == len(res.minibuckets)
    for i, (a, b) in enumerate(zip(mbs, res.minibuckets)):
        assert a.var == b.var and a.out_scope.tolist() == b.out_scope.tolist()
        got = plan.util_table(prob, i, a.out_rows)
        if exact:
            assert np.array_equal(got, b.table), (prob, i, np.nonzero(got != b.table)[0][:10])
        else:
            np.testing.assert_allclose(got.astype(np.float64), b.table, rtol=rtol, atol=0)


def _check_int(plan, prob, inst, res, tables=True):
    b, u, a = plan.results(prob)
    assert b == res.lb, (prob, b, res.lb)
    assert u == res.ub, (prob, u, res.ub)
    assert a.tolist() == res.assignment.tolist()
    if tables:
        _check_tables(plan, prob, res)


def test_random_wcsp_be_brute_force(oracle_mod):
    # 12 variables, domain 3, 20 binary constraints + unary, min-degree, BE
    for seed in range(10):
        inst = synth.random_wcsp(seed)
        plan = _run([inst], "be", 0, order="min-degree")
        o = plan.order(0)
        res = oracle_mod.solve(inst, o, 0)
        _check_int(plan, 0, inst, res)
        opt, _ = brute.optimum(inst)
        assert res.lb == opt


@pytest.mark.parametrize("ibound", [0, 2, 3])
def test_tiny_random_with_infinities(oracle_mod, ibound):
    insts = [synth.tiny_random(100 + s, n_lo=2, n_hi=9, d_lo=1, d_hi=4, m_lo=1, m_hi=14)
             for s in range(60)]
    algo = "mbe" if ibound else "be"
    plan = _run(insts, algo, ibound)
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), ibound)
        _check_int(plan, k, inst, res)


@pytest.mark.parametrize("schedule", ["per-bucket", "level"])
def test_schedules_agree(oracle_mod, schedule):
    inst = synth.grid_wcsp(2, rows=10, cols=10)
    plan = _run([inst], "mbe", 8, schedule=schedule)
    res = oracle_mod.solve(inst, plan.order(0), 8)
    _check_int(plan, 0, inst, res)


@pytest.mark.skip(reason="the persistent dataflow schedule hung on the device twice and is "
                         "disabled (it returns BX_E_UNSUPPORTED); its cause is not yet shown")
def test_schedule_dataflow_agrees(oracle_mod):
    inst = synth.grid_wcsp(2, rows=10, cols=10)
    plan = _run([inst], "mbe", 8, schedule="dataflow")
    res = oracle_mod.solve(inst, plan.order(0), 8)
    _check_int(plan, 0, inst, res)


def test_graph_replay_matches_eager(oracle_mod):
    import torch
    inst = synth.grid_wcsp(4, rows=10, cols=10)
    plan = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=8)
    plan.allocate()
    s = torch.cuda.Stream()
    res = oracle_mod.solve(inst, plan.order(0), 8)
    with torch.cuda.stream(s):          # every call below runs on s
        plan.upload(s)
        plan.graph_create("level", s)
        for rep in range(4):
            plan.graph_launch(s)
            _check_int(plan, 0, inst, res, tables=(rep == 3))
            # eager work and a synchronisation between replays
            plan.execute(schedule="per-bucket", stream=s)
            s.synchronize()
            _check_int(plan, 0, inst, res, tables=False)


def test_domains_one_to_nine(oracle_mod):
    # every eliminated-domain specialisation, including the generic one
    insts = []
    for d in range(1, 10):
        rng = np.random.default_rng(d)
        n = 7
        doms = np.full(n, d, np.int32)
        doms[rng.integers(0, n)] = max(1, d - 1)
        edges = synth.gnm_edges(rng, n, 10)
        insts.append(synth.wcsp_from_edges(rng, doms, edges, 0, 50, tightness=0.1))
    plan = _run(insts, "mbe", 3)
    for k, inst in enumerate(insts):
        _check_int(plan, k, inst, oracle_mod.solve(inst, plan.order(k), 3))


def test_repeat_and_poisoned_workspace(oracle_mod):
    import torch
    inst = synth.grid_wcsp(3, rows=9, cols=9)
    plan = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=7)
    ws = plan.allocate()
    # garbage everywhere; upload rewrites the inputs and descriptors, the
    # device must overwrite every message and result it reads
    ws.fill_(0xFF)
    plan.upload()
    res = oracle_mod.solve(inst, plan.order(0), 7)
    for rep in range(3):
        plan.execute()
        torch.cuda.synchronize()
        _check_int(plan, 0, inst, res, tables=(rep != 1))


def test_grid_mbe_ibound12_full(oracle_mod):
    # 20x20 grid, domain 4, costs in [0, 1000], MBE i-bound 12, min-fill
    inst = synth.grid_wcsp(0)
    plan = _run([inst], "mbe", 12)
    res = oracle_mod.solve(inst, plan.order(0), 12)
    _check_int(plan, 0, inst, res, tables=True)
    assert plan.stats().util_rows == 140224149


def test_mpe_float_tolerance_small(oracle_mod):
    for seed in range(20):
        inst = synth.tiny_bayes_net(seed)
        plan = _run([inst], "be", 0)
        res = oracle_mod.solve(inst, plan.order(0), 0)
        b, u, a = plan.results(0)
        assert abs(b - res.lb) <= 1e-5 * abs(res.lb)
        pmax, _ = brute.mpe(inst)
        assert abs(b + np.log(pmax)) <= 1e-5 * abs(np.log(pmax))
        _check_tables(plan, 0, res, exact=False, rtol=1e-5)


def test_mpe_bn100_ibound20(oracle_mod):
    # belief network: 100 binary variables, 3 parents each, Dirichlet(1) CPTs,
    # FP32 -ln p on the device vs the FP64 oracle, MBE i-bound 20
    for seed in range(2):
        inst = synth.bayes_net(seed)
        plan = _run([inst], "mbe", 20)
        res = oracle_mod.solve(inst, plan.order(0), 20, keep_tables=False)
        b, u, a = plan.results(0)
        assert abs(b - res.lb) <= 1e-5 * abs(res.lb), (b, res.lb)
        # the device's assignment is valid: its cost (fp64) is >= the bound
        assert u >= b - 1e-5 * abs(b)


def _max_sep_oracle(oracle_mod, inst):
    o, par = oracle_mod.order(inst, "dfs")
    seps = oracle_mod.separators(inst, par)
    return max(len(s) for s in seps)


def test_dpop_small(oracle_mod):
    for seed in range(8):
        inst = synth.dcop_candidate(seed, n=14, density=0.3, d=3)
        plan = _run([inst], "dpop", 0)
        res = oracle_mod.solve(inst, plan.order(0), 0)
        _check_int(plan, 0, inst, res)


@pytest.mark.slow
def test_dpop_25_agents_sep10(oracle_mod):
    # 25 agents, domain 5, density 0.3 (90 constraints), DFS pseudo-tree with
    # largest separator <= 10, accepted by rejection sampling over seeds
    inst = _dcop25(oracle_mod)
    plan = _run([inst], "dpop", 0)
    res = oracle_mod.solve(inst, plan.order(0), 0, keep_tables=True)
    _check_int(plan, 0, inst, res, tables=True)


def _dcop25(oracle_mod):
    return synth.accepted(lambda s: synth.dcop_candidate(s), 1, 0,
                          accept=lambda i: _max_sep_oracle(oracle_mod, i) <= 10)[0]


@pytest.mark.parametrize("ibound", [4, 6, 8])
def test_adpop_25_agents(oracle_mod, ibound):
    """ADPOP (Sec. 4.2): MBE along the DFS pseudo-tree order of the 25-agent,
    domain-5 DCOP.  The library's pseudo-tree equals the oracle's; every UTIL
    message, the bound, the cost and the assignment equal the oracle's MBE
    run along that order bit for bit; every message scope stays within the
    bound (i-bound - 1 output variables, functions are binary); and the bound
    brackets the DPOP optimum on the same pseudo-tree."""
    inst = _dcop25(oracle_mod)
    o, par = oracle_mod.order(inst, "dfs")
    plan = _run([inst], "adpop", ibound)
    assert plan.order(0).tolist() == o.tolist()
    res = oracle_mod.solve(inst, o, ibound, keep_tables=True)
    _check_int(plan, 0, inst, res, tables=True)
    assert max(len(mb.out_scope) for mb in plan.minibuckets(0)) <= ibound - 1
    opt = oracle_mod.solve(inst, o, 0, keep_tables=False).lb
    b, u, _ = plan.results(0)
    assert b <= opt <= u


def test_batched_uneven(oracle_mod):
    # uneven batch: 30-80 variables, domains 2-4, MBE i-bound 10
    insts = [synth.batch_candidate(s) for s in range(48)]
    plan = _run(insts, "mbe", 10)
    per = _run(insts, "mbe", 10, schedule="per-bucket")
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), 10, keep_tables=False)
        _check_int(plan, k, inst, res, tables=False)
        assert per.results(k)[0] == res.lb


def test_batched_family_256_with_tables(oracle_mod):
    """The batched family at its full size: 256 uneven random WCSPs (30-80
    variables, domains 2-4, min-fill width 8-16 by the oracle's own width),
    MBE i-bound 10, autotuned (packing chosen by the tuner), replayed from a
    captured hipGraph: every UTIL table, bound, cost and assignment against
    the oracle bit for bit."""
    import torch

    def width_ok(inst):
        o, _ = oracle_mod.order(inst, "min-fill")
        return 8 <= oracle_mod.induced_width(inst, o) <= 16
    insts = synth.accepted(synth.batch_candidate, 256, 0, accept=width_ok)
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=10)
    plan.upload()
    plan.autotune(reps=1)
    s = torch.cuda.Stream()
    plan.graph_create("auto", s)
    plan.graph_launch(s)
    s.synchronize()
    for k, inst in enumerate(insts):
        res = oracle_mod.solve(inst, plan.order(k), 10, keep_tables=True)
        _check_int(plan, k, inst, res, tables=True)


def _edge_instances():
    INF = 2**31 - 1

    def inst(doms, scopes, tables):
        return synth.Instance(domains=np.array(doms, np.int32),
                              scopes=[np.array(s, np.int32) for s in scopes],
                              tables=[np.array(t, np.int32) for t in tables], kind="cost_i32")
    return [
        inst([], [], []),                                    # no variables at all
        inst([], [[]], [[7]]),                               # a constant only
        inst([3], [], []),                                   # a variable without functions
        inst([3], [[0]], [[5, 2, 9]]),                       # one unary function
        inst([2, 2], [[0, 1]], [[INF, INF, INF, INF]]),      # every combination forbidden
        inst([1, 1, 1], [[0, 1], [2]], [[4], [INF]]),        # domain-1 variables, infeasible
        inst([2, 3, 2], [[2, 0], [1]], [[1, 2, 3, 4], [0, 0, 1]]),
    ]


@pytest.mark.parametrize("algo,ibound", [("be", 0), ("mbe", 1), ("mbe", 2)])
def test_degenerate_instances(oracle_mod, algo, ibound):
    """Empty problems, constants only, variables without functions, domain-1
    variables and infeasible problems: alone and batched with a normal
    instance, bounds, costs and assignments equal the oracle's."""
    edge = _edge_instances()
    for group in [[e] for e in edge] + [edge + [synth.random_wcsp(3)]]:
        plan = _run(group, algo, ibound)
        for k, inst in enumerate(group):
            res = oracle_mod.solve(inst, plan.order(k), ibound)
            _check_int(plan, k, inst, res)


def test_autotune_discards_the_captured_graph(oracle_mod, tmp_path):
    """graph_create -> autotune -> graph_launch: the graph baked in the old
    tiling, so the launch is refused (BX_E_STATE); a new capture runs and
    matches the oracle.  A second plan of the same shape class reuses the
    tuned choice (in-process and through the cache file) and also matches."""
    import torch
    cache = str(tmp_path / "tune.txt")
    insts = [synth.grid_wcsp(7, rows=10, cols=10), synth.grid_wcsp(8, rows=10, cols=10)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = bx.Plan([bx.Problem.from_instance(insts[0])], algo="mbe", ibound=8, tune_cache=cache)
        plan.upload(s)
        plan.graph_create("level", s)
        plan.autotune(reps=1, stream=s)
        with pytest.raises(bx.BxError) as e:
            plan.graph_launch(s)
        assert e.value.status == -6
        plan.graph_create("auto", s)
        plan.graph_launch(s)
        res = oracle_mod.solve(insts[0], plan.order(0), 8)
        _check_int(plan, 0, insts[0], res)
        assert "cached=0" in plan.describe()
        # same shape class, other costs: the stored choice, no timing
        other = bx.Plan([bx.Problem.from_instance(insts[1])], algo="mbe", ibound=8, tune_cache=cache)
        other.upload(s)
        other.autotune(reps=1, stream=s)
        assert "cached=1" in other.describe()
        other.execute(stream=s)
        res1 = oracle_mod.solve(insts[1], other.order(0), 8)
        _check_int(other, 0, insts[1], res1)
    assert open(cache).read().startswith("bxtune2 ")


@pytest.mark.parametrize("D,ibound", [(12, 4), (16, 4), (25, 4), (33, 3), (100, 3)])
def test_large_domains_lane_groups(oracle_mod, D, ibound):
    """Eliminated domains above the tiled path's (the paper's random networks
    use d up to 100, Sec. 8.1): lane groups share one row's values and reduce
    their minima by lane exchanges.  Every UTIL table, the bound, the cost and
    the assignment bit for bit; infinite entries included."""
    insts = []
    for s in range(3):
        rng = np.random.default_rng(1000 * D + s)
        n = 7
        doms = np.full(n, D, np.int32)
        doms[rng.integers(0, n)] = max(2, D // 3)       # one smaller domain
        edges = synth.gnm_edges(rng, n, 9)
        insts.append(synth.wcsp_from_edges(rng, doms, edges, 0, 100, tightness=0.2))
    # unpacked (every mini-bucket on its own tiles: the lane-group path), and
    # packed (the small ones one row per thread)
    for packing in (False, True):
        plan = _run(insts, "mbe", ibound, packing=packing)
        lanes = sum(plan.level_info(lv).n_lane_tiles for lv in range(plan.stats().n_levels))
        assert lanes > 0 or packing
        for k, inst in enumerate(insts):
            _check_int(plan, k, inst, oracle_mod.solve(inst, plan.order(k), ibound))


def test_large_domain_float_lane_groups(oracle_mod):
    """FP32 costs (-ln p of a belief network with 20-valued variables) on the
    lane-group path: tables within 1e-5 relative of the FP64 oracle."""
    inst = synth.tiny_bayes_net(5, n=6, n_parents=2, d_hi=20)     # domains 2..17
    plan = _run([inst], "be", 0, packing=False)
    assert sum(plan.level_info(lv).n_lane_tiles for lv in range(plan.stats().n_levels)) > 0
    res = oracle_mod.solve(inst, plan.order(0), 0)
    b, u, a = plan.results(0)
    assert abs(b - res.lb) <= 1e-5 * abs(res.lb)
    _check_tables(plan, 0, res, exact=False, rtol=1e-5)


@pytest.mark.parametrize("seed", range(4))
def test_random_problems_and_options(oracle_mod, seed):
    """Random problems (domains 2-6, arities 1-3, several copies per plan)
    under MBE at random i-bounds, BE and DPOP, with random packing limits and
    flags (no blocking, XCD order, forced non-temporal stores and staging),
    each executed once: bound, cost, assignment and every table bit for bit
    against the oracle."""
    rng = np.random.default_rng(5000 + seed)
    for k in range(6):
        n = int(rng.integers(6, 30))
        doms = rng.integers(2, 7, size=n).astype(np.int32)
        scopes, tables = [], []
        for _ in range(int(rng.integers(n, 3 * n))):
            ar = int(rng.integers(1, 4))
            sc = np.sort(rng.choice(n, size=ar, replace=False)).astype(np.int32)
            scopes.append(sc)
            tables.append(rng.integers(0, 100, size=int(np.prod(doms[sc]))).astype(np.int32))
        inst = synth.Instance(domains=doms, scopes=scopes, tables=tables, kind="cost_i32")
        algo = ["mbe", "be", "dpop"][k % 3]
        ib = int(rng.integers(2, 8)) if algo == "mbe" else 0
        flags = int(rng.choice([0, bx.FLAG_NO_BLOCKING, bx.FLAG_XCD_ORDER, bx.FLAG_FORCE_NT | bx.FLAG_STAGE_ALWAYS]))
        pack = None if rng.random() < 0.5 else dict(pack_max_rows=int(rng.choice([16, 64, 256, 1024])),
                                                   fuse_max_rows=int(rng.choice([64, 1024, 4096])),
                                                   fuse_max_stages=int(rng.integers(1, 6)))
        copies = int(rng.integers(1, 4))
        try:
            plan = bx.Plan([bx.Problem.from_instance(inst)] * copies, algo=algo, ibound=ib, flags=flags, pack=pack,
                           packing=bool(rng.random() < 0.8))
        except bx.BxError as e:   # a table above the size limit
            assert "large" in str(e) or "limit" in str(e), str(e)
            continue
        plan.upload()
        plan.execute()
        for c in range(copies):
            res = oracle_mod.solve(inst, plan.order(c), ib, keep_tables=True)
            _check_int(plan, c, inst, res)
