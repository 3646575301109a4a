"""Host-side checks of the C-ABI library (no device calls): it loads, it
exports every entry point include/bx.h declares, and the planner's host
logic (orders, buckets, partitions, message scopes, validation) agrees with
the CPU oracle, which is written separately."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"typedef[^;]*;", "", txt)
        names |= set(re.findall(r"\b(bx_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = bx.lib()
    declared = _declared()
    assert len(declared) >= 25
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(bx.EXPORTS) <= declared
    assert b"gfx950" in L.bx_version()


def test_options_default():
    o = bx.Options()
    bx.lib().bx_options_default(ctypes.byref(o))
    assert o.algo == 0 and o.order == bx.ORDER["min-fill"] and o.schedule == bx.SCHED["auto"]


@pytest.mark.parametrize("heur", ["min-degree", "min-fill", "dfs", "degree-sort"])
def test_orders_match_oracle(oracle_mod, heur):
    for seed in range(25):
        inst = synth.batch_candidate(seed, n_lo=20, n_hi=60)
        p = bx.Problem.from_instance(inst)
        o, par = p.compute_order(heur)
        eo, epar = oracle_mod.order(inst, heur)
        assert o.tolist() == eo.tolist(), (seed, heur)
        if heur == "dfs":
            assert par.tolist() == epar.tolist()
        assert p.induced_width(o) == oracle_mod.induced_width(inst, o)


def test_grid_order_matches_oracle(oracle_mod):
    inst = synth.grid_wcsp(0, rows=12, cols=12)
    p = bx.Problem.from_instance(inst)
    o, _ = p.compute_order("min-fill")
    eo, _ = oracle_mod.order(inst, "min-fill")
    assert o.tolist() == eo.tolist()


@pytest.mark.parametrize("heur", ["min-fill", "min-degree"])
def test_large_orders_match_oracle(oracle_mod, heur):
    """The library updates the greedy scores incrementally (only the
    eliminated vertex's neighbours are rescored, and a fill edge lowers the
    fill of the common neighbours of its ends); the oracle rescores every
    vertex at every step.  Same orders, ties included, on a 625-variable grid
    and on scale-free graphs (hubs: many fill edges per step)."""
    for inst in [synth.grid_wcsp(0, rows=25, cols=25, d=2)] + [synth.scale_free_wcsp(s, n=120) for s in range(3)]:
        p = bx.Problem.from_instance(inst)
        o, _ = p.compute_order(heur)
        eo, _ = oracle_mod.order(inst, heur)
        assert o.tolist() == eo.tolist()


def _structure_equal(plan, prob, res):
    mbs = plan.minibuckets(prob)
    assert len(mbs) == len(res.minibuckets)
    for a, b in zip(mbs, res.minibuckets):
        assert a.var == b.var
        assert sorted(a.members) == sorted(b.members)
        assert a.out_id == b.out_id
        assert a.out_scope.tolist() == b.out_scope.tolist()


@pytest.mark.parametrize("ibound", [0, 2, 3, 5])
def test_plan_structure_matches_oracle(oracle_mod, ibound):
    for seed in range(30):
        inst = synth.tiny_random(seed, n_lo=3, n_hi=9, m_lo=3, m_hi=14)
        p = bx.Problem.from_instance(inst)
        algo = "mbe" if ibound else "be"
        plan = bx.Plan([p], algo=algo, ibound=ibound, order="min-fill")
        eo, _ = oracle_mod.order(inst, "min-fill")
        assert plan.order(0).tolist() == eo.tolist()
        res = oracle_mod.solve(inst, eo, ibound)
        _structure_equal(plan, 0, res)


def test_grid_mbe_structure_matches_oracle(oracle_mod):
    inst = synth.grid_wcsp(0, rows=8, cols=8)
    p = bx.Problem.from_instance(inst)
    plan = bx.Plan([p], algo="mbe", ibound=6, order="min-fill")
    eo, _ = oracle_mod.order(inst, "min-fill")
    res = oracle_mod.solve(inst, eo, 6, keep_tables=False)
    _structure_equal(plan, 0, res)
    st = plan.stats()
    assert st.n_minibuckets == len(res.minibuckets)
    assert st.max_scope == res.max_union


def test_batched_plan_structure(oracle_mod):
    insts = [synth.batch_candidate(s, n_lo=20, n_hi=40) for s in range(6)]
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=5)
    for k, inst in enumerate(insts):
        eo, _ = oracle_mod.order(inst, "min-fill")
        _structure_equal(plan, k, oracle_mod.solve(inst, eo, 5, keep_tables=False))


def test_dpop_plan_checks_separators(oracle_mod):
    inst = synth.dcop_candidate(3, n=14, density=0.3, d=2)
    p = bx.Problem.from_instance(inst)
    plan = bx.Plan([p], algo="dpop")
    o, par = oracle_mod.order(inst, "dfs")
    assert plan.order(0).tolist() == o.tolist()
    seps = oracle_mod.separators(inst, par)
    for mb in plan.minibuckets(0):
        assert sorted(mb.out_scope.tolist()) == seps[mb.var]


def test_dpop_user_pseudotree_and_rejection():
    g = {"functions": [[0, 1], [0, 3], [1, 2], [1, 3], [2, 3]]}
    inst = synth.Instance(domains=np.full(4, 2, np.int32),
                          scopes=[np.array(s, np.int32) for s in g["functions"]],
                          tables=[np.arange(4, dtype=np.int32) for _ in g["functions"]])
    p = bx.Problem.from_instance(inst)
    p.set_pseudotree([-1, 0, 1, 2])
    plan = bx.Plan([p], algo="dpop")
    assert plan.order(0).tolist() == [0, 1, 2, 3]
    assert plan.minibuckets(0)[0].out_scope.tolist() == [0, 1, 2]
    # x2 and x4 (ids 1, 3) share a function but sit on different branches
    p2 = bx.Problem.from_instance(inst)
    p2.set_pseudotree([-1, 0, 1, 0])
    with pytest.raises(bx.BxError) as e:
        bx.Plan([p2], algo="dpop")
    assert e.value.status == -1


def test_invalid_inputs_rejected():
    p = bx.Problem([2, 3])
    with pytest.raises(bx.BxError):
        p.add_function([0, 0], np.zeros(4, np.int32))            # repeated variable
    with pytest.raises(bx.BxError):
        p.add_function([0, 2], np.zeros(6, np.int32))            # out of range
    with pytest.raises(bx.BxError):
        p.add_function([0, 1], np.zeros(5, np.int32))            # wrong size
    with pytest.raises(bx.BxError):
        p.add_function([1], np.array([1, -1, 2], np.int32))      # negative cost
    with pytest.raises(bx.BxError):
        p.set_order([0, 0])
    with pytest.raises(bx.BxError):
        bx.Problem([2, 0])
    pf = bx.Problem([2], cost="f32")
    with pytest.raises(bx.BxError):
        pf.add_function([0], np.array([0.5, np.nan], np.float32))
    with pytest.raises(bx.BxError):
        pf.add_prob_table([0], np.array([0.5, 1.5]))
    p.add_function([0, 1], np.zeros(6, np.int32))
    with pytest.raises(bx.BxError):
        bx.Plan([p], algo="mbe", ibound=0)


def test_size_limit_reports_too_large():
    inst = synth.random_wcsp(0, n=12, m_edges=40, d=3)
    p = bx.Problem.from_instance(inst)
    with pytest.raises(bx.BxError) as e:
        bx.Plan([p], algo="be", max_table_entries=100)
    assert e.value.status == -3


def test_plan_stats_match_oracle_sizes(oracle_mod):
    inst = synth.grid_wcsp(1, rows=10, cols=10)
    plan = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=8)
    eo, _ = oracle_mod.order(inst, "min-fill")
    res = oracle_mod.solve(inst, eo, 8)
    st = plan.stats()
    rows = sum(mb.table.size for mb in res.minibuckets)
    joint = sum(mb.table.size * int(inst.domains[mb.var]) for mb in res.minibuckets)
    assert st.util_rows == rows and st.joint_entries == joint
    assert plan.workspace_bytes() > 4 * rows


def test_dataflow_schedule_is_refused_before_any_device_call():
    # the persistent dataflow schedule is disabled: the call must fail with
    # BX_E_UNSUPPORTED before it touches the (here fake) workspace
    inst = synth.random_wcsp(0)
    plan = bx.Plan([bx.Problem.from_instance(inst)])
    rc = bx.lib().bx_plan_execute_sched(plan._h, ctypes.c_void_p(256), plan.workspace_bytes(),
                                        bx.SCHED["dataflow"], None)
    assert rc == -5


def test_results_before_execute_is_state_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only check")
    inst = synth.random_wcsp(0)
    plan = bx.Plan([bx.Problem.from_instance(inst)])
    b = ctypes.c_double()
    rc = bx.lib().bx_plan_results(plan._h, ctypes.c_void_p(256), 0, ctypes.byref(b), None, None, None)
    assert rc == -6


def test_one_hip_runtime_in_the_process():
    """Loading the library before anything imports torch must still leave one
    HIP runtime in the process (torch's), so that torch's device memory and
    streams are valid for the library."""
    import subprocess
    import sys
    code = ("import paper_1608_05288_amd as bx; bx.lib(); import torch;"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l};"
            "print(len(libs))")
    out = subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, text=True)
    assert out.strip() == "1"


def test_tile_region_holds_every_tiling():
    """The workspace reserves room for the largest tile list of any tiling
    the tuner may pick; tiles of mixed-domain mini-buckets are boxes whose
    count is not that of a fixed number of rows per tile."""
    for seed in range(6):
        insts = [synth.batch_candidate(seed * 50 + s, n_lo=30, n_hi=60) for s in range(8)]
        for ib in (6, 10):
            plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=ib)
            st = plan.stats()
            assert 0 < st.n_tiles <= st.tile_capacity
    grid = bx.Plan([bx.Problem.from_instance(synth.grid_wcsp(0, rows=10, cols=10))], algo="mbe", ibound=8)
    assert grid.stats().n_tiles <= grid.stats().tile_capacity


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_register_blocking_flag():
    """Blocking is a planner choice: on by default where the scopes allow it,
    off with BX_FLAG_NO_BLOCKING; the plan's sizes do not depend on it and
    unknown flag bits are rejected."""
    import re
    inst = synth.grid_wcsp(0, rows=10, cols=10)

    def blocked(plan):
        return int(re.search(r"blocked_minibuckets=(\d+)", plan.describe()).group(1))
    on = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=9)
    off = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=9, blocking=False)
    assert blocked(on) > 0 and blocked(off) == 0
    a, b = on.stats(), off.stats()
    assert (a.util_rows, a.algo_bytes, a.n_minibuckets) == (b.util_rows, b.algo_bytes, b.n_minibuckets)
    assert "tile_goals=" in on.describe()
    L = bx.lib()
    opt = bx.Options()
    L.bx_options_default(ctypes.byref(opt))
    opt.algo, opt.ibound, opt.flags = 1, 4, 0x80
    p = bx.Problem.from_instance(synth.random_wcsp(0))
    arr = (ctypes.c_void_p * 1)(p.handle.value)
    h = ctypes.c_void_p()
    assert L.bx_plan_create(arr, 1, ctypes.byref(opt), ctypes.byref(h)) == -1   # BX_E_INVALID
    assert b"flags" in L.bx_last_error()


def test_store_and_staging_flags_and_level_info():
    """The forcing flags are accepted and show in the per-level description;
    per-level rows and bytes add up to the plan's totals; per-level timing is
    a state error before any timed execute."""
    inst = synth.grid_wcsp(1, rows=8, cols=8)
    for flags, st, nt in ((bx.FLAG_FORCE_NT, None, 1), (bx.FLAG_STAGE_ALWAYS, 1, None),
                          (bx.FLAG_STAGE_NEVER, 0, None), (bx.FLAG_STAGE_ALWAYS | bx.FLAG_STAGE_NEVER, 1, None)):
        plan = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=7, flags=flags)
        s = plan.stats()
        rows = byts = tiles = mbs = 0
        for lv in range(s.n_levels):
            li = plan.level_info(lv)
            rows += li.util_rows
            byts += li.algo_bytes
            tiles += li.n_tiles
            mbs += li.n_minibuckets
            assert 0 <= li.n_row_tiles <= li.n_tiles
            if st is not None:
                assert li.staged == st
            if nt is not None:
                assert li.nontemporal == nt
        assert (rows, byts, tiles, mbs) == (s.util_rows, s.algo_bytes, s.n_tiles, s.n_minibuckets)
        with pytest.raises(bx.BxError) as e:
            plan.level_timing()
        assert e.value.status == -6
    with pytest.raises(bx.BxError):
        bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=7).level_info(10_000)


def test_tune_cache_option_is_copied(tmp_path):
    """The cache path is copied at planning time (the caller's string may go
    away); planning never touches the file."""
    path = str(tmp_path / "tune.txt")
    plan = bx.Plan([bx.Problem.from_instance(synth.random_wcsp(0))], algo="mbe", ibound=4, tune_cache=path)
    plan._tune_cache = None
    import gc
    gc.collect()
    assert "schedule=" in plan.describe()
    assert not os.path.exists(path)


def _dcop(n, edges, parent):
    p = bx.Problem([2] * n)
    for a, b in edges:
        p.add_function([a, b], np.arange(4, dtype=np.int32))
    p.set_pseudotree(parent)
    return p


def test_simulated_runtime_chain_and_star():
    """Simulated runtime (Sec. 8's DCOP metric) against hand-worked critical
    paths.  Chain 0-1-2-3 rooted at 0: UTIL = t3 + L + t2 + L + t1 + L + t0,
    and three VALUE hops.  Star with root 0 and leaves 1-3: UTIL = max of the
    leaves + L + t0, one VALUE hop.  A missing timed execute is a state error."""
    L = 0.5
    t = {0: 1.0, 1: 2.0, 2: 4.0, 3: 8.0}
    for algo in ("dpop", "adpop"):
        chain = bx.Plan([_dcop(4, [(0, 1), (1, 2), (2, 3)], [-1, 0, 1, 2])], algo=algo, ibound=2)
        ms = [t[mb.var] for mb in chain.minibuckets(0)]
        u, v, h = chain.simulated_runtime(0, ms, L)
        assert u == pytest.approx(8 + L + 4 + L + 2 + L + 1)
        assert v == pytest.approx(3 * L) and h == 3
        star = bx.Plan([_dcop(4, [(0, 1), (0, 2), (0, 3)], [-1, 0, 0, 0])], algo=algo, ibound=2)
        ms = [t[mb.var] for mb in star.minibuckets(0)]
        u, v, h = star.simulated_runtime(0, ms, L)
        assert u == pytest.approx(8 + L + 1)
        assert v == pytest.approx(L) and h == 1
    with pytest.raises(bx.BxError):
        star.simulated_runtime(0)
    with pytest.raises(bx.BxError):
        star.simulated_runtime(0, [1.0] * len(star.minibuckets(0)), -1.0)


def test_adpop_bounds_message_scopes(oracle_mod):
    """ADPOP (Sec. 4.2) plans MBE along the DFS pseudo-tree order: the
    library's order is the oracle's DFS order, mini-buckets and their output
    scopes equal the oracle's MBE run along it, and every message stays
    within the i-bound; with the bound at the largest separator + 1 it is
    DPOP itself (one mini-bucket per agent, scope = separator)."""
    from paper_1608_05288_amd import synth
    for seed in range(4):
        inst = synth.dcop_candidate(seed, n=14, density=0.3, d=3)
        o, par = oracle_mod.order(inst, "dfs")
        seps = oracle_mod.separators(inst, par)
        for ib in (2, 3, 4):
            plan = bx.Plan([bx.Problem.from_instance(inst)], algo="adpop", ibound=ib)
            assert plan.order(0).tolist() == o.tolist()
            res = oracle_mod.solve(inst, o, ib, keep_tables=False)
            mbs = plan.minibuckets(0)
            assert [(m.var, m.out_scope.tolist()) for m in mbs] == \
                [(m.var, m.out_scope.tolist()) for m in res.minibuckets]
            assert max(len(m.out_scope) for m in mbs) <= ib - 1
        full = bx.Plan([bx.Problem.from_instance(inst)], algo="adpop", ibound=max(len(s) for s in seps) + 1)
        for m in full.minibuckets(0):
            assert sorted(m.out_scope.tolist()) == seps[m.var]


@pytest.mark.parametrize("name", ["grid", "batch", "bn", "tiny", "dcop"])
def test_packed_schedule_is_valid_and_shorter(name):
    """Packing small mini-buckets (several per workgroup, connected parts of
    the bucket tree fused stage by stage): the library's own schedule check
    passes with packing on and off (every mini-bucket computed once, each
    after its producers, packed stages consistent), packing never adds a
    dependency level and removes some on every family here, and the plan's
    mini-buckets are the same either way."""
    cases = {"grid": ([synth.grid_wcsp(0)], dict(algo="mbe", ibound=12)),
             "batch": ([synth.batch_candidate(s) for s in range(32)], dict(algo="mbe", ibound=10)),
             "bn": ([synth.bayes_net(s) for s in range(2)], dict(algo="mbe", ibound=20)),
             "tiny": ([synth.tiny_random(s) for s in range(40)], dict(algo="mbe", ibound=2)),
             "dcop": ([synth.dcop_candidate(3, n=14, density=0.3, d=3)], dict(algo="dpop"))}
    insts, kw = cases[name]
    on = bx.Plan([bx.Problem.from_instance(i) for i in insts], packing=True, **kw)
    off = bx.Plan([bx.Problem.from_instance(i) for i in insts], packing=False, **kw)
    on.validate()
    off.validate()
    n_on, n_off = on.stats().n_levels, off.stats().n_levels
    assert n_on < n_off
    assert sum(on.level_info(l).n_packed for l in range(n_on)) > 0
    assert sum(off.level_info(l).n_packed for l in range(n_off)) == 0
    for k in range(len(insts)):
        a, b = on.minibuckets(k), off.minibuckets(k)
        assert [(m.var, m.out_scope.tolist()) for m in a] == [(m.var, m.out_scope.tolist()) for m in b]


def test_sum_product_plans(oracle_mod):
    """The sum-product algorithms need float costs; their mini-buckets are
    those of the min-sum plan (the same partition rule)."""
    with pytest.raises(bx.BxError) as e:
        bx.Plan([bx.Problem.from_instance(synth.random_wcsp(0))], algo="be-sum")
    assert e.value.status == -5
    inst = synth.bayes_net(1)
    a = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe-sum", ibound=12)
    b = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=12)
    a.validate()
    res = oracle_mod.solve(inst, a.order(0), 12, keep_tables=False, semiring="sum")
    assert [(m.var, m.out_scope.tolist()) for m in a.minibuckets(0)] == \
        [(m.var, m.out_scope.tolist()) for m in b.minibuckets(0)] == \
        [(m.var, m.out_scope.tolist()) for m in res.minibuckets]


def test_bnb_rejects_float_costs_and_bad_arguments():
    """Branch and bound takes integer costs; argument errors come back
    before any device work (the pointer below is never dereferenced)."""
    L = bx.lib()
    opt = bx.Options()
    L.bx_options_default(ctypes.byref(opt))
    opt.algo = bx.ALGO["mbe"]
    opt.ibound = 2
    val = ctypes.c_double()
    asg = np.zeros(4, np.int32)
    st = (ctypes.c_int64 * 4)()
    pf = bx.Problem([2, 2], "f32")
    rc = L.bx_bnb_solve(pf.handle, ctypes.byref(opt), ctypes.c_void_p(256), 1 << 20, None, 0,
                        ctypes.byref(val), asg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), st)
    assert rc == -5
    pi = bx.Problem([2, 2], "i32")
    rc = L.bx_bnb_solve(pi.handle, ctypes.byref(opt), ctypes.c_void_p(100), 1 << 20, None, 0,
                        ctypes.byref(val), asg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), st)
    assert rc == -1      # unaligned workspace
    nb = ctypes.c_size_t()
    pi.add_function([0, 1], np.arange(4, dtype=np.int32))
    assert L.bx_bnb_workspace_bytes(pi.handle, ctypes.byref(opt), ctypes.byref(nb)) == 0 and nb.value > 0


def test_streamed_execution_needs_an_unblocked_plan():
    inst = synth.grid_wcsp(0, rows=6, cols=6)
    blocked = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=6)
    plain = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=6, blocking=False)
    if "blocked_minibuckets=0" not in blocked.describe():
        with pytest.raises(bx.BxError) as e:
            blocked.stream_bytes(4096)
        assert e.value.status == -5
    d, h = plain.stream_bytes(4096)
    assert 0 < d and 0 < h
    with pytest.raises(bx.BxError):
        plain.stream_bytes(100)          # chunks below 256 rows


def test_xcd_order_flag():
    """FLAG_XCD_ORDER is accepted and puts every level in XCD order (the
    plan's description counts them); without it no level is, until tuned;
    a flag bit beyond the known ones is refused."""
    inst = synth.grid_wcsp(1, rows=8, cols=8)
    plan = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=7, flags=bx.FLAG_XCD_ORDER)
    assert f"xcd_levels={plan.stats().n_levels} " in plan.describe()
    plain = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=7)
    assert "xcd_levels=0 " in plain.describe()
    with pytest.raises(bx.BxError):
        bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=7, flags=0x40)


@pytest.mark.parametrize("seed", range(6))
def test_random_plans_pass_the_schedule_check(seed):
    """Plans of random problems (mixed domains 2-6 and arities, MBE at random
    i-bounds, BE, DPOP) under random packing limits and flags pass the
    planner's own schedule check (tile ranges, segment records, levels,
    register-blocked box shapes), and their per-level rows and bytes add up to
    the plan's totals."""
    rng = np.random.default_rng(4000 + seed)
    for k in range(8):
        n = int(rng.integers(6, 40))
        doms = rng.integers(2, 7, size=n).astype(np.int32)
        scopes, tables = [], []
        for _ in range(int(rng.integers(n, 3 * n))):
            ar = int(rng.integers(1, 4))
            sc = np.sort(rng.choice(n, size=ar, replace=False)).astype(np.int32)
            scopes.append(sc)
            tables.append(rng.integers(0, 100, size=int(np.prod(doms[sc]))).astype(np.int32))
        inst = synth.Instance(domains=doms, scopes=scopes, tables=tables, kind="cost_i32")
        algo = ["mbe", "be", "dpop"][k % 3]
        ib = int(rng.integers(2, 9)) if algo == "mbe" else 0
        flags = int(rng.choice([0, bx.FLAG_NO_BLOCKING, bx.FLAG_XCD_ORDER, bx.FLAG_FORCE_NT | bx.FLAG_STAGE_ALWAYS]))
        pack = None if rng.random() < 0.5 else dict(pack_max_rows=int(rng.choice([16, 64, 256, 1024])),
                                                   fuse_max_rows=int(rng.choice([64, 1024, 4096])),
                                                   fuse_max_stages=int(rng.integers(1, 6)))
        try:
            plan = bx.Plan([bx.Problem.from_instance(inst)] * int(rng.integers(1, 4)), algo=algo, ibound=ib,
                           flags=flags, pack=pack, packing=bool(rng.random() < 0.8))
        except bx.BxError as e:   # a table above the size limit is refused, nothing else
            assert "large" in str(e) or "limit" in str(e), str(e)
            continue
        plan.validate()
        s = plan.stats()
        rows = byts = 0
        for lv in range(s.n_levels):
            li = plan.level_info(lv)
            rows += li.util_rows
            byts += li.algo_bytes
        assert (rows, byts) == (s.util_rows, s.algo_bytes)
