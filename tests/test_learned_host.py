"""Host-side checks of the partition decisions (no device calls): whatever a
chooser picks, every mini-bucket respects the i-bound and the buckets are
partitioned exactly, as the independently written oracle confirms by
re-running MBE with the same partitions (Alg. 2: any partition whose
mini-buckets respect the bound gives a valid lower bound)."""
import numpy as np
import pytest

import paper_1608_05288_amd as bx
from paper_1608_05288_amd import synth

NF = 32


def _family(count, seed0=500):
    def ok(inst):
        p = bx.Problem.from_instance(inst)
        o, _ = p.compute_order("min-fill")
        return 8 <= p.induced_width(o) <= 16
    return synth.accepted(synth.batch_candidate, count, seed0, accept=ok)


def _parts(plan, prob):
    parts = {}
    for mb in plan.minibuckets(prob):
        parts.setdefault(mb.var, []).append(list(mb.members))
    return parts


def _structure_equal(plan, prob, res):
    mbs = plan.minibuckets(prob)
    assert len(mbs) == len(res.minibuckets)
    for a, b in zip(mbs, res.minibuckets):
        assert a.var == b.var
        assert sorted(a.members) == sorted(b.members)
        assert a.out_id == b.out_id
        assert a.out_scope.tolist() == b.out_scope.tolist()


def test_feature_count():
    assert bx.partition_num_features() == NF


def test_greedy_choice_reproduces_greedy_plan():
    insts = _family(6)
    probs = [bx.Problem.from_instance(i) for i in insts]
    seen = []

    def zero(n, dec_prob, off, feats):
        seen.append(n)
        return np.zeros(n, np.int32)
    a = bx.Plan(probs, algo="mbe", ibound=8, chooser=zero)
    b = bx.Plan(probs, algo="mbe", ibound=8)
    assert sum(seen) > 0
    d, ng = a.partition_stats()
    assert d == sum(seen) and ng == 0
    for k in range(len(probs)):
        ma, mb_ = a.minibuckets(k), b.minibuckets(k)
        assert [(m.var, m.members, m.out_id, m.out_scope.tolist()) for m in ma] == \
               [(m.var, m.members, m.out_id, m.out_scope.tolist()) for m in mb_]


@pytest.mark.parametrize("ibound", [4, 6, 9])
def test_any_choice_is_a_valid_partition(oracle_mod, ibound):
    insts = _family(8, seed0=900 + ibound)
    probs = [bx.Problem.from_instance(i) for i in insts]
    rng = np.random.default_rng(ibound)
    taken = []

    def rand(n, dec_prob, off, feats):
        assert feats.shape == (off[-1], NF) and np.isfinite(feats).all()
        assert len(dec_prob) == n and len(set(dec_prob.tolist())) == n   # one decision per problem per round
        ch = np.array([rng.integers(0, off[d + 1] - off[d]) for d in range(n)], np.int32)
        taken.extend(ch.tolist())
        return ch
    plan = bx.Plan(probs, algo="mbe", ibound=ibound, chooser=rand)
    d, ng = plan.partition_stats()
    assert d == len(taken) and ng == sum(c != 0 for c in taken) and ng > 0
    for k, inst in enumerate(insts):
        for mb in plan.minibuckets(k):
            assert len(mb.out_scope) + 1 <= ibound or len(mb.members) == 1
        eo, _ = oracle_mod.order(inst, "min-fill")
        res = oracle_mod.solve(inst, eo, ibound, keep_tables=False, parts=_parts(plan, k))
        _structure_equal(plan, k, res)


def test_candidates_do_not_depend_on_batch_position():
    insts = _family(3, seed0=77)
    rec = {}

    def record(tag):
        def f(n, dec_prob, off, feats):
            for d in range(n):
                rec.setdefault((tag, int(dec_prob[d])), []).append(feats[off[d]:off[d + 1]].copy())
            return np.zeros(n, np.int32)
        return f
    alone = bx.Plan([bx.Problem.from_instance(insts[2])], algo="mbe", ibound=7, chooser=record("a"))
    batch = bx.Plan([bx.Problem.from_instance(i) for i in insts], algo="mbe", ibound=7, chooser=record("b"))
    x, y = rec[("a", 0)], rec[("b", 2)]
    assert len(x) == len(y) > 0
    for u, v in zip(x, y):
        assert np.array_equal(u, v)
    del alone, batch


def test_first_candidate_is_greedy_and_candidates_are_distinct():
    insts = _family(4, seed0=31)
    probs = [bx.Problem.from_instance(i) for i in insts]
    rows = []

    def look(n, dec_prob, off, feats):
        for d in range(n):
            f = feats[off[d]:off[d + 1]]
            rows.append(f)
        return np.zeros(n, np.int32)
    bx.Plan(probs, algo="mbe", ibound=6, chooser=look)
    assert rows
    for f in rows:
        assert f.shape[0] >= 2
        assert f[0, 15] == 0.0                   # generator 0: the greedy rule
        assert np.all(f[:, 3] <= 1.0 + 1e-6)     # largest mini-bucket within the bound
        assert np.all(f[:, 0] > 0) and np.all(f[:, 0] <= 1.0)
        # second half: difference to the greedy candidate
        assert np.array_equal(f[:, 16:], f[:, :16] - f[0, :16]) and not f[0, 16:].any()


def test_no_decision_when_the_bound_covers_the_width():
    inst = _family(1, seed0=3)[0]
    p = bx.Problem.from_instance(inst)
    o, _ = p.compute_order("min-fill")
    w = p.induced_width(o)
    calls = []

    def never(n, dec_prob, off, feats):
        calls.append(n)
        return np.zeros(n, np.int32)
    plan = bx.Plan([p], algo="mbe", ibound=w + 1, chooser=never)
    assert not calls and plan.partition_stats() == (0, 0)


def test_invalid_choice_is_rejected():
    p = bx.Problem.from_instance(_family(1, seed0=11)[0])

    def bad(n, dec_prob, off, feats):
        return np.full(n, 99, np.int32)
    with pytest.raises(bx.BxError) as e:
        bx.Plan([p], algo="mbe", ibound=5, chooser=bad)
    assert e.value.status == -1


def test_chooser_exception_propagates():
    p = bx.Problem.from_instance(_family(1, seed0=12)[0])

    def boom(n, dec_prob, off, feats):
        raise KeyError("from the chooser")
    with pytest.raises(KeyError):
        bx.Plan([p], algo="mbe", ibound=5, chooser=boom)


def test_choose_and_realised_gain_by_hand():
    from paper_1608_05288_amd.learn import choose, realised_gain
    # problem 0 has decisions 0 and 1, problem 1 has decision 2
    pred = np.array([0.0, 0.5, 0.1, 0.2, 0.9, 1.0, 1.05])
    y = np.array([0.0, 1.0, -2.0, 0.0, 3.0, 0.0, -1.0])
    g = np.array([0, 0, 0, 1, 1, 2, 2])
    c = np.array([0, 1, 2, 0, 1, 0, 1])
    p = np.array([0, 0, 0, 0, 0, 1, 1])
    # problem 0: best gain is decision 1 / candidate 1 (+0.7); problem 1: +0.05
    assert choose(pred, g, c, p, 0.0) == {0: 4, 1: 6}
    assert realised_gain(pred, y, g, c, p, 0.0) == (2.0, 2)
    assert choose(pred, g, c, p, 0.1) == {0: 4}
    assert realised_gain(pred, y, g, c, p, 0.1) == (3.0, 1)
    assert realised_gain(pred, y, g, c, p, 0.8) == (0.0, 0)


@pytest.mark.parametrize("ibound", [1, 2, 3])
def test_mixed_arity_choices_match_oracle(oracle_mod, ibound):
    """Mixed arities (0..3) below and at the largest arity: candidates put a
    function wider than the bound in a part of its own (R3); the oracle's
    explicit-partition branch accepts every such choice and builds the same
    mini-buckets."""
    insts = [synth.tiny_random(700 + 13 * ibound + s, n_lo=4, n_hi=9, d_lo=1, d_hi=3, max_arity=3,
                               m_lo=4, m_hi=14) for s in range(40)]
    rng = np.random.default_rng(100 + ibound)
    nongreedy = 0
    for inst in insts:
        def rand(n, dec_prob, off, feats):
            return np.array([rng.integers(0, off[d + 1] - off[d]) for d in range(n)], np.int32)
        plan = bx.Plan([bx.Problem.from_instance(inst)], algo="mbe", ibound=ibound, chooser=rand)
        nongreedy += plan.partition_stats()[1]
        res = oracle_mod.solve(inst, plan.order(0), ibound, keep_tables=False, parts=_parts(plan, 0))
        _structure_equal(plan, 0, res)
    # at i-bound 1 every part is a singleton: there is nothing to choose
    assert nongreedy > 0 or ibound == 1
