"""Pins of the sampled candidate value (oracle/candidates.py): a hand-worked
bucket, the split inequality of Sec. 2.2 on every sample, and the exact
average over all assignments when the samples enumerate them."""
import itertools

import numpy as np

from oracle import candidates
from paper_1608_05288_amd import synth


def _bucket():
    # x = 2 (domain 2) with f(a=0, x) and g(b=1, x); domains 2, 3, 2
    inst = synth.Instance(domains=np.array([2, 3, 2], np.int32),
                          scopes=[[0, 2], [1, 2]],
                          tables=[np.array([[1, 5], [4, 0]], np.int32),
                                  np.array([[0, 3], [2, 2], [7, 1]], np.int32)],
                          kind="cost_i32")
    return inst, candidates.function_tables(inst, type("R", (), {"minibuckets": []})())


def test_hand_worked_bucket():
    inst, tabs = _bucket()
    # all six (a, b) once: slot 0 = a (mod 2), slot 1 = b (mod 3)
    rnd = np.array([[a, b] + [0] * 30 for a in range(2) for b in range(3)], np.uint32)
    # together: min_x f(a,x)+g(b,x); a=0: rows (1,5): b0 (1,8)->1, b1 (3,7)->3, b2 (8,6)->6
    #                                  a=1: rows (4,0): b0 (4,3)->3, b1 (6,2)->2, b2 (11,1)->1
    assert candidates.candidate_value(inst, tabs, 2, [0, 1], [0, 0], rnd) == (1 + 3 + 6 + 3 + 2 + 1) / 6
    # split: min_x f + min_x g = (1 or 0) + (0, 2, 1)
    split = ((1 + 0) + (1 + 2) + (1 + 1) + (0 + 0) + (0 + 2) + (0 + 1)) / 6
    assert candidates.candidate_value(inst, tabs, 2, [0, 1], [0, 1], rnd) == split


def test_split_never_exceeds_the_whole_bucket():
    rng = np.random.default_rng(3)
    for seed in range(40):
        inst = synth.tiny_random(seed, n_lo=3, n_hi=6, d_lo=2, d_hi=3, m_lo=3, m_hi=7)
        tabs = candidates.function_tables(inst, type("R", (), {"minibuckets": []})())
        x = int(inst.n - 1)
        fns = [i for i, s in enumerate(inst.scopes) if x in [int(v) for v in s]]
        if len(fns) < 2:
            continue
        parts = rng.integers(0, len(fns), len(fns))
        for s in range(5):
            rnd = rng.integers(0, 2**32, (1, 32), dtype=np.uint64).astype(np.uint32)
            whole = candidates.candidate_value(inst, tabs, x, fns, [0] * len(fns), rnd)
            split = candidates.candidate_value(inst, tabs, x, fns, parts.tolist(), rnd)
            assert split <= whole


def test_enumerating_samples_gives_the_exact_average():
    inst = synth.tiny_random(7, n_lo=4, n_hi=4, d_lo=2, d_hi=3, m_lo=5, m_hi=6)
    tabs = candidates.function_tables(inst, type("R", (), {"minibuckets": []})())
    x = 3
    fns = [i for i, s in enumerate(inst.scopes) if x in [int(v) for v in s]] or [0]
    others = sorted({int(u) for f in fns for u in inst.scopes[f] if int(u) != x})
    combos = list(itertools.product(*[range(int(inst.domains[u])) for u in others]))
    rnd = np.zeros((len(combos), 32), np.uint32)
    for i, c in enumerate(combos):
        rnd[i, :len(c)] = c
    got = candidates.candidate_value(inst, tabs, x, fns, [0] * len(fns), rnd)
    # the exact average over all assignments of the other variables, by brute force
    exact = 0.0
    for c in combos:
        a = dict(zip(others, c))
        best = None
        for v in range(int(inst.domains[x])):
            a[x] = v
            s = sum(int(np.asarray(inst.tables[f]).reshape([int(inst.domains[u]) for u in inst.scopes[f]])
                        [tuple(a[int(u)] for u in inst.scopes[f])]) for f in fns)
            s = min(s, 2**31 - 1)
            best = s if best is None else min(best, s)
        exact += best
    assert got == exact / len(combos)
