"""Sampled candidate values of bucket partitions -- TEST INFRASTRUCTURE ONLY.

For the bucket of variable x, a partition {Q_k} of its functions and samples s
of the bucket's other variables,
    value = (1/S) sum_s sum_k min_x sum_{f in Q_k} f(s, x),
the part of the mini-bucket bound (Alg. 2; Sec. 2.2: a split keeps
sum_k min <= min sum) the partition keeps at that bucket.  The digit of
variable u in sample s is rnd[s][slot(u)] mod |D_u|, slot(u) being the rank of
u among the bucket's variables other than x in increasing id.  Integer sums
saturate at INF = 2^31 - 1 (Sec. 2), the sum over the parts included.

Function values are read from the oracle's own tables: the instance's inputs
and the mini-bucket outputs of oracle.solve run with the same partitions.
"""
from __future__ import annotations

import numpy as np

INF_I32 = 2**31 - 1


def function_tables(inst, res):
    """{function id: (scope, table shaped by the scope's domains)} for the
    instance's inputs (ids 0..m-1) and the outputs of `res` (by out_id)."""
    out = {}
    for i, (sc, t) in enumerate(zip(inst.scopes, inst.tables)):
        sc = [int(v) for v in sc]
        out[i] = (sc, np.asarray(t).reshape([int(inst.domains[v]) for v in sc]) if sc else np.asarray(t).reshape(()))
    for mb in res.minibuckets:
        if mb.out_id >= 0:
            sc = [int(v) for v in mb.out_scope]
            out[mb.out_id] = (sc, mb.table.reshape([int(inst.domains[v]) for v in sc]) if sc else mb.table.reshape(()))
    return out


def _value_at(fn, assign):
    sc, t = fn
    return t[tuple(assign[v] for v in sc)] if sc else t[()]


def candidate_value(inst, tables, x, fn_ids, part_of_fn, rnd, integer=True) -> float:
    """Mean over the samples (rows of rnd) of sum_k min_x sum_{f in part k} f."""
    others = sorted({int(u) for f in fn_ids for u in tables[f][0] if int(u) != x})
    total = 0.0
    for s in range(rnd.shape[0]):
        assign = {u: int(rnd[s][j]) % int(inst.domains[u]) for j, u in enumerate(others)}
        tot = 0.0
        for k in sorted(set(int(p) for p in part_of_fn)):
            best = None
            for v in range(int(inst.domains[x])):
                assign[x] = v
                acc = 0
                for f, p in zip(fn_ids, part_of_fn):
                    if p == k:
                        acc += _value_at(tables[f], assign).item()
                if integer:
                    acc = min(int(acc), INF_I32)
                best = acc if best is None or acc < best else best
            tot += float(best)
        if integer:
            tot = min(tot, float(INF_I32))     # the parts' outputs meet again in a saturating sum
        total += tot
    return total / rnd.shape[0]
