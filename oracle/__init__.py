"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The device library never imports it and shares no code
with it.

`bx_oracle.c` is a plain C bucket eliminator (Alg. 1 and Alg. 2 of the paper:
aggregate by summation, eliminate by min-projection, one function and one
table at a time); this module compiles it with gcc and wraps it with ctypes.
`brute.py` holds exhaustive search for tiny instances.

Every function with no independent pin is marked "parity unpinned" in its
docstring; at present every part of the oracle has a pin in
tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bx_oracle.c")
_LIB = os.path.join(_HERE, "libbx_oracle.so")

HEUR = {"min-degree": 0, "min-fill": 1, "dfs": 2, "degree-sort": 3}
INF_I32 = 2**31 - 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, single thread, no vectorisation hints)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.or_solve.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p, i32p, i32p, dp,
                               ctypes.c_int, i32p, ctypes.c_int, ctypes.POINTER(vp)]
        L.or_solve.restype = ctypes.c_int
        L.or_solve_parts.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p, i32p, i32p, dp,
                                     ctypes.c_int, i32p, ctypes.c_int, i32p, ctypes.c_int,
                                     ctypes.POINTER(vp)]
        L.or_solve_parts.restype = ctypes.c_int
        L.or_solve_sum.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p, i32p, dp, ctypes.c_int, i32p,
                                   ctypes.c_int, ctypes.POINTER(vp)]
        L.or_solve_sum.restype = ctypes.c_int
        L.or_order.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int, i32p, i32p]
        L.or_induced_width.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p]
        L.or_separators.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p,
                                    ctypes.POINTER(ctypes.c_uint8)]
        L.or_map_rows.argtypes = [ctypes.c_int, i32p, ctypes.c_int, i32p, ctypes.c_int, i32p, i64p]
        L.or_sat_add.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.or_sat_add.restype = ctypes.c_int32
        L.or_result_lb.argtypes = [vp]
        L.or_result_lb.restype = ctypes.c_double
        L.or_result_ub.argtypes = [vp]
        L.or_result_ub.restype = ctypes.c_double
        L.or_result_max_union.argtypes = [vp]
        L.or_result_assignment.argtypes = [vp, i32p]
        L.or_result_num_minibuckets.argtypes = [vp]
        L.or_result_mb_info.argtypes = [vp, ctypes.c_int, i32p, i32p, i32p, i32p, i32p, i64p]
        L.or_result_mb_data.argtypes = [vp, ctypes.c_int, i32p, i32p, i32p, dp]
        L.or_result_free.argtypes = [vp]
        _lib = L
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _flat(inst):
    arity = np.array([len(s) for s in inst.scopes], dtype=np.int32)
    scope = (np.concatenate([np.asarray(s, np.int32) for s in inst.scopes])
             if inst.scopes else np.zeros(0, np.int32))
    return arity, scope


def order(inst, heuristic: str = "min-fill"):
    """Elimination order (order[p] = variable at position p; the variable at
    position n-1 is eliminated first) and pseudo-tree parents (DFS only)."""
    L = lib()
    arity, scope = _flat(inst)
    arity, ap = _i32(arity)
    scope, sp = _i32(scope if scope.size else np.zeros(1, np.int32))
    o = np.zeros(max(inst.n, 1), np.int32)
    par = np.full(max(inst.n, 1), -1, np.int32)
    _, op = _i32(o)
    _, pp = _i32(par)
    rc = L.or_order(inst.n, len(inst.scopes), ap, sp, HEUR[heuristic], op, pp)
    assert rc == 0
    return o[:inst.n].copy(), par[:inst.n].copy()


def induced_width(inst, order_) -> int:
    L = lib()
    arity, scope = _flat(inst)
    arity, ap = _i32(arity)
    scope, sp = _i32(scope if scope.size else np.zeros(1, np.int32))
    o, op = _i32(order_)
    return int(L.or_induced_width(inst.n, len(inst.scopes), ap, sp, op))


def separators(inst, parent) -> List[List[int]]:
    """sep(a_i) for every agent of a pseudo-tree (Sec. 4), sorted ids."""
    L = lib()
    n = inst.n
    arity, scope = _flat(inst)
    arity, ap = _i32(arity)
    scope, sp = _i32(scope if scope.size else np.zeros(1, np.int32))
    par, pp = _i32(parent)
    out = np.zeros((n, n), np.uint8)
    L.or_separators(n, len(inst.scopes), ap, sp, pp,
                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return [sorted(int(u) for u in np.nonzero(out[i])[0]) for i in range(n)]


def map_rows(domains, out_scope, in_scope) -> np.ndarray:
    """Row of the input table addressed by every row of the output table
    (Sec. 6.3, Eq. (3))."""
    L = lib()
    d, dp_ = _i32(domains)
    o, op = _i32(out_scope)
    i, ip = _i32(in_scope if len(in_scope) else np.zeros(1, np.int32))
    size = int(np.prod([domains[v] for v in out_scope])) if len(out_scope) else 1
    out = np.zeros(size, np.int64)
    L.or_map_rows(len(domains), dp_, len(out_scope), op, len(in_scope), ip,
                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def sat_add(a: int, b: int) -> int:
    return int(lib().or_sat_add(a, b))


@dataclasses.dataclass
class MiniBucket:
    var: int
    k: int
    members: List[int]
    out_id: int
    out_scope: np.ndarray
    table: Optional[np.ndarray]


@dataclasses.dataclass
class Result:
    lb: float
    ub: float
    assignment: np.ndarray
    minibuckets: List[MiniBucket]
    max_union: int


def solve(inst, order_, ibound: int = 0, keep_tables: bool = True, parts=None, semiring: str = "min") -> Result:
    """Run (mini-)bucket elimination along `order_` with bound `ibound`
    (<= 0: plain BE) and return the bound, the assignment's cost, the
    assignment and every mini-bucket's members and output table.  `parts`
    optionally fixes the partition of some buckets: {var: [[fn ids], ...]}.
    semiring "sum": the sum-product variant (double costs; bound = -ln Z for
    BE, a lower bound of it with mini-buckets, R18)."""
    L = lib()
    n = inst.n
    arity, scope = _flat(inst)
    kind = {"cost_i32": 0, "cost_f64": 1, "prob_f64": 2}[inst.kind]
    if kind == 0:
        ti = (np.concatenate([np.asarray(t, np.int32).reshape(-1) for t in inst.tables])
              if inst.tables else np.zeros(1, np.int32))
        td = np.zeros(1, np.float64)
    else:
        ti = np.zeros(1, np.int32)
        td = (np.concatenate([np.asarray(t, np.float64).reshape(-1) for t in inst.tables])
              if inst.tables else np.zeros(1, np.float64))
    dom, domp = _i32(inst.domains if n else np.zeros(1, np.int32))
    arity, ap = _i32(arity if arity.size else np.zeros(1, np.int32))
    scope, sp = _i32(scope if scope.size else np.zeros(1, np.int32))
    ti, tip = _i32(ti)
    td = np.ascontiguousarray(td, np.float64)
    o, op = _i32(order_ if n else np.zeros(1, np.int32))
    h = ctypes.c_void_p()
    trip = []
    for v, plist in (parts or {}).items():
        for k, members in enumerate(plist):
            for fid in members:
                trip += [int(v), k, int(fid)]
    ov, ovp = _i32(trip if trip else [0, 0, 0])
    if semiring == "sum":
        if parts:
            raise ValueError("given partitions apply to min-sum only")
        rc = L.or_solve_sum(n, domp, len(inst.scopes), ap, sp,
                            td.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), kind, op, int(ibound),
                            ctypes.byref(h))
        if rc == -3:
            raise ValueError("the sum-product variant needs double costs")
    elif semiring == "min":
        rc = L.or_solve_parts(n, domp, len(inst.scopes), ap, sp, tip,
                              td.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), kind, op,
                              int(ibound), ovp, len(trip) // 3, ctypes.byref(h))
    else:
        raise ValueError(f"unknown semiring {semiring}")
    if rc == -2:
        raise ValueError("given partition is not a valid partition of its bucket")
    assert rc == 0
    try:
        asg = np.zeros(max(n, 1), np.int32)
        L.or_result_assignment(h, asg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        mbs = []
        for i in range(L.or_result_num_minibuckets(h)):
            var, k, nm, oid, oa = (ctypes.c_int32() for _ in range(5))
            osz = ctypes.c_int64()
            L.or_result_mb_info(h, i, ctypes.byref(var), ctypes.byref(k), ctypes.byref(nm),
                                ctypes.byref(oid), ctypes.byref(oa), ctypes.byref(osz))
            mem = np.zeros(max(nm.value, 1), np.int32)
            osc = np.zeros(max(oa.value, 1), np.int32)
            tab = None
            tip_ = None
            tdp_ = None
            if keep_tables:
                if kind == 0:
                    tab = np.zeros(osz.value, np.int32)
                    tip_ = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
                else:
                    tab = np.zeros(osz.value, np.float64)
                    tdp_ = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            L.or_result_mb_data(h, i, mem.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                osc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), tip_, tdp_)
            mbs.append(MiniBucket(var=var.value, k=k.value, members=[int(x) for x in mem[:nm.value]],
                                  out_id=oid.value, out_scope=osc[:oa.value].copy(), table=tab))
        return Result(lb=L.or_result_lb(h), ub=L.or_result_ub(h), assignment=asg[:n].copy(),
                      minibuckets=mbs, max_union=int(L.or_result_max_union(h)))
    finally:
        L.or_result_free(h)
