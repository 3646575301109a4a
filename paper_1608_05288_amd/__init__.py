"""Python binding of the MI355X UTIL-table engine (libbx.so, include/bx.h).

Argument marshalling only: every step of the solve path runs in the C++
planner and the HIP kernels of libbx.so.  PyTorch provides device memory
(the workspace tensor) and streams.  There is no CPU fallback: if the
library is missing, importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbx.so")

BX_OK = 0
STATUS = {0: "BX_OK", -1: "BX_E_INVALID", -2: "BX_E_NOMEM", -3: "BX_E_TOO_LARGE",
          -4: "BX_E_DEVICE", -5: "BX_E_UNSUPPORTED", -6: "BX_E_STATE"}
COST = {"i32": 0, "f32": 1}
ALGO = {"be": 0, "mbe": 1, "dpop": 2, "adpop": 3}
ORDER = {"min-degree": 0, "min-fill": 1, "dfs": 2, "degree-sort": 3}
PARTITION = {"greedy": 0, "learned": 1}
SCHED = {"per-bucket": 0, "level": 1, "dataflow": 2, "auto": 3}
INF_I32 = 2**31 - 1

# names exported by libbx.so, as declared in include/bx.h
EXPORTS = [
    "bx_options_default", "bx_problem_create", "bx_problem_add_function",
    "bx_problem_add_prob_table", "bx_problem_set_order", "bx_problem_set_pseudotree",
    "bx_problem_num_vars", "bx_problem_destroy", "bx_compute_order", "bx_induced_width",
    "bx_plan_create", "bx_plan_workspace_bytes", "bx_plan_upload", "bx_plan_execute",
    "bx_plan_execute_sched", "bx_plan_results", "bx_plan_get_stats", "bx_plan_num_minibuckets",
    "bx_plan_minibucket_info", "bx_plan_order", "bx_plan_util_table", "bx_plan_autotune",
    "bx_plan_describe", "bx_plan_set_timing", "bx_plan_last_timing", "bx_plan_graph_create",
    "bx_plan_graph_launch", "bx_plan_destroy",
    "bx_last_error", "bx_version",
]


class BxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("ibound", ctypes.c_int32), ("order", ctypes.c_int),
                ("partition", ctypes.c_int), ("schedule", ctypes.c_int),
                ("max_table_entries", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n_minibuckets", ctypes.c_int64), ("util_rows", ctypes.c_int64),
                ("joint_entries", ctypes.c_int64), ("algo_bytes", ctypes.c_int64),
                ("n_levels", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("max_scope", ctypes.c_int32), ("value_levels", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libbx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_1608_05288_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    vp = ctypes.c_void_p
    L.bx_options_default.argtypes = [ctypes.POINTER(Options)]
    L.bx_options_default.restype = None
    L.bx_problem_create.argtypes = [ctypes.c_int32, i32p, ctypes.c_int, ctypes.POINTER(vp)]
    L.bx_problem_add_function.argtypes = [vp, ctypes.c_int32, i32p, vp, ctypes.c_int64]
    L.bx_problem_add_prob_table.argtypes = [vp, ctypes.c_int32, i32p,
                                            ctypes.POINTER(ctypes.c_double), ctypes.c_int64]
    L.bx_problem_set_order.argtypes = [vp, i32p]
    L.bx_problem_set_pseudotree.argtypes = [vp, i32p]
    L.bx_problem_num_vars.argtypes = [vp]
    L.bx_problem_destroy.argtypes = [vp]
    L.bx_problem_destroy.restype = None
    L.bx_compute_order.argtypes = [vp, ctypes.c_int, i32p, i32p]
    L.bx_induced_width.argtypes = [vp, i32p, i32p]
    L.bx_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(Options),
                                 ctypes.POINTER(vp)]
    L.bx_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.bx_plan_upload.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.bx_plan_execute.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.bx_plan_execute_sched.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]
    L.bx_plan_results.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), i32p, vp]
    L.bx_plan_get_stats.argtypes = [vp, ctypes.POINTER(PlanStats)]
    L.bx_plan_num_minibuckets.argtypes = [vp, ctypes.c_int32, i32p]
    L.bx_plan_minibucket_info.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, i32p, i32p, i32p,
                                          i32p, i32p, i32p, ctypes.POINTER(ctypes.c_int64)]
    L.bx_plan_order.argtypes = [vp, ctypes.c_int32, i32p]
    L.bx_plan_util_table.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64, vp]
    L.bx_plan_autotune.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp]
    L.bx_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.bx_plan_set_timing.argtypes = [vp, ctypes.c_int32]
    L.bx_plan_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_float)]
    L.bx_plan_graph_create.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]
    L.bx_plan_graph_launch.argtypes = [vp, vp]
    L.bx_plan_destroy.argtypes = [vp]
    L.bx_plan_destroy.restype = None
    L.bx_last_error.restype = ctypes.c_char_p
    L.bx_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int):
    if status != BX_OK:
        raise BxError(status, lib().bx_last_error().decode())


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Problem:
    """A problem handle (bx_problem).  Build from arrays or from an
    `Instance` of `paper_1608_05288_amd.synth`."""

    def __init__(self, domains: Sequence[int], cost: str = "i32"):
        L = lib()
        self.domains = _i32(domains)
        self.cost = cost
        h = ctypes.c_void_p()
        _check(L.bx_problem_create(len(self.domains), _p(self.domains), COST[cost], ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def add_function(self, scope: Sequence[int], table: np.ndarray):
        s = _i32(scope)
        dt = np.int32 if self.cost == "i32" else np.float32
        t = np.ascontiguousarray(np.asarray(table).reshape(-1), dtype=dt)
        _check(lib().bx_problem_add_function(self._h, len(s), _p(s) if len(s) else None,
                                             t.ctypes.data_as(ctypes.c_void_p), t.size))

    def add_prob_table(self, scope: Sequence[int], probs: np.ndarray):
        s = _i32(scope)
        t = np.ascontiguousarray(np.asarray(probs, np.float64).reshape(-1))
        _check(lib().bx_problem_add_prob_table(self._h, len(s), _p(s) if len(s) else None,
                                               t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), t.size))

    def set_order(self, order: Sequence[int]):
        o = _i32(order)
        _check(lib().bx_problem_set_order(self._h, _p(o)))

    def set_pseudotree(self, parent: Sequence[int]):
        p = _i32(parent)
        _check(lib().bx_problem_set_pseudotree(self._h, _p(p)))

    def compute_order(self, heuristic: str = "min-fill"):
        n = len(self.domains)
        o = np.zeros(max(n, 1), np.int32)
        par = np.full(max(n, 1), -1, np.int32)
        _check(lib().bx_compute_order(self._h, ORDER[heuristic], _p(o), _p(par)))
        return o[:n].copy(), par[:n].copy()

    def induced_width(self, order) -> int:
        o = _i32(order)
        w = ctypes.c_int32()
        _check(lib().bx_induced_width(self._h, _p(o), ctypes.byref(w)))
        return int(w.value)

    @classmethod
    def from_instance(cls, inst) -> "Problem":
        if inst.kind == "cost_i32":
            p = cls(inst.domains, "i32")
            for s, t in zip(inst.scopes, inst.tables):
                p.add_function(s, t)
        elif inst.kind == "prob_f64":
            p = cls(inst.domains, "f32")
            for s, t in zip(inst.scopes, inst.tables):
                p.add_prob_table(s, t)
        elif inst.kind == "cost_f32":
            p = cls(inst.domains, "f32")
            for s, t in zip(inst.scopes, inst.tables):
                p.add_function(s, t)
        else:
            raise ValueError(inst.kind)
        if inst.parents is not None:
            p.set_pseudotree(inst.parents)
        return p

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bx_problem_destroy(h)
            self._h = None


@dataclasses.dataclass
class MiniBucketInfo:
    var: int
    members: List[int]
    out_id: int
    out_scope: np.ndarray
    out_rows: int


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A plan (bx_plan) for one or more problems, plus its device workspace."""

    def __init__(self, problems, algo: str = "be", ibound: int = 0, order: str = "min-fill",
                 schedule: str = "auto", partition: str = "greedy", max_table_entries: int = 0):
        L = lib()
        if isinstance(problems, Problem):
            problems = [problems]
        self.problems = list(problems)
        opt = Options()
        L.bx_options_default(ctypes.byref(opt))
        opt.algo = ALGO[algo]
        opt.ibound = int(ibound)
        opt.order = ORDER[order]
        opt.partition = PARTITION[partition]
        opt.schedule = SCHED[schedule]
        opt.max_table_entries = int(max_table_entries)
        arr = (ctypes.c_void_p * len(self.problems))(*[p.handle.value for p in self.problems])
        h = ctypes.c_void_p()
        _check(L.bx_plan_create(arr, len(self.problems), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.workspace = None
        self.cost = self.problems[0].cost

    # -------------------------------------------------------------- info
    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().bx_plan_workspace_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def stats(self) -> PlanStats:
        s = PlanStats()
        _check(lib().bx_plan_get_stats(self._h, ctypes.byref(s)))
        return s

    def order(self, prob: int = 0) -> np.ndarray:
        n = len(self.problems[prob].domains)
        o = np.zeros(max(n, 1), np.int32)
        _check(lib().bx_plan_order(self._h, prob, _p(o)))
        return o[:n].copy()

    def minibuckets(self, prob: int = 0) -> List[MiniBucketInfo]:
        L = lib()
        c = ctypes.c_int32()
        _check(L.bx_plan_num_minibuckets(self._h, prob, ctypes.byref(c)))
        out = []
        for i in range(c.value):
            var, nm, oid, oa = (ctypes.c_int32() for _ in range(4))
            mem = np.zeros(256, np.int32)
            osc = np.zeros(64, np.int32)
            rows = ctypes.c_int64()
            _check(L.bx_plan_minibucket_info(self._h, prob, i, ctypes.byref(var), ctypes.byref(nm),
                                             _p(mem), ctypes.byref(oid), ctypes.byref(oa), _p(osc),
                                             ctypes.byref(rows)))
            out.append(MiniBucketInfo(var=var.value, members=mem[:nm.value].tolist(), out_id=oid.value,
                                      out_scope=osc[:oa.value].copy(), out_rows=int(rows.value)))
        return out

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(256)
        _check(lib().bx_plan_describe(self._h, buf, 256))
        return buf.value.decode()

    # ------------------------------------------------------------ device
    def allocate(self, device="cuda"):
        """Workspace as a torch uint8 tensor, 256-byte aligned."""
        import torch
        nbytes = self.workspace_bytes()
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self._buf = buf
        self.workspace = buf[off:off + nbytes]
        self._ws_ptr = ctypes.c_void_p(buf.data_ptr() + off)
        return self.workspace

    def upload(self, stream=None):
        if self.workspace is None:
            self.allocate()
        _check(lib().bx_plan_upload(self._h, self._ws_ptr, self.workspace_bytes(), _stream_ptr(stream)))

    def execute(self, schedule: Optional[str] = None, stream=None):
        if schedule is None:
            _check(lib().bx_plan_execute(self._h, self._ws_ptr, self.workspace_bytes(), _stream_ptr(stream)))
        else:
            _check(lib().bx_plan_execute_sched(self._h, self._ws_ptr, self.workspace_bytes(),
                                               SCHED[schedule], _stream_ptr(stream)))

    def results(self, prob: int = 0, stream=None):
        n = len(self.problems[prob].domains)
        b = ctypes.c_double()
        u = ctypes.c_double()
        asg = np.zeros(max(n, 1), np.int32)
        _check(lib().bx_plan_results(self._h, self._ws_ptr, prob, ctypes.byref(b), ctypes.byref(u),
                                     _p(asg), _stream_ptr(stream)))
        return b.value, u.value, asg[:n].copy()

    def util_table(self, prob: int, i: int, rows: int, stream=None) -> np.ndarray:
        dt = np.int32 if self.cost == "i32" else np.float32
        out = np.zeros(max(rows, 1), dt)
        _check(lib().bx_plan_util_table(self._h, self._ws_ptr, prob, i,
                                        out.ctypes.data_as(ctypes.c_void_p), rows, _stream_ptr(stream)))
        return out[:rows]

    def autotune(self, reps: int = 3, stream=None):
        _check(lib().bx_plan_autotune(self._h, self._ws_ptr, self.workspace_bytes(), reps,
                                      _stream_ptr(stream)))

    def set_timing(self, on: bool = True):
        _check(lib().bx_plan_set_timing(self._h, int(on)))

    def last_timing(self):
        """(util phase ms, util kernels ms, value kernel ms) of the last timed execute."""
        a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        _check(lib().bx_plan_last_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def graph_create(self, schedule: str = "auto", stream=None):
        """Capture one execute into a hipGraph kept by the plan (non-default stream)."""
        _check(lib().bx_plan_graph_create(self._h, self._ws_ptr, self.workspace_bytes(), SCHED[schedule],
                                          _stream_ptr(stream)))

    def graph_launch(self, stream=None):
        _check(lib().bx_plan_graph_launch(self._h, _stream_ptr(stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bx_plan_destroy(h)
            self._h = None


@dataclasses.dataclass
class Solution:
    bound: float
    ub: float
    assignment: np.ndarray


def solve(inst, algo: str = "be", ibound: int = 0, order: str = "min-fill",
          schedule: str = "auto", stream=None) -> Solution:
    """Solve one instance on the current GPU: plan, upload, execute, results."""
    p = Problem.from_instance(inst)
    pl = Plan([p], algo=algo, ibound=ibound, order=order, schedule=schedule)
    pl.upload(stream)
    pl.execute(stream=stream)
    b, u, a = pl.results(0, stream)
    return Solution(b, u, a)


def solve_batch(insts, algo: str = "mbe", ibound: int = 10, order: str = "min-fill",
                schedule: str = "auto", stream=None) -> List[Solution]:
    ps = [Problem.from_instance(i) for i in insts]
    pl = Plan(ps, algo=algo, ibound=ibound, order=order, schedule=schedule)
    pl.upload(stream)
    pl.execute(stream=stream)
    out = []
    for k in range(len(ps)):
        b, u, a = pl.results(k, stream)
        out.append(Solution(b, u, a))
    return out
