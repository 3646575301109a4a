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
ALGO = {"be": 0, "mbe": 1, "dpop": 2, "adpop": 3, "be-sum": 4, "mbe-sum": 5}
ORDER = {"min-degree": 0, "min-fill": 1, "dfs": 2, "degree-sort": 3}
PARTITION = {"greedy": 0, "learned": 1}
SCHED = {"per-bucket": 0, "level": 1, "dataflow": 2, "auto": 3}
FLAG_NO_BLOCKING = 0x1          # bx_options.flags: no register blocking (BX_FLAG_NO_BLOCKING)
FLAG_FORCE_NT = 0x2             # blocked rows stored non-temporally on every level
FLAG_STAGE_ALWAYS = 0x4         # the LDS-staging tiled kernel on every level
FLAG_STAGE_NEVER = 0x8          # never the staging kernel
FLAG_NO_PACKING = 0x10          # no packing / fusion of small mini-buckets
FLAG_XCD_ORDER = 0x20           # every level's tiles taken XCD by XCD
INF_I32 = 2**31 - 1
MLP_NOALLOC_MAX_BATCH = 4096    # samples bx_mlp_backward_noalloc's static scratch holds

# names exported by libbx.so, as declared in include/bx.h
EXPORTS = [
    "bx_options_default", "bx_problem_create", "bx_problem_add_function",
    "bx_problem_add_prob_table", "bx_problem_set_order", "bx_problem_set_pseudotree",
    "bx_problem_num_vars", "bx_problem_destroy", "bx_compute_order", "bx_induced_width",
    "bx_plan_create", "bx_plan_workspace_bytes", "bx_plan_upload", "bx_plan_execute",
    "bx_plan_execute_sched", "bx_plan_results", "bx_plan_get_stats", "bx_plan_num_minibuckets",
    "bx_plan_minibucket_info", "bx_plan_order", "bx_plan_util_table", "bx_plan_level_info",
    "bx_plan_level_timing", "bx_plan_validate", "bx_plan_minibucket_timing", "bx_plan_simulated_runtime",
    "bx_stream_probe", "bx_plan_autotune",
    "bx_plan_describe", "bx_plan_set_timing", "bx_plan_last_timing", "bx_plan_graph_create",
    "bx_plan_graph_launch", "bx_plan_destroy", "bx_partition_num_features", "bx_plan_create_chooser",
    "bx_plan_partition_stats", "bx_plan_num_decisions", "bx_plan_decision_info", "bx_plan_candidate_parts",
    "bx_plan_candidate_scratch_bytes", "bx_plan_candidate_values", "bx_mlp_num_params", "bx_mlp_forward", "bx_mlp_backward",
    "bx_mlp_backward_noalloc",
    "bx_mlp_adam_step", "bx_mlp_pack_bf16", "bx_mlp_mse", "bx_mlp_infer_bf16", "bx_plan_create_learned",
    "bx_bnb_workspace_bytes", "bx_bnb_solve", "bx_plan_stream_bytes", "bx_plan_execute_streamed",
    "bx_plan_stream_table", "bx_last_error", "bx_version",
]

CHOOSER = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                           ctypes.POINTER(ctypes.c_int32))


class MlpDesc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("d_params", ctypes.c_void_p), ("d_params_bf16", ctypes.c_void_p)]


class BxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int), ("ibound", ctypes.c_int32), ("order", ctypes.c_int),
                ("partition", ctypes.c_int), ("schedule", ctypes.c_int),
                ("max_table_entries", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("tune_cache", ctypes.c_char_p), ("pack_max_rows", ctypes.c_int32),
                ("fuse_max_rows", ctypes.c_int32), ("fuse_max_stages", ctypes.c_int32),
                ("fuse_max_stage_rows", ctypes.c_int32), ("pack_stage_rows", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n_minibuckets", ctypes.c_int64), ("util_rows", ctypes.c_int64),
                ("joint_entries", ctypes.c_int64), ("algo_bytes", ctypes.c_int64),
                ("n_levels", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("max_scope", ctypes.c_int32), ("value_levels", ctypes.c_int32),
                ("tile_capacity", ctypes.c_int64)]


class LevelInfo(ctypes.Structure):
    _fields_ = [("n_minibuckets", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("n_row_tiles", ctypes.c_int32), ("n_blocked", ctypes.c_int32),
                ("util_rows", ctypes.c_int64), ("algo_bytes", ctypes.c_int64),
                ("staged", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("tile_goal", ctypes.c_int32), ("n_lane_tiles", ctypes.c_int32),
                ("n_pack_tiles", ctypes.c_int32), ("n_packed", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libbx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_1608_05288_amd.build)")
    # torch's HIP runtime is loaded first so that the library binds to it (it
    # has the same SONAME) rather than pulling a second runtime into the
    # process: device pointers and streams then belong to one runtime
    import torch  # noqa: F401
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
    L.bx_plan_level_info.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(LevelInfo)]
    L.bx_plan_level_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int32]
    L.bx_plan_validate.argtypes = [vp]
    L.bx_plan_stream_bytes.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t)]
    L.bx_plan_execute_streamed.argtypes = [vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t, ctypes.c_int64, vp,
                                           ctypes.POINTER(ctypes.c_double)]
    L.bx_plan_stream_table.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int64]
    L.bx_bnb_workspace_bytes.argtypes = [vp, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]
    L.bx_bnb_solve.argtypes = [vp, ctypes.POINTER(Options), vp, ctypes.c_size_t, vp, ctypes.c_int64,
                               ctypes.POINTER(ctypes.c_double), i32p, ctypes.POINTER(ctypes.c_int64)]
    L.bx_plan_minibucket_timing.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.c_int32]
    L.bx_plan_simulated_runtime.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.c_double,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                            i32p]
    L.bx_plan_autotune.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp]
    L.bx_stream_probe.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_size_t, ctypes.c_int32, vp]
    L.bx_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.bx_plan_set_timing.argtypes = [vp, ctypes.c_int32]
    L.bx_plan_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_float)]
    L.bx_plan_graph_create.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]
    L.bx_plan_graph_launch.argtypes = [vp, vp]
    L.bx_plan_destroy.argtypes = [vp]
    L.bx_plan_destroy.restype = None
    L.bx_partition_num_features.restype = ctypes.c_int32
    L.bx_plan_create_chooser.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(Options), CHOOSER,
                                         vp, ctypes.POINTER(vp)]
    L.bx_plan_partition_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.bx_plan_num_decisions.argtypes = [vp, i32p, ctypes.POINTER(ctypes.c_int64)]
    L.bx_plan_decision_info.argtypes = [vp, ctypes.c_int32, i32p, i32p, i32p, i32p, i32p, i32p]
    L.bx_plan_candidate_parts.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, i32p]
    L.bx_plan_candidate_scratch_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.bx_plan_candidate_values.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp, vp, vp, ctypes.c_size_t,
                                           vp]
    L.bx_mlp_num_params.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.bx_mlp_num_params.restype = ctypes.c_int64
    mp = ctypes.POINTER(MlpDesc)
    L.bx_mlp_forward.argtypes = [mp, vp, vp, vp, ctypes.c_int32, vp]
    L.bx_mlp_backward.argtypes = [mp, vp, vp, vp, vp, vp, ctypes.c_int32, vp]
    L.bx_mlp_backward_noalloc.argtypes = [mp, vp, vp, vp, vp, ctypes.c_int32, vp]
    L.bx_mlp_adam_step.argtypes = [mp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_int32, vp]
    L.bx_mlp_pack_bf16.argtypes = [mp, vp]
    L.bx_mlp_infer_bf16.argtypes = [mp, vp, vp, ctypes.c_int32, vp]
    L.bx_mlp_mse.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp]
    L.bx_plan_create_learned.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(Options), mp, vp,
                                         ctypes.c_size_t, ctypes.c_float, vp, ctypes.POINTER(vp)]
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


def partition_num_features() -> int:
    return int(lib().bx_partition_num_features())


class Plan:
    """A plan (bx_plan) for one or more problems, plus its device workspace.

    Partitions of over-full buckets: the greedy rule by default; `chooser`
    (a Python callable (n_decisions, decision_problem, cand_offsets,
    features) -> choices) or `model` (a PartitionMLP scored on the device)
    choose among candidates.
    """

    def __init__(self, problems, algo: str = "be", ibound: int = 0, order: str = "min-fill",
                 schedule: str = "auto", partition: str = "greedy", max_table_entries: int = 0,
                 chooser=None, model=None, margin: float = 0.0, stream=None, blocking: bool = True,
                 flags: int = 0, tune_cache: Optional[str] = None, packing: bool = True,
                 pack: Optional[dict] = None):
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
        opt.flags = int(flags) | (0 if blocking else FLAG_NO_BLOCKING) | (0 if packing else FLAG_NO_PACKING)
        for k, v in (pack or {}).items():      # packing limits (bx_options fields)
            if k not in ("pack_max_rows", "fuse_max_rows", "fuse_max_stages", "fuse_max_stage_rows",
                         "pack_stage_rows"):
                raise ValueError(f"unknown packing limit {k}")
            setattr(opt, k, int(v))
        self._tune_cache = tune_cache.encode() if tune_cache else None
        opt.tune_cache = self._tune_cache
        arr = (ctypes.c_void_p * len(self.problems))(*[p.handle.value for p in self.problems])
        h = ctypes.c_void_p()
        if chooser is not None:
            nf = partition_num_features()
            err = []

            def _cb(user, n_dec, dec_prob, offs, feats, choices):
                try:
                    probs_ = np.ctypeslib.as_array(dec_prob, shape=(n_dec,)).copy()
                    off = np.ctypeslib.as_array(offs, shape=(n_dec + 1,)).copy()
                    f = np.ctypeslib.as_array(feats, shape=(int(off[-1]), nf)).copy()
                    ch = np.asarray(chooser(int(n_dec), probs_, off, f), dtype=np.int32)
                    for d in range(n_dec):
                        choices[d] = int(ch[d])
                    return 0
                except Exception as e:      # reported as a planning failure
                    err.append(e)
                    return -1
            self._cb = CHOOSER(_cb)
            rc = L.bx_plan_create_chooser(arr, len(self.problems), ctypes.byref(opt), self._cb, None,
                                          ctypes.byref(h))
            if err:
                raise err[0]
            _check(rc)
        elif model is not None:
            import torch
            nf = partition_num_features()
            cap = 1 << 16                       # candidates per round
            self._score_buf = torch.empty(cap * (nf + 1), dtype=torch.float32, device="cuda")
            _check(L.bx_plan_create_learned(arr, len(self.problems), ctypes.byref(opt),
                                            ctypes.byref(model.desc), ctypes.c_void_p(self._score_buf.data_ptr()),
                                            self._score_buf.numel() * 4, float(margin), _stream_ptr(stream),
                                            ctypes.byref(h)))
        else:
            _check(L.bx_plan_create(arr, len(self.problems), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.workspace = None
        self.cost = self.problems[0].cost

    def partition_stats(self):
        """(decisions taken, decisions that differ from the greedy rule)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().bx_plan_partition_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def decisions(self):
        """Recorded partition decisions: list of dicts (prob, var, fns, n_cands,
        choice), in the order the chooser saw them."""
        L = lib()
        n = ctypes.c_int32()
        _check(L.bx_plan_num_decisions(self._h, ctypes.byref(n), None))
        out = []
        for d in range(n.value):
            pr, var, nf, nc, ch = (ctypes.c_int32() for _ in range(5))
            ids = np.zeros(256, np.int32)
            _check(L.bx_plan_decision_info(self._h, d, ctypes.byref(pr), ctypes.byref(var), ctypes.byref(nf),
                                           _p(ids), ctypes.byref(nc), ctypes.byref(ch)))
            out.append({"prob": pr.value, "var": var.value, "fns": ids[:nf.value].tolist(),
                        "n_cands": nc.value, "choice": ch.value})
        return out

    def candidate_parts(self, d: int, c: int) -> np.ndarray:
        n = len(self.decisions()[d]["fns"])
        part = np.zeros(max(n, 1), np.int32)
        _check(lib().bx_plan_candidate_parts(self._h, d, c, _p(part)))
        return part[:n]

    def candidate_values(self, rnd, stream=None):
        """Sampled bound contributions of every recorded candidate (see
        bx_plan_candidate_values); rnd: torch uint32-valued int32/int64 tensor
        [n_decisions, samples, 32] on the device.  Returns a float64 tensor."""
        import torch
        L = lib()
        n, nc = ctypes.c_int32(), ctypes.c_int64()
        _check(L.bx_plan_num_decisions(self._h, ctypes.byref(n), ctypes.byref(nc)))
        rnd = rnd.contiguous()
        if rnd.dim() != 3 or rnd.shape[0] != n.value or rnd.shape[2] != 32 or rnd.element_size() != 4:
            raise ValueError("rnd must be a 4-byte tensor of shape [n_decisions, samples, 32]")
        out = torch.full((max(nc.value, 1),), float("nan"), dtype=torch.float64, device="cuda")
        sb = ctypes.c_size_t()
        _check(L.bx_plan_candidate_scratch_bytes(self._h, ctypes.byref(sb)))
        scratch = torch.empty(sb.value + 256, dtype=torch.uint8, device="cuda")
        sp = scratch.data_ptr() + (-scratch.data_ptr()) % 256
        _check(L.bx_plan_candidate_values(self._h, self._ws_ptr, self.workspace_bytes(), int(rnd.shape[1]),
                                          ctypes.c_void_p(rnd.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(sp), sb.value, _stream_ptr(stream)))
        return out[:nc.value]

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

    def level_info(self, level: int) -> LevelInfo:
        r = LevelInfo()
        _check(lib().bx_plan_level_info(self._h, int(level), ctypes.byref(r)))
        return r

    def level_timing(self) -> np.ndarray:
        """Per-level device ms of the last timed LEVEL execute (after results())."""
        n = self.stats().n_levels
        out = (ctypes.c_float * max(n, 1))()
        _check(lib().bx_plan_level_timing(self._h, out, n))
        return np.array(out[:n], np.float64)

    def stream_bytes(self, chunk_rows: int = 1 << 20):
        """(device bytes, host bytes) of a streamed execute."""
        d, h = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().bx_plan_stream_bytes(self._h, int(chunk_rows), ctypes.byref(d), ctypes.byref(h)))
        return d.value, h.value

    def execute_streamed(self, chunk_rows: int = 1 << 20, stream=None):
        """Streamed execute (tables in pinned host memory, chunks overlapped
        with copies); returns the bound of every problem.  The host tables
        stay in self.host_tables (a pinned uint8 tensor)."""
        import torch
        dbytes, hbytes = self.stream_bytes(chunk_rows)
        # the device buffer and the pinned host tables of an earlier call are
        # reused when large enough (pinning hundreds of MB costs more than a pass)
        buf = getattr(self, "_stream_buf", None)
        if buf is None or buf.numel() < dbytes + 256:
            buf = torch.empty(dbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = buf.data_ptr() + (-buf.data_ptr()) % 256
        if getattr(self, "host_tables", None) is None or self.host_tables.numel() < max(hbytes, 1):
            self.host_tables = torch.empty(max(hbytes, 1), dtype=torch.uint8, pin_memory=True)
        out = (ctypes.c_double * len(self.problems))()
        _check(lib().bx_plan_execute_streamed(self._h, ctypes.c_void_p(ptr), dbytes,
                                              ctypes.c_void_p(self.host_tables.data_ptr()), hbytes,
                                              int(chunk_rows), _stream_ptr(stream), out))
        self._stream_buf = buf
        return np.array(out[:], np.float64)

    def stream_table(self, prob: int, i: int, rows: int) -> np.ndarray:
        dt = np.int32 if self.cost == "i32" else np.float32
        out = np.zeros(max(rows, 1), dt)
        _check(lib().bx_plan_stream_table(self._h, ctypes.c_void_p(self.host_tables.data_ptr()), prob, i,
                                          out.ctypes.data_as(ctypes.c_void_p), rows))
        return out[:rows]

    def validate(self):
        """Host self-check of the launch schedule (raises BxError on a violation)."""
        _check(lib().bx_plan_validate(self._h))

    def minibucket_timing(self, prob: int = 0) -> np.ndarray:
        """Device ms of every mini-bucket of problem `prob` (creation order) in
        the last timed per-bucket execute (after results())."""
        n = len(self.minibuckets(prob))
        out = (ctypes.c_float * max(n, 1))()
        _check(lib().bx_plan_minibucket_timing(self._h, int(prob), out, n))
        return np.array(out[:n], np.float64)

    def simulated_runtime(self, prob: int = 0, mb_ms=None, latency_ms: float = 0.0):
        """(util_ms, value_ms, value_hops) of the simulated distributed run:
        agents = variables, per-agent UTIL work = its mini-buckets' times
        (`mb_ms`, creation order; None: the last timed per-bucket execute)."""
        ptr = None
        if mb_ms is not None:
            arr = np.ascontiguousarray(mb_ms, np.float32)
            if arr.size != len(self.minibuckets(prob)):
                raise ValueError("mb_ms needs one time per mini-bucket")
            ptr = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        u, v, h = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(lib().bx_plan_simulated_runtime(self._h, int(prob), ptr, float(latency_ms),
                                               ctypes.byref(u), ctypes.byref(v), ctypes.byref(h)))
        return u.value, v.value, h.value

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        _check(lib().bx_plan_describe(self._h, buf, 1024))
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


def stream_probe(kind: str, dst, src=None, nbytes: int = 0, grid: int = 0, stream=None):
    """Streaming bandwidth reference (bx_stream_probe): kind "copy" (src ->
    dst), "write" (dst) or "read" (src; one int32 per workgroup into dst);
    dst / src are torch device tensors."""
    k = {"copy": 0, "write": 1, "read": 2}[kind]
    dp = ctypes.c_void_p(dst.data_ptr()) if dst is not None else None
    sp = ctypes.c_void_p(src.data_ptr()) if src is not None else None
    _check(lib().bx_stream_probe(k, dp, sp, int(nbytes), int(grid), _stream_ptr(stream)))


class PartitionMLP:
    """The candidate-scoring network (2 x 128 ReLU + linear output) with its
    parameters, Adam moments and bf16 copy in device memory (torch tensors);
    every step runs in the library's kernels."""

    def __init__(self, n_in: int = None, hidden: int = 128, seed: int = 0, params: np.ndarray = None,
                 margin: float = 0.0):
        import torch
        self.margin = float(margin)          # decision margin chosen at training time
        self.n_in = int(n_in if n_in is not None else partition_num_features())
        self.hidden = int(hidden)
        n = int(lib().bx_mlp_num_params(self.n_in, self.hidden))
        if params is None:
            params = self.init_params(self.n_in, self.hidden, seed)
        params = np.asarray(params, np.float32).reshape(-1)
        if params.size != n:
            raise ValueError(f"expected {n} parameters, got {params.size}")
        self.params = torch.from_numpy(params.copy()).cuda()
        self.bf16 = torch.zeros(n, dtype=torch.int16, device="cuda")
        self.m = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.v = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.grads = torch.zeros(n, dtype=torch.float32, device="cuda")
        self.step_count = 0
        self.desc = MlpDesc(self.n_in, self.hidden, ctypes.c_void_p(self.params.data_ptr()),
                            ctypes.c_void_p(self.bf16.data_ptr()))
        self.pack_bf16()

    @staticmethod
    def init_params(n_in: int, hidden: int, seed: int = 0) -> np.ndarray:
        """He-uniform weights, zero biases, in the library's parameter layout."""
        rng = np.random.default_rng(seed)
        w1 = rng.uniform(-1, 1, (hidden, n_in)) * np.sqrt(6.0 / n_in)
        w2 = rng.uniform(-1, 1, (hidden, hidden)) * np.sqrt(6.0 / hidden)
        w3 = rng.uniform(-1, 1, hidden) * np.sqrt(6.0 / hidden)
        return np.concatenate([w1.reshape(-1), np.zeros(hidden), w2.reshape(-1), np.zeros(hidden),
                               w3, np.zeros(1)]).astype(np.float32)

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr())

    def forward(self, x, stream=None):
        """fp32 outputs and activations for x (torch float32 [B, n_in] on the device)."""
        import torch
        x = x.contiguous()
        B = x.shape[0]
        act = torch.empty(B, 2 * self.hidden, dtype=torch.float32, device="cuda")
        y = torch.empty(B, dtype=torch.float32, device="cuda")
        _check(lib().bx_mlp_forward(ctypes.byref(self.desc), self._p(x), self._p(act), self._p(y), B,
                                    _stream_ptr(stream)))
        return y, act

    def backward(self, x, act, dy, stream=None):
        import torch
        B = x.shape[0]
        work = torch.empty(B, 2 * self.hidden, dtype=torch.float32, device="cuda")
        _check(lib().bx_mlp_backward(ctypes.byref(self.desc), self._p(x.contiguous()), self._p(act),
                                     self._p(dy.contiguous()), self._p(self.grads), self._p(work), B,
                                     _stream_ptr(stream)))
        return self.grads

    def backward_noalloc(self, x, act, dy, stream=None):
        """backward() with the library's static per-GPU scratch instead of a
        work buffer (no allocation; at most MLP_NOALLOC_MAX_BATCH samples)."""
        _check(lib().bx_mlp_backward_noalloc(ctypes.byref(self.desc), self._p(x.contiguous()), self._p(act),
                                             self._p(dy.contiguous()), self._p(self.grads), x.shape[0],
                                             _stream_ptr(stream)))
        return self.grads

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        _check(lib().bx_mlp_adam_step(ctypes.byref(self.desc), self._p(self.grads), self._p(self.m),
                                      self._p(self.v), lr, beta1, beta2, eps, self.step_count,
                                      _stream_ptr(stream)))

    def pack_bf16(self, stream=None):
        _check(lib().bx_mlp_pack_bf16(ctypes.byref(self.desc), _stream_ptr(stream)))

    def infer_bf16(self, x, stream=None):
        import torch
        x = x.contiguous()
        y = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().bx_mlp_infer_bf16(ctypes.byref(self.desc), self._p(x), self._p(y), x.shape[0],
                                       _stream_ptr(stream)))
        return y

    def mse(self, y, target, stream=None):
        """(loss tensor [1], dL/dy) of the mean squared error."""
        import torch
        dy = torch.empty_like(y)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(lib().bx_mlp_mse(self._p(y), self._p(target.contiguous()), self._p(dy), self._p(loss),
                                y.shape[0], _stream_ptr(stream)))
        return loss, dy

    def train_step(self, x, target, lr=1e-3, stream=None):
        """One Adam step on the mean squared error; returns the loss (a
        device tensor, read it with float() when needed)."""
        y, act = self.forward(x, stream)
        loss, dy = self.mse(y, target, stream)
        self.backward(x, act, dy, stream)
        self.adam_step(lr, stream=stream)
        return loss

    def numpy_params(self) -> np.ndarray:
        return self.params.detach().cpu().numpy().copy()

    def save(self, path: str):
        np.savez(path, params=self.numpy_params(), n_in=self.n_in, hidden=self.hidden, margin=self.margin)

    @classmethod
    def load(cls, path: str) -> "PartitionMLP":
        z = np.load(path)
        margin = float(z["margin"]) if "margin" in z.files else 0.0
        return cls(int(z["n_in"]), int(z["hidden"]), params=z["params"], margin=margin)


def bnb_solve(problem: "Problem", algo: str = "mbe", ibound: int = 4, order: str = "min-fill",
              max_nodes: int = 0, stream=None, packing: bool = True):
    """Branch and bound with the mini-bucket bound recomputed at every node
    (one batched device pass per expansion).  Returns (value, assignment,
    stats) with stats = dict(nodes, passes, pruned, proved)."""
    import torch
    L = lib()
    opt = Options()
    L.bx_options_default(ctypes.byref(opt))
    opt.algo = ALGO[algo]
    opt.ibound = int(ibound)
    opt.order = ORDER[order]
    opt.flags = 0 if packing else FLAG_NO_PACKING
    nb = ctypes.c_size_t()
    _check(L.bx_bnb_workspace_bytes(problem.handle, ctypes.byref(opt), ctypes.byref(nb)))
    buf = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    ptr = buf.data_ptr() + (-buf.data_ptr()) % 256
    n = len(problem.domains)
    val = ctypes.c_double()
    asg = np.zeros(max(n, 1), np.int32)
    st = (ctypes.c_int64 * 4)()
    _check(L.bx_bnb_solve(problem.handle, ctypes.byref(opt), ctypes.c_void_p(ptr), nb.value,
                          _stream_ptr(stream), int(max_nodes), ctypes.byref(val), _p(asg), st))
    return val.value, asg[:n].copy(), dict(nodes=st[0], passes=st[1], pruned=st[2], proved=bool(st[3]))
