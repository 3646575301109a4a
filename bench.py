#!/usr/bin/env python3
"""Benchmark of the UTIL-table engine on one MI355X.

Workload (default): 20x20 grid WCSP, domain 4, unary + 4-neighbour binary
int32 costs uniform in [0, 1000], Mini-Bucket Elimination at i-bound 12
(tables up to 4^12 entries), min-fill order; synthetic, seeded.  One step is
one device pass of the whole path -- every UTIL table (fused aggregate +
min-project), the bound, the value assignment and its cost -- with the plan
built and the inputs resident in HBM before the timed region.

Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, batch: int, seed0: int):
    from paper_1608_05288_amd import synth
    if name == "grid":
        insts = [synth.grid_wcsp(seed0 + s) for s in range(batch)]
        return insts, dict(algo="mbe", ibound=12, order="min-fill"), \
            f"grid20x20_d4_mbe_i12_minfill_x{batch}"
    if name == "batch":
        import paper_1608_05288_amd as bx

        def width_ok(inst):
            p = bx.Problem.from_instance(inst)
            o, _ = p.compute_order("min-fill")
            return 8 <= p.induced_width(o) <= 16
        insts = synth.accepted(synth.batch_candidate, batch, seed0, accept=width_ok)
        return insts, dict(algo="mbe", ibound=10, order="min-fill"), \
            f"batch_wcsp_n30-80_d2-4_w8-16_mbe_i10_x{batch}"
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid", choices=["grid", "batch"])
    ap.add_argument("--batch", type=int, default=0, help="instances per step (0: workload default)")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--compare-per-bucket", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="first run one device-to-device copy of MB MiB (a reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import torch
    import paper_1608_05288_amd as bx
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.arange(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    batch = args.batch or (16 if args.workload == "grid" else 256)
    insts, opts, wname = make_workload(args.workload, batch, args.seed)
    t0 = time.perf_counter()
    probs = [bx.Problem.from_instance(i) for i in insts]
    plan = bx.Plan(probs, schedule=args.schedule, **opts)
    plan_ms = (time.perf_counter() - t0) * 1e3
    st = plan.stats()
    plan.allocate()
    # a non-default stream (graph capture needs one), made current so every
    # library call below runs on it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    t0 = time.perf_counter()
    plan.upload(stream)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] workload={wname} mbs={st.n_minibuckets} rows={st.util_rows} joint={st.joint_entries} "
        f"levels={st.n_levels} algo_bytes={st.algo_bytes} plan_ms={plan_ms:.1f} upload_ms={upload_ms:.1f}")
    if args.schedule == "auto":
        plan.autotune(reps=3)
    log(f"[bench] config: {plan.describe()}")
    sched = "auto" if args.schedule == "auto" else args.schedule
    # the timed steps replay one captured hipGraph of the whole device pass
    plan.graph_create(sched, stream)
    for _ in range(args.warmup):
        plan.graph_launch(stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        plan.graph_launch(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    b, ub, _ = plan.results(0)
    # per-launch device time of the UTIL kernels, from events the library
    # records around each launch on the execute stream (eager runs)
    plan.set_timing(True)
    util_ms, kern_ms, value_ms = [], [], []
    for _ in range(min(args.steps, 10)):
        plan.execute(schedule=None if sched == "auto" else sched, stream=stream)
        plan.results(0)
        u, k, v = plan.last_timing()
        util_ms.append(u)
        kern_ms.append(k)
        value_ms.append(v)
    plan.set_timing(False)
    util_avg = sum(util_ms) / len(util_ms)
    kern_avg = sum(kern_ms) / len(kern_ms)
    value_avg = sum(value_ms) / len(value_ms)
    rows = st.util_rows
    value = rows / (ms_per_step * 1e-3)
    achieved = st.algo_bytes / (kern_avg * 1e-3) / 1e9
    out = {
        "metric": "UTIL entries/s",
        "value": value,
        "unit": "UTIL entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wname, "instances": batch, "algo": opts["algo"], "ibound": opts["ibound"],
                   "order": opts["order"], "schedule": plan.describe(), "seed0": args.seed,
                   "minibuckets": st.n_minibuckets, "levels": st.n_levels},
        "joint_entries_per_s": st.joint_entries / (ms_per_step * 1e-3),
        "util_phase_ms": util_avg,
        "util_kernels_ms": kern_avg,
        "util_launches_per_step": st.n_levels,
        "value_phase_ms": value_avg,
        "algo_bytes_per_step": st.algo_bytes,
        "hbm_GBps_step": st.algo_bytes / (ms_per_step * 1e-3) / 1e9,
        "plan_ms": plan_ms,
        "upload_ms": upload_ms,
        "bound": b,
        "ub": ub,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": None,
    }
    if args.compare_per_bucket:
        plan.execute(schedule="per-bucket")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(max(1, args.steps // 4)):
            plan.execute(schedule="per-bucket")
        e1.record(stream)
        torch.cuda.synchronize()
        pb_ms = e0.elapsed_time(e1) / max(1, args.steps // 4)
        out["per_bucket_ms_per_step"] = pb_ms
        out["per_bucket_entries_per_s"] = rows / (pb_ms * 1e-3)
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        done_rows = 0
        n = 0
        for inst in insts:
            o, _ = oracle.order(inst, opts["order"])
            res = oracle.solve(inst, o, opts["ibound"], keep_tables=False)
            done_rows += sum(int(_rows(inst, mb)) for mb in res.minibuckets)
            n += 1
            if time.perf_counter() - t0 > args.cpu_budget:
                break
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done_rows / dt, "unit": "UTIL entries/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{n} of {batch} instance(s) of the same workload, order + "
                                         f"elimination + value assignment, single thread, {dt:.1f} s"}
    print(json.dumps(out), flush=True)


def _rows(inst, mb):
    r = 1
    for v in mb.out_scope:
        r *= int(inst.domains[int(v)])
    return r


if __name__ == "__main__":
    main()
