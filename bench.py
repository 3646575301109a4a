#!/usr/bin/env python3
"""Benchmark of the UTIL-table engine on one MI355X.

Workload (default): 20x20 grid WCSP, domain 4, unary + 4-neighbour binary
int32 costs uniform in [0, 1000], Mini-Bucket Elimination at i-bound 12
(tables up to 4^12 entries), min-fill order; synthetic, seeded.  One step is
one device pass of the whole path -- every UTIL table (fused aggregate +
min-project), the bound, the value assignment and its cost -- with the plan
built and the inputs resident in HBM before the timed region.

Prints one JSON line: the throughput (UTIL rows per second), the UTIL
phase's algorithmic bytes over its kernel time against the HBM peak
(`roofline`), the oracle on the host cores (`cpu_baseline`) and, unless
--no-extra, the per-bucket schedule, one instance alone, the batched
random-WCSP family and the learned partition.
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


def time_graph(plan, stream, sched, steps, warmup):
    """ms per step of one captured hipGraph of the whole device pass."""
    import torch
    plan.graph_create(sched, stream)
    for _ in range(warmup):
        plan.graph_launch(stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.graph_launch(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def prepare(bx, insts, opts, stream, schedule="auto", tune=True, blocking=True):
    import torch
    t0 = time.perf_counter()
    plan = bx.Plan([bx.Problem.from_instance(i) for i in insts], schedule=schedule, blocking=blocking, **opts)
    plan_ms = (time.perf_counter() - t0) * 1e3
    plan.allocate()
    t0 = time.perf_counter()
    plan.upload(stream)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t0) * 1e3
    if tune and schedule == "auto":
        plan.autotune(reps=3)
    return plan, plan_ms, upload_ms


# the sources that fix the UTIL kernels' memory traffic: the kernels and the
# planner that lays out tables, tiles and their order
TRAFFIC_SOURCES = ["bx_exec.hip", "bx_plan.cpp", "bx_internal.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1608_05288_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_from_profile():
    """HBM bytes per UTIL launch measured by hardware counters, from the
    committed counter summary, if it was taken on these kernel and planner
    sources."""
    path = os.path.join(ROOT, "profiles", "util_tiles_grid20x20_x16_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src_hash = kernel_source_hash()
    if vals.get("kernel_source_sha256", "").split(" ")[0] != src_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the per-bucket, single-instance, batched-family and learned comparisons")
    ap.add_argument("--no-blocking", action="store_true",
                    help="plain one-row-per-slot loop everywhere (no register blocking)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="first run one device-to-device copy of MB MiB (a reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; --gpus must be 1 "
                          "(sharding over several GPUs is not built)"}))
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
    # a non-default stream (graph capture needs one), made current so every
    # library call below runs on it
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    batch = args.batch or (16 if args.workload == "grid" else 256)
    insts, opts, wname = make_workload(args.workload, batch, args.seed)
    plan, plan_ms, upload_ms = prepare(bx, insts, opts, stream, args.schedule, blocking=not args.no_blocking)
    st = plan.stats()
    log(f"[bench] workload={wname} mbs={st.n_minibuckets} rows={st.util_rows} joint={st.joint_entries} "
        f"levels={st.n_levels} algo_bytes={st.algo_bytes} plan_ms={plan_ms:.1f} upload_ms={upload_ms:.1f}")
    log(f"[bench] config: {plan.describe()}")
    sched = "auto" if args.schedule == "auto" else args.schedule
    ms_per_step = time_graph(plan, stream, sched, args.steps, args.warmup)
    log(f"[bench] {ms_per_step:.3f} ms/step")
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
    launches = st.n_levels
    traffic = traffic_from_profile()
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
        "util_launches_per_step": launches,
        "value_phase_ms": value_avg,
        "algo_bytes_per_step": st.algo_bytes,
        "algo_bytes_per_launch": st.algo_bytes / launches,
        "hbm_GBps_step": st.algo_bytes / (ms_per_step * 1e-3) / 1e9,
        "plan_ms": plan_ms,
        "upload_ms": upload_ms,
        "bound": b,
        "ub": ub,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": None,
    }
    if not args.no_extra:
        # the same batch, one launch per mini-bucket (the plain method)
        plan.execute(schedule="per-bucket", stream=stream)
        torch.cuda.synchronize()
        pb_ms = time_graph(plan, stream, "per-bucket", max(2, args.steps // 4), 1)
        out["per_bucket_ms_per_step"] = pb_ms
        out["batched_speedup_vs_per_bucket"] = pb_ms / ms_per_step
        log(f"[bench] per-bucket {pb_ms:.3f} ms/step")
        del plan
        # the same batch without register blocking (one row per slot)
        if not args.no_blocking:
            p0, _, _ = prepare(bx, insts, opts, stream, blocking=False)
            nb_ms = time_graph(p0, stream, "auto", args.steps, args.warmup)
            out["no_blocking_ms_per_step"] = nb_ms
            log(f"[bench] without register blocking {nb_ms:.3f} ms/step")
            del p0
        # one instance of the configuration alone
        p1, _, _ = prepare(bx, insts[:1], opts, stream)
        out["single_instance_ms_per_step"] = time_graph(p1, stream, "auto", args.steps, args.warmup)
        del p1
        out["extra"] = extra_comparisons(bx, stream, args)
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


def config_throughput(bx, stream, args, insts, opts, name):
    """Device throughput of one more configuration (autotuned level schedule,
    hipGraph replay)."""
    plan, plan_ms, _ = prepare(bx, insts, opts, stream)
    st = plan.stats()
    ms = time_graph(plan, stream, "auto", args.steps, args.warmup)
    r = {"workload": name, "instances": len(insts), "minibuckets": st.n_minibuckets, "levels": st.n_levels,
         "util_rows": st.util_rows, "algo_bytes": st.algo_bytes, "plan_ms": plan_ms, "ms_per_step": ms,
         "entries_per_s": st.util_rows / (ms * 1e-3), "GBps_step": st.algo_bytes / (ms * 1e-3) / 1e9,
         "bound": plan.results(0)[0], "schedule": plan.describe()}
    log(f"[bench] {name}: {ms:.3f} ms/step, {r['GBps_step']:.0f} GB/s")
    del plan
    return r


def extra_comparisons(bx, stream, args):
    """The batched random-WCSP family (256 instances, i-bound 10): one launch
    per level against one per mini-bucket; single-GPU DPOP on a random DCOP
    (25 agents, domain 5, density 0.3, separators <= 10) and FP32 MPE on random
    belief networks (100 binary variables, 3 parents, MBE i-bound 20); and the
    trained partition network against the greedy partition on held-out
    instances at i-bound 14."""
    from paper_1608_05288_amd import synth
    out = {}

    def separators_fit(inst):
        try:
            p = bx.Plan([bx.Problem.from_instance(inst)], algo="dpop")
        except bx.BxError:
            return False
        return p.stats().max_scope - 1 <= 10
    dcop = synth.accepted(lambda s: synth.dcop_candidate(s), 1, args.seed, accept=separators_fit)
    out["dpop_dcop"] = config_throughput(bx, stream, args, dcop, dict(algo="dpop", ibound=0, order="min-fill"),
                                         f"dpop_dcop_n25_d5_p0.3_sep10_seed{dcop[0].seed}")
    nets = [synth.bayes_net(args.seed + s) for s in range(10)]
    out["mpe_bn"] = config_throughput(bx, stream, args, nets, dict(algo="mbe", ibound=20, order="min-fill"),
                                      "mpe_bn_n100_p3_dirichlet1_f32_mbe_i20_x10")
    insts, opts, wname = make_workload("batch", 256, args.seed)
    plan, plan_ms, _ = prepare(bx, insts, opts, stream)
    st = plan.stats()
    lv = time_graph(plan, stream, "auto", args.steps, args.warmup)
    pb = time_graph(plan, stream, "per-bucket", max(2, args.steps // 4), 1)
    out["batched_family"] = {"workload": wname, "minibuckets": st.n_minibuckets, "levels": st.n_levels,
                             "util_rows": st.util_rows, "algo_bytes": st.algo_bytes, "plan_ms": plan_ms,
                             "level_ms_per_step": lv, "per_bucket_ms_per_step": pb,
                             "entries_per_s": st.util_rows / (lv * 1e-3),
                             "GBps_step": st.algo_bytes / (lv * 1e-3) / 1e9, "speedup": pb / lv,
                             "schedule": plan.describe()}
    log(f"[bench] batched family: level {lv:.3f} ms, per-bucket {pb:.3f} ms")
    del plan
    weights = os.path.join(ROOT, "paper_1608_05288_amd", "weights", "partition_mlp.npz")
    if os.path.exists(weights):
        from paper_1608_05288_amd import learn
        model = bx.PartitionMLP.load(weights)
        held = learn.family(64, learn.EVAL_SEED0)
        r = learn.evaluate(model, held, 14)
        out["learned_partition"] = r
        out["learned_partition_4_rounds"] = learn.evaluate(model, held, 14, passes=4)
        log(f"[bench] learned: gain {r['lb_gain_pct_mean']:.4f}% improved {r['improved']} worse {r['worse']}")
    return out


def _rows(inst, mb):
    r = 1
    for v in mb.out_scope:
        r *= int(inst.domains[int(v)])
    return r


if __name__ == "__main__":
    main()
