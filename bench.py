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
(`roofline`, with the streaming copy / write / read rates the same device
reaches as `copy_ceiling`), the oracle on the host cores (`cpu_baseline`:
one thread, and every core over the instances) and, unless --no-extra, the
per-bucket schedule, one instance alone, the batched random-WCSP family,
DPOP, MPE and the learned partition.  --level-table FILE writes the per-level
bytes, device time and code paths of the timed workload.
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
    if name == "dcop":
        import paper_1608_05288_amd as bx

        def separators_fit(inst):
            try:
                p = bx.Plan([bx.Problem.from_instance(inst)], algo="dpop")
            except bx.BxError:
                return False
            return p.stats().max_scope - 1 <= 10
        insts = synth.accepted(lambda s: synth.dcop_candidate(s), batch, seed0, accept=separators_fit)
        return insts, dict(algo="dpop", ibound=0, order="min-fill"), \
            f"dpop_dcop_n25_d5_p0.3_sep10_x{batch}"
    if name == "bn":
        insts = [synth.bayes_net(seed0 + s) for s in range(batch)]
        return insts, dict(algo="mbe", ibound=20, order="min-fill"), \
            f"mpe_bn_n100_p3_dirichlet1_f32_mbe_i20_x{batch}"
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
TRAFFIC_SOURCES = ["bx_exec.hip", "bx_util_kernels.h", "bx_device.h", "bx_plan.cpp", "bx_internal.h"]


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


def copy_ceiling(bx, stream, nbytes=1 << 30, reps=5):
    """GB/s of the library's streaming copy / write / read kernels on buffers
    of `nbytes` (larger than the 256 MB last-level cache), best of reps."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for kind, moved in (("copy", 2 * nbytes), ("write", nbytes), ("read", nbytes)):
        best = 1e30
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            bx.stream_probe(kind, dst, src, nbytes, 0, stream)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[f"{kind}_GBps"] = moved / (best * 1e-3) / 1e9
    out["bytes"] = nbytes
    del src, dst
    torch.cuda.empty_cache()
    return out


def level_table(plan, path, title):
    """Per level: mini-buckets, tiles, code paths, rows, algorithmic bytes and
    the device time of the last timed execute."""
    ms = plan.level_timing()
    st = plan.stats()
    lines = [f"# {title}", "# level mbs tiles row_tiles blocked util_rows algo_bytes us TBps staged nt tile_goal"]
    tot_b = tot_ms = 0.0
    for lv in range(st.n_levels):
        li = plan.level_info(lv)
        t = ms[lv]
        tot_b += li.algo_bytes
        tot_ms += t
        lines.append(f"{lv:3d} {li.n_minibuckets:5d} {li.n_tiles:6d} {li.n_row_tiles:5d} {li.n_blocked:5d} "
                     f"{li.util_rows:11d} {li.algo_bytes:12d} {t * 1e3:9.2f} "
                     f"{(li.algo_bytes / (t * 1e-3) / 1e12) if t > 0 else 0:6.3f} {li.staged} {li.nontemporal} "
                     f"{li.tile_goal}")
    lines.append(f"# total {tot_b:.0f} bytes in {tot_ms * 1e3:.1f} us = {tot_b / (tot_ms * 1e-3) / 1e12:.3f} TB/s "
                 f"over {st.n_levels} levels")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    smt = None
    try:
        smt = open("/sys/devices/system/cpu/smt/active").read().strip() == "1"
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    # the job's CPU share, where the environment states one
    share = os.environ.get("OMP_NUM_THREADS", "")
    if share.isdigit() and int(share) > 0:
        cores = min(cores, int(share))
    return model, smt, cores


def _oracle_rows(args):
    """UTIL rows of one oracle solve (elimination + value assignment)."""
    inst, order, ibound = args
    import oracle
    res = oracle.solve(inst, order, ibound, keep_tables=False)
    return sum(int(_rows(inst, mb)) for mb in res.minibuckets)


def cpu_baseline(insts, opts, budget_s):
    """The oracle on the host: the elimination and value phases (the phases
    the device's timed region covers; orders computed beforehand), one thread
    on as many instances as fit `budget_s`, then every core of the job's CPU
    share over the instances (one process per core, one instance each)."""
    import multiprocessing as mp
    import oracle
    from concurrent.futures import ProcessPoolExecutor
    oracle.build(force=False)
    work = [(inst, oracle.order(inst, opts["order"])[0], opts["ibound"]) for inst in insts]
    t0 = time.perf_counter()
    rows1 = n1 = 0
    while n1 < len(work) and (n1 == 0 or time.perf_counter() - t0 < budget_s):
        rows1 += _oracle_rows(work[n1])
        n1 += 1
    dt1 = time.perf_counter() - t0
    model, smt, cores = cpu_info()
    per_inst = dt1 / n1
    n_all = min(len(work), max(cores, int(cores * budget_s / per_inst)))
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_rows, work[:1]))          # workers started and warm
        t0 = time.perf_counter()
        rows_all = sum(ex.map(_oracle_rows, work[:n_all]))
        dt_all = time.perf_counter() - t0
    return {"value": rows_all / dt_all, "unit": "UTIL entries/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_all} of {len(insts)} instances of the same workload, elimination + value "
                      f"assignment (orders computed beforehand), one instance per process on {cores} "
                      f"processes, {dt_all:.1f} s",
            "single_thread": {"value": rows1 / dt1, "cores": 1,
                              "sample": f"{n1} instance(s), one thread, {dt1:.1f} s"},
            "cpu_model": model, "smt": smt, "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid", choices=["grid", "batch", "dcop", "bn"])
    ap.add_argument("--batch", type=int, default=0, help="instances per step (0: workload default)")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the per-bucket, single-instance, batched-family and learned comparisons")
    ap.add_argument("--no-blocking", action="store_true",
                    help="plain one-row-per-slot loop everywhere (no register blocking)")
    ap.add_argument("--level-table", default="", metavar="FILE",
                    help="write the per-level table of the timed workload to FILE")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the streaming bandwidth reference")
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
    from paper_1608_05288_amd import synth  # noqa: F401  (workload generators)
    batch = args.batch or {"grid": 16, "batch": 256, "dcop": 1, "bn": 10}[args.workload]
    insts, opts, wname = make_workload(args.workload, batch, args.seed)
    # the host baseline runs first, before this process touches the GPU
    cpu = None if args.no_cpu else cpu_baseline(insts, opts, args.cpu_budget)
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
    if args.level_table:
        level_table(plan, args.level_table, f"{wname}: per-level UTIL launches, one eager timed step")
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
        "dtype": "f32" if args.workload == "bn" else "int32",
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
        "cpu_baseline": cpu,
    }
    if not args.no_ceiling:
        out["roofline"]["copy_ceiling"] = copy_ceiling(bx, stream)
        log(f"[bench] copy ceiling {out['roofline']['copy_ceiling']}")
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
    belief networks (100 binary variables, 3 parents, MBE i-bound 20), the
    sum-product variant (-ln Z) on the same networks, one grid instance in
    streamed execution (tables in host memory), branch and bound with the
    mini-bucket bound on small random WCSPs; and the
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
    # the sum-product variant on the same networks: a lower bound of -ln Z
    # (Z = 1 here, so the bound is <= 0)
    out["sum_bn"] = config_throughput(bx, stream, args, nets, dict(algo="mbe-sum", ibound=20, order="min-fill"),
                                      "logz_bn_n100_p3_dirichlet1_f32_mbe_sum_i20_x10")
    # streamed execution of one grid instance: every table in pinned host
    # memory, outputs computed in chunks copied out while the next chunk runs
    import paper_1608_05288_amd as bxm
    sp = bxm.Plan([bxm.Problem.from_instance(synth.grid_wcsp(args.seed))], algo="mbe", ibound=12, blocking=False)
    chunk = 1 << 20
    dbytes, hbytes = sp.stream_bytes(chunk)
    sp.execute_streamed(chunk, stream=stream)
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        sb = sp.execute_streamed(chunk, stream=stream)
    st_ms = (time.perf_counter() - t0) * 1e3 / reps
    out["streamed_grid"] = {"workload": "grid20x20_d4_mbe_i12_minfill_x1_streamed", "chunk_rows": chunk,
                            "device_bytes": dbytes, "resident_workspace_bytes": sp.workspace_bytes(),
                            "host_bytes": hbytes, "ms_per_pass": st_ms, "bound": float(sb[0]),
                            "pcie_bytes_per_pass": sp.stats().algo_bytes}
    log(f"[bench] streamed grid: {st_ms:.1f} ms per pass, device {dbytes / 2**20:.1f} MiB "
        f"of {sp.workspace_bytes() / 2**20:.1f} MiB")
    del sp
    # branch and bound with the mini-bucket bound recomputed at every node
    # (one batched device pass per expansion), 10 random WCSPs of 12
    # variables, domain 3, at i-bound 2
    t0 = time.perf_counter()
    nodes = passes = 0
    proved = True
    for s in range(10):
        _, _, st = bx.bnb_solve(bx.Problem.from_instance(synth.random_wcsp(args.seed + s)), ibound=2,
                                stream=stream)
        nodes += st["nodes"]
        passes += st["passes"]
        proved = proved and st["proved"]
    out["bnb_random_wcsp"] = {"workload": "random_wcsp_n12_d3_m20_bnb_mbe_i2_x10", "instances": 10,
                              "nodes": nodes, "device_passes": passes, "proved": proved,
                              "seconds": time.perf_counter() - t0}
    log(f"[bench] branch and bound: {nodes} nodes, {passes} passes, {time.perf_counter() - t0:.2f} s")
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
        held = learn.family(256, learn.EVAL_SEED0)
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
