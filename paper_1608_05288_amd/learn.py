"""Learned mini-bucket partitions: training data, training and evaluation of
the candidate-scoring network.

Mini-Bucket Elimination (Alg. 2) may split an over-full bucket in any way
whose mini-buckets respect the i-bound; every such split gives a valid lower
bound, but some give tighter bounds than others.  The planner offers up to
six candidate splits per over-full bucket, candidate 0 being the greedy rule
(functions by decreasing arity, first fit), and describes each by
bx_partition_num_features() structural numbers (and their difference to the
greedy candidate).

Two passes, the greedy run being both the fallback and the judge:
  1. the greedy plan is built (recording every decision's candidates) and
     executed; bx_plan_candidate_values then estimates, on its tables, what
     each candidate would keep of the bound at its bucket (a sampled
     sum_k min_x sum_{f in part k} f);
  2. the network scores every candidate from the structural features and the
     sampled values; per problem, the best-scoring single deviation from the
     greedy plan, if it beats the greedy candidate of its decision by more
     than a margin, is planned and executed (the "learned" bound).  The
     "judged" bound keeps a deviation only where it raised the bound -- valid
     because every bound computed is a lower bound.  Further rounds
     (`passes`) propose one more deviation on each problem's current plan,
     again kept only if it raises the bound.

Labels come from the bounds MBE itself computes on the device: for each
decision of the greedy run and each other candidate at it, the instance is
solved again with that one candidate forced (greedy everywhere else); the
label is the change of the lower bound in percent of the greedy bound
(candidate 0: 0).  Training runs on the device in the library's own forward /
backward / Adam kernels; the margin is chosen on held-out problems.

Command line (on a GPU):
    python -m paper_1608_05288_amd.learn train --instances 10000 --ibound 14 --out W.npz
    python -m paper_1608_05288_amd.learn evaluate --weights W.npz --instances 256 --ibound 14
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import PartitionMLP, Plan, Problem, partition_num_features
from . import synth

CLIP = 3.0                  # labels are clipped to +-3 percent for training
MARGINS = (0.0, 0.02, 0.05, 0.1, 0.15, 0.2, 0.3, 0.5)
SAMPLES = 256               # samples per decision for the candidate values
N_LOCAL = 2                 # features from the candidate values
TRAIN_SEED0 = 100_000       # training instances: seeds from here
EVAL_SEED0 = 900_000        # held-out instances: seeds from here (disjoint)


def n_features() -> int:
    return partition_num_features() + N_LOCAL


def family(count: int, seed0: int, w_lo: int = 8, w_hi: int = 16) -> List[synth.Instance]:
    """Instances of the uneven random-WCSP family (30-80 variables, domains
    2-4, unary + binary costs in [0, 100]) whose min-fill induced width lies
    in [w_lo, w_hi]."""
    def ok(inst):
        p = Problem.from_instance(inst)
        o, _ = p.compute_order("min-fill")
        return w_lo <= p.induced_width(o) <= w_hi
    return synth.accepted(synth.batch_candidate, count, seed0, accept=ok)


class Forcing:
    """Partition chooser that takes candidate c at the k-th decision of the
    problems listed in `forced` ({problem: (k, c)} or {problem: {k: c, ...}})
    and the greedy candidate everywhere else, recording every decision's
    candidate features."""

    def __init__(self, forced=None, record: bool = False):
        self.forced: Dict[int, Dict[int, int]] = {}
        for p, f in (forced or {}).items():
            self.forced[p] = dict([f]) if isinstance(f, tuple) else dict(f)
        self.count: Dict[int, int] = {}
        self.record = record
        self.features: Dict[Tuple[int, int], np.ndarray] = {}

    def __call__(self, n, dec_prob, off, feats):
        ch = np.zeros(n, np.int32)
        for d in range(n):
            p = int(dec_prob[d])
            k = self.count.get(p, 0)
            self.count[p] = k + 1
            if self.record:
                self.features[(p, k)] = feats[off[d]:off[d + 1]].copy()
            c = self.forced.get(p, {}).get(k)
            if c is not None and c < off[d + 1] - off[d]:
                ch[d] = c
        return ch


def _sync():
    import torch
    torch.cuda.synchronize()


def run_bounds(problems: Sequence[Problem], ibound: int, chooser=None, stream=None):
    """Plan, execute and read back one batch; returns (lb, ub, plan seconds,
    device seconds)."""
    t0 = time.perf_counter()
    pl = Plan(list(problems), algo="mbe", ibound=ibound, chooser=chooser, stream=stream)
    t1 = time.perf_counter()
    pl.upload(stream)
    _sync()
    t2 = time.perf_counter()
    pl.execute(stream=stream)
    _sync()
    t3 = time.perf_counter()
    lb = np.zeros(len(problems))
    ub = np.zeros(len(problems))
    for k in range(len(problems)):
        lb[k], ub[k], _ = pl.results(k, stream)
    del pl
    return lb, ub, t1 - t0, t3 - t2


def greedy_pass(problems: Sequence[Problem], ibound: int, seed: int = 0, samples: int = SAMPLES, forced=None):
    """Pass 1: the greedy plan (with the `forced` deviations, if any),
    executed, with every decision's candidates described.  Returns (lb, ub,
    rows, seconds) where rows lists (problem, k-th decision of that problem,
    features [n_cands, n_features()])."""
    import torch
    t0 = time.perf_counter()
    rec = Forcing(forced, record=True)
    pl = Plan(list(problems), algo="mbe", ibound=ibound, chooser=rec)
    pl.upload()
    pl.execute()
    lb = np.zeros(len(problems))
    ub = np.zeros(len(problems))
    for k in range(len(problems)):
        lb[k], ub[k], _ = pl.results(k)
    decs = pl.decisions()
    rows = []
    if decs:
        rng = np.random.default_rng(seed)
        rnd = rng.integers(0, 2**32, (len(decs), samples, 32), dtype=np.uint64).astype(np.uint32)
        vals = pl.candidate_values(torch.from_numpy(rnd.view(np.int32)).cuda()).cpu().numpy()
        count: Dict[int, int] = {}
        off = 0
        for d in decs:
            p = d["prob"]
            k = count.get(p, 0)
            count[p] = k + 1
            v = vals[off:off + d["n_cands"]]
            off += d["n_cands"]
            loc = np.stack([100.0 * (v - v[0]) / max(1.0, abs(lb[p])),
                            (v - v[0]) / max(1.0, abs(v[0]))], 1)
            loc = np.nan_to_num(loc, nan=0.0, posinf=0.0, neginf=0.0)
            rows.append((p, k, np.concatenate([rec.features[(p, k)], loc], 1).astype(np.float32)))
    _sync()
    del pl
    return lb, ub, rows, time.perf_counter() - t0


def _chunks(n: int, size: int):
    for a in range(0, n, size):
        yield a, min(n, a + size)


def make_labels(insts: Sequence[synth.Instance], ibound: int, chunk: int = 128, log=print):
    """Features X [N, F], labels y [N] (percent change of the lower bound
    against greedy), decision index g [N], candidate index c [N] and problem
    index p [N]."""
    probs = [Problem.from_instance(i) for i in insts]
    lb_g = np.zeros(len(probs))
    feats: Dict[Tuple[int, int], np.ndarray] = {}
    for a, b in _chunks(len(probs), chunk):
        lb, _, rows, _ = greedy_pass(probs[a:b], ibound, seed=a)
        lb_g[a:b] = lb
        for p, k, f in rows:
            feats[(a + p, k)] = f
    variants = [(p, k, c) for (p, k), f in sorted(feats.items()) for c in range(1, f.shape[0])]
    log(f"[labels] {len(insts)} instances, {len(feats)} decisions, {len(variants)} variants")
    lb_v = np.zeros(len(variants))
    for a, b in _chunks(len(variants), chunk):
        sub = variants[a:b]
        forced = {j: (k, c) for j, (_, k, c) in enumerate(sub)}
        lb, _, _, _ = run_bounds([probs[p] for p, _, _ in sub], ibound, chooser=Forcing(forced))
        lb_v[a:b] = lb
        if (a // chunk) % 20 == 0:
            log(f"[labels] variants {b}/{len(variants)}")
    X, y, g, c_, p_ = [], [], [], [], []
    dec_id = {key: i for i, key in enumerate(sorted(feats))}
    for (p, k), f in sorted(feats.items()):
        X.append(f[0]); y.append(0.0); g.append(dec_id[(p, k)]); c_.append(0); p_.append(p)
    for (p, k, c), lv in zip(variants, lb_v):
        X.append(feats[(p, k)][c])
        y.append(100.0 * (lv - lb_g[p]) / max(1.0, abs(lb_g[p])))
        g.append(dec_id[(p, k)]); c_.append(c); p_.append(p)
    return (np.asarray(X, np.float32).reshape(-1, n_features()), np.asarray(y, np.float32),
            np.asarray(g, np.int64), np.asarray(c_, np.int64), np.asarray(p_, np.int64))


def train(X: np.ndarray, y: np.ndarray, epochs: int = 200, batch: int = 512, lr: float = 1e-3, seed: int = 0,
          log=print) -> Tuple[PartitionMLP, List[float]]:
    """Trains a fresh network on (X, y) with minibatch Adam on the mean
    squared error (labels clipped to +-CLIP percent); returns the model and
    the loss of each epoch over the whole set."""
    import torch
    y = np.clip(y, -CLIP, CLIP)
    model = PartitionMLP(X.shape[1], seed=seed)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(X.shape[0], generator=gen).cuda()
        for a in range(0, X.shape[0], batch):
            idx = perm[a:a + batch]
            model.train_step(Xd[idx].contiguous(), yd[idx].contiguous(), lr=lr)
        y_all, _ = model.forward(Xd)
        loss, _ = model.mse(y_all, yd)
        hist.append(float(loss))
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            log(f"[train] epoch {ep} mse {hist[-1]:.5f}")
    model.pack_bf16()
    return model, hist


def choose(pred: np.ndarray, g: np.ndarray, c: np.ndarray, p: np.ndarray, margin: float):
    """Per problem, the row of the best single deviation: the candidate whose
    score exceeds the greedy candidate of its decision by the most, if by
    more than `margin`.  Returns {problem: row index}."""
    base = {}
    for i in range(len(g)):
        if c[i] == 0:
            base[int(g[i])] = pred[i]
    best: Dict[int, Tuple[float, int]] = {}
    for i in range(len(g)):
        if c[i] == 0:
            continue
        gain = float(pred[i] - base[int(g[i])])
        if gain > margin and (int(p[i]) not in best or gain > best[int(p[i])][0]):
            best[int(p[i])] = (gain, i)
    return {k: v[1] for k, v in best.items()}


def realised_gain(pred, y, g, c, p, margin: float):
    """Sum over problems of the label of the deviation `choose` takes, and
    the number of deviations."""
    ch = choose(pred, g, c, p, margin)
    return float(sum(y[i] for i in ch.values())), len(ch)


def fit(X, y, g, c, p, epochs: int = 200, lr: float = 1e-3, val_frac: float = 0.2, seed: int = 0, log=print):
    """Trains on the problems outside a held-out fraction, picks the margin
    with the best realised gain on the held-out problems, then retrains on
    everything; returns the model (margin set) and a report."""
    import torch
    rng = np.random.default_rng(seed)
    probs = np.unique(p)
    val = set(rng.choice(probs, size=max(1, int(val_frac * len(probs))), replace=False).tolist())
    mv = np.array([k in val for k in p])
    model, hist = train(X[~mv], y[~mv], epochs=epochs, lr=lr, seed=seed, log=log)
    pred = model.infer_bf16(torch.from_numpy(np.ascontiguousarray(X[mv])).cuda()).cpu().numpy()
    table = {m: realised_gain(pred, y[mv], g[mv], c[mv], p[mv], m) for m in MARGINS}
    best_possible = sum(max(0.0, float(y[mv][p[mv] == k].max())) for k in np.unique(p[mv]))
    best = max(MARGINS, key=lambda m: (table[m][0], -m))
    for m in MARGINS:
        log(f"[fit] margin {m}: held-out realised gain {table[m][0]:.2f} over {table[m][1]} deviations "
            f"(best possible {best_possible:.2f})")
    model, hist = train(X, y, epochs=epochs, lr=lr, seed=seed, log=log)
    model.margin = best if table[best][0] > 0 else float("inf")
    return model, {"margin": model.margin, "val_gain": table[best][0], "val_best_possible": best_possible,
                   "first_mse": hist[0], "last_mse": hist[-1]}


def _deviations(model, rows, margin, fixed, tried):
    """Per problem, the best-scoring deviation (k, c) at a decision not yet
    fixed and not tried on the problem's current plan, if it beats the
    decision's greedy candidate by more than margin."""
    import torch
    rows = [(p, k, f) for p, k, f in rows if k not in fixed.get(p, {})]
    if not rows:
        return {}
    X = np.concatenate([f for _, _, f in rows])
    g = np.concatenate([np.full(f.shape[0], i) for i, (_, _, f) in enumerate(rows)])
    c = np.concatenate([np.arange(f.shape[0]) for _, _, f in rows])
    p = np.concatenate([np.full(f.shape[0], pp) for pp, _, f in rows])
    pred = model.infer_bf16(torch.from_numpy(X).cuda()).cpu().numpy()
    for i in range(len(pred)):
        if (int(p[i]), rows[int(g[i])][1], int(c[i])) in tried:
            pred[i] = -np.inf
    ch = choose(pred, g, c, p, margin)
    return {int(p[i]): (rows[int(g[i])][1], int(c[i])) for i in ch.values()}


def solve_learned(model: PartitionMLP, problems: Sequence[Problem], ibound: int,
                  margin: Optional[float] = None, seed: int = 0, passes: int = 1):
    """The greedy run, then `passes` rounds of network-chosen deviations on
    one batch.  Round 1 takes one deviation per problem and is reported as is
    (the learned bound).  Every round's deviation is kept only when it raises
    the problem's bound (the greedy run and the earlier rounds judge it); a
    later round proposes one more deviation on each problem's current plan.
    Returns (lb_greedy, ub_greedy, lb_learned, ub_learned, lb_judged,
    ub_judged, deviations of round 1, seconds of the greedy run, seconds of
    the rounds)."""
    if margin is None:
        margin = model.margin
    lb_g, ub_g, rows, t_greedy = greedy_pass(problems, ibound, seed=seed)
    lb_l, ub_l = lb_g.copy(), ub_g.copy()
    lb_f, ub_f = lb_g.copy(), ub_g.copy()
    t0 = time.perf_counter()
    base_rows: Dict[int, list] = {}
    for r in rows:
        base_rows.setdefault(r[0], []).append(r)
    fixed: Dict[int, Dict[int, int]] = {}          # kept deviations per problem
    tried = set()                                  # (problem, k, c) tried on its current plan
    n_dev1 = 0
    for it in range(passes):
        dev = _deviations(model, [r for q in sorted(base_rows) for r in base_rows[q]], margin, fixed, tried)
        if it == 0:
            n_dev1 = len(dev)
        if not dev:
            break
        idx = sorted(dev)
        trial = {j: {**fixed.get(q, {}), dev[q][0]: dev[q][1]} for j, q in enumerate(idx)}
        lb, ub, _, _ = run_bounds([problems[q] for q in idx], ibound, chooser=Forcing(trial))
        kept = []
        for j, q in enumerate(idx):
            tried.add((q, dev[q][0], dev[q][1]))
            if it == 0:
                lb_l[q], ub_l[q] = lb[j], ub[j]
            ub_f[q] = min(ub_f[q], ub[j])
            if lb[j] > lb_f[q]:
                fixed[q] = trial[j]
                lb_f[q] = lb[j]
                kept.append(q)
        if it + 1 < passes and kept:
            # new plans for the problems whose deviation was kept
            _, _, rows_k, _ = greedy_pass([problems[q] for q in kept], ibound, seed=seed + it + 1,
                                          forced={j: fixed[q] for j, q in enumerate(kept)})
            for q in kept:
                base_rows[q] = []
                tried = {t for t in tried if t[0] != q}
            for pp, k, f in rows_k:
                base_rows[kept[pp]].append((kept[pp], k, f))
    return lb_g, ub_g, lb_l, ub_l, lb_f, ub_f, n_dev1, t_greedy, time.perf_counter() - t0


def evaluate(model: PartitionMLP, insts: Sequence[synth.Instance], ibound: int, margin: Optional[float] = None,
             chunk: int = 128, passes: int = 1) -> dict:
    """Greedy against learned partitions on the same instances: lower bounds,
    upper bounds (cost of the assignment VALUE builds), gaps and times.
    `margin` defaults to the one chosen at training time; with passes > 1 the
    judged figures are those of the last round."""
    if margin is None:
        margin = model.margin
    probs = [Problem.from_instance(i) for i in insts]
    n = len(probs)
    lg, ug, ll, ul, jl, ju = (np.zeros(n) for _ in range(6))
    t1 = t2 = 0.0
    ndev = 0
    for a, b in _chunks(n, chunk):
        r = solve_learned(model, probs[a:b], ibound, margin, seed=a, passes=passes)
        lg[a:b], ug[a:b], ll[a:b], ul[a:b], jl[a:b], ju[a:b] = r[:6]
        ndev += r[6]
        t1 += r[7]
        t2 += r[8]
    gain = 100.0 * (ll - lg) / np.maximum(1.0, np.abs(lg))

    def gap(lb, ub):
        return float(np.mean((ub - lb) / np.maximum(1.0, ub)))
    return {
        "instances": n, "ibound": ibound, "margin": margin, "passes": passes, "deviations": int(ndev),
        "lb_gain_pct_mean": float(gain.mean()), "lb_gain_pct_median": float(np.median(gain)),
        "improved": int((ll > lg).sum()), "equal": int((ll == lg).sum()), "worse": int((ll < lg).sum()),
        "judged_improved": int((jl > lg).sum()),
        "judged_gain_pct_mean": float((100.0 * (jl - lg) / np.maximum(1.0, np.abs(lg))).mean()),
        "gap_greedy": gap(lg, ug), "gap_learned": gap(ll, ul), "gap_judged": gap(jl, ju),
        "seconds_greedy": t1, "seconds_learned_extra": t2,
        "lb_greedy_sum": float(lg.sum()), "lb_learned_sum": float(ll.sum()), "lb_judged_sum": float(jl.sum()),
    }


def _log(msg):
    print(msg, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--instances", type=int, default=10000)
    t.add_argument("--ibound", type=int, default=14)
    t.add_argument("--epochs", type=int, default=200)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", required=True)
    t.add_argument("--labels", default="", help="save / reuse the labelled set (npz)")
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", required=True)
    e.add_argument("--instances", type=int, default=256)
    e.add_argument("--ibound", type=int, default=14)
    e.add_argument("--margin", type=float, default=None)
    e.add_argument("--passes", type=int, default=1)
    args = ap.parse_args(argv)
    if args.cmd == "train":
        import os
        if args.labels and os.path.exists(args.labels):
            z = np.load(args.labels)
            X, y, g, c, p = z["X"], z["y"], z["g"], z["c"], z["p"]
            _log(f"[labels] loaded {X.shape[0]} rows from {args.labels}")
        else:
            t0 = time.perf_counter()
            insts = family(args.instances, TRAIN_SEED0)
            _log(f"[family] {len(insts)} instances in {time.perf_counter() - t0:.1f} s")
            t0 = time.perf_counter()
            X, y, g, c, p = make_labels(insts, args.ibound, log=_log)
            _log(f"[labels] {X.shape[0]} rows in {time.perf_counter() - t0:.1f} s; "
                 f"positive {int((y > 0).sum())}, zero {int((y == 0).sum())}, negative {int((y < 0).sum())}")
            if args.labels:
                np.savez(args.labels, X=X, y=y, g=g, c=c, p=p)
        model, rep = fit(X, y, g, c, p, epochs=args.epochs, lr=args.lr, log=_log)
        model.save(args.out)
        rep["rows"] = int(X.shape[0])
        _log(json.dumps(rep))
    else:
        model = PartitionMLP.load(args.weights)
        insts = family(args.instances, EVAL_SEED0)
        r = evaluate(model, insts, args.ibound, margin=args.margin, passes=args.passes)
        _log(json.dumps(r))
    return 0


if __name__ == "__main__":
    sys.exit(main())
