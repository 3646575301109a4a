"""Learned mini-bucket partitions: training data, training and evaluation of
the candidate-scoring network.

Mini-Bucket Elimination (Alg. 2) may split an over-full bucket in any way
whose mini-buckets respect the i-bound; every such split gives a valid lower
bound, but some give tighter bounds than others.  The planner offers up to
six candidate splits per over-full bucket, candidate 0 being the greedy rule
(functions by decreasing arity, first fit), and describes each by
bx_partition_num_features() numbers.

Labels come from the bounds MBE itself computes on the device.  For each
decision of the greedy run and each other candidate at it, the instance is
solved again with that one candidate forced (greedy everywhere else); the
label is the change of the lower bound in percent of the greedy bound
(candidate 0: 0).  The network, trained on the device by the library's own
forward / backward / Adam kernels, predicts that change; at planning time a
decision takes the best candidate whose predicted change exceeds the greedy
candidate's by more than a margin, else the greedy one.  The greedy run is
thus both the fallback and the judge: evaluation reports the learned bound
alone and the better of the two bounds ("judged"), which is valid because
both are lower bounds.

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
TRAIN_SEED0 = 100_000       # training instances: seeds from here
EVAL_SEED0 = 900_000        # held-out instances: seeds from here (disjoint)


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
    problems listed in `forced` ({problem: (k, c)}) and the greedy candidate
    everywhere else, recording every decision's candidate features."""

    def __init__(self, forced: Optional[Dict[int, Tuple[int, int]]] = None, record: bool = False):
        self.forced = forced or {}
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
            f = self.forced.get(p)
            if f is not None and f[0] == k:
                ch[d] = f[1]
        return ch


def run_bounds(problems: Sequence[Problem], ibound: int, chooser=None, model=None, margin: float = 0.0,
               stream=None):
    """Plan, execute and read back one batch; returns (lb, ub, plan seconds,
    device seconds, decisions, non-greedy decisions)."""
    import torch
    t0 = time.perf_counter()
    pl = Plan(list(problems), algo="mbe", ibound=ibound, chooser=chooser, model=model, margin=margin,
              stream=stream)
    t1 = time.perf_counter()
    pl.upload(stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pl.execute(stream=stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    lb = np.zeros(len(problems))
    ub = np.zeros(len(problems))
    for k in range(len(problems)):
        lb[k], ub[k], _ = pl.results(k, stream)
    dec, ng = pl.partition_stats()
    del pl
    return lb, ub, t1 - t0, t3 - t2, dec, ng


def _chunks(n: int, size: int):
    for a in range(0, n, size):
        yield a, min(n, a + size)


def make_labels(insts: Sequence[synth.Instance], ibound: int, chunk: int = 128, log=print):
    """Features X [N, F], labels y [N] (percent change of the lower bound
    against greedy), decision index g [N] and candidate index c [N]."""
    probs = [Problem.from_instance(i) for i in insts]
    lb_g = np.zeros(len(probs))
    feats: Dict[Tuple[int, int], np.ndarray] = {}
    for a, b in _chunks(len(probs), chunk):
        rec = Forcing(record=True)
        lb, _, _, _, _, _ = run_bounds(probs[a:b], ibound, chooser=rec)
        lb_g[a:b] = lb
        for (p, k), f in rec.features.items():
            feats[(a + p, k)] = f
    variants = [(p, k, c) for (p, k), f in sorted(feats.items()) for c in range(1, f.shape[0])]
    log(f"[labels] {len(insts)} instances, {len(feats)} decisions, {len(variants)} variants")
    lb_v = np.zeros(len(variants))
    for a, b in _chunks(len(variants), chunk):
        sub = variants[a:b]
        forced = {j: (k, c) for j, (_, k, c) in enumerate(sub)}
        lb, _, _, _, _, _ = run_bounds([probs[p] for p, _, _ in sub], ibound, chooser=Forcing(forced))
        lb_v[a:b] = lb
        if (a // chunk) % 20 == 0:
            log(f"[labels] variants {b}/{len(variants)}")
    X, y, g, c_ = [], [], [], []
    dec_id = {key: i for i, key in enumerate(sorted(feats))}
    for (p, k), f in sorted(feats.items()):
        X.append(f[0]); y.append(0.0); g.append(dec_id[(p, k)]); c_.append(0)
    for (p, k, c), lv in zip(variants, lb_v):
        X.append(feats[(p, k)][c])
        y.append(100.0 * (lv - lb_g[p]) / max(1.0, abs(lb_g[p])))
        g.append(dec_id[(p, k)]); c_.append(c)
    return (np.asarray(X, np.float32).reshape(-1, partition_num_features()), np.asarray(y, np.float32),
            np.asarray(g, np.int64), np.asarray(c_, np.int64))


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


def realised_gain(pred: np.ndarray, y: np.ndarray, g: np.ndarray, c: np.ndarray, margin: float):
    """Sum over decisions of the label of the candidate a chooser with this
    margin takes (0 where it keeps the greedy candidate), and the number of
    non-greedy choices."""
    total, n = 0.0, 0
    order = np.argsort(g, kind="stable")
    gs, starts = np.unique(g[order], return_index=True)
    bounds = list(starts) + [len(order)]
    for k in range(len(gs)):
        idx = order[bounds[k]:bounds[k + 1]]
        p0 = pred[idx[c[idx] == 0][0]]
        j = int(np.argmax(pred[idx]))
        if pred[idx[j]] - p0 > margin:
            total += float(y[idx[j]])
            n += 1
    return total, n


def fit(X, y, g, c, epochs: int = 200, lr: float = 1e-3, val_frac: float = 0.2, seed: int = 0, log=print):
    """Trains on the decisions outside a held-out fraction, picks the margin
    with the best realised gain on the held-out decisions, then retrains on
    everything; returns the model (margin set) and a report."""
    import torch
    rng = np.random.default_rng(seed)
    dec = np.unique(g)
    val = set(rng.choice(dec, size=max(1, int(val_frac * len(dec))), replace=False).tolist())
    mv = np.array([k in val for k in g])
    model, hist = train(X[~mv], y[~mv], epochs=epochs, lr=lr, seed=seed, log=log)
    pred = model.infer_bf16(torch.from_numpy(np.ascontiguousarray(X[mv])).cuda()).cpu().numpy()
    table = {m: realised_gain(pred, y[mv], g[mv], c[mv], m) for m in MARGINS}
    oracle_gain = sum(max(0.0, float(y[mv][g[mv] == k].max())) for k in np.unique(g[mv]))
    best = max(MARGINS, key=lambda m: (table[m][0], -m))
    for m in MARGINS:
        log(f"[fit] margin {m}: held-out realised gain {table[m][0]:.2f} over {table[m][1]} choices "
            f"(best possible {oracle_gain:.2f})")
    model, hist = train(X, y, epochs=epochs, lr=lr, seed=seed, log=log)
    model.margin = best if table[best][0] > 0 else float("inf")
    return model, {"margin": model.margin, "val_gain": table[best][0], "val_best_possible": oracle_gain,
                   "first_mse": hist[0], "last_mse": hist[-1]}


def evaluate(model: PartitionMLP, insts: Sequence[synth.Instance], ibound: int, margin: Optional[float] = None,
             chunk: int = 128) -> dict:
    """Greedy against learned partitions on the same instances: lower bounds,
    upper bounds (cost of the assignment VALUE builds), gaps and times.
    `margin` defaults to the one chosen at training time."""
    if margin is None:
        margin = model.margin
    probs = [Problem.from_instance(i) for i in insts]
    n = len(probs)
    lg, ug, ll, ul = (np.zeros(n) for _ in range(4))
    tg = [0.0, 0.0]
    tl = [0.0, 0.0]
    dec = ng = 0
    for a, b in _chunks(n, chunk):
        lb, ub, tp, td, _, _ = run_bounds(probs[a:b], ibound)
        lg[a:b], ug[a:b] = lb, ub
        tg[0] += tp; tg[1] += td
        lb, ub, tp, td, d, g_ = run_bounds(probs[a:b], ibound, model=model, margin=margin)
        ll[a:b], ul[a:b] = lb, ub
        tl[0] += tp; tl[1] += td
        dec += d; ng += g_
    gain = 100.0 * (ll - lg) / np.maximum(1.0, np.abs(lg))
    judged_lb = np.maximum(lg, ll)
    best_ub = np.minimum(ug, ul)

    def gap(lb, ub):
        return float(np.mean((ub - lb) / np.maximum(1.0, ub)))
    return {
        "instances": n, "ibound": ibound, "margin": margin,
        "decisions": int(dec), "non_greedy": int(ng),
        "lb_gain_pct_mean": float(gain.mean()), "lb_gain_pct_median": float(np.median(gain)),
        "improved": int((ll > lg).sum()), "equal": int((ll == lg).sum()), "worse": int((ll < lg).sum()),
        "gap_greedy": gap(lg, ug), "gap_learned": gap(ll, ul), "gap_judged": gap(judged_lb, best_ub),
        "plan_s_greedy": tg[0], "device_s_greedy": tg[1],
        "plan_s_learned": tl[0], "device_s_learned": tl[1],
        "lb_greedy_sum": float(lg.sum()), "lb_learned_sum": float(ll.sum()),
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
    args = ap.parse_args(argv)
    if args.cmd == "train":
        import os
        if args.labels and os.path.exists(args.labels):
            z = np.load(args.labels)
            X, y, g, c = z["X"], z["y"], z["g"], z["c"]
            _log(f"[labels] loaded {X.shape[0]} rows from {args.labels}")
        else:
            t0 = time.perf_counter()
            insts = family(args.instances, TRAIN_SEED0)
            _log(f"[family] {len(insts)} instances in {time.perf_counter() - t0:.1f} s")
            t0 = time.perf_counter()
            X, y, g, c = make_labels(insts, args.ibound, log=_log)
            _log(f"[labels] {X.shape[0]} rows in {time.perf_counter() - t0:.1f} s; "
                 f"positive {int((y > 0).sum())}, zero {int((y == 0).sum())}, negative {int((y < 0).sum())}")
            if args.labels:
                np.savez(args.labels, X=X, y=y, g=g, c=c)
        model, rep = fit(X, y, g, c, epochs=args.epochs, lr=args.lr, log=_log)
        model.save(args.out)
        rep["rows"] = int(X.shape[0])
        _log(json.dumps(rep))
    else:
        model = PartitionMLP.load(args.weights)
        insts = family(args.instances, EVAL_SEED0)
        r = evaluate(model, insts, args.ibound, margin=args.margin)
        _log(json.dumps(r))
    return 0


if __name__ == "__main__":
    sys.exit(main())
