"""Collect split timings with the autotuner and train the cost model.

    python -m paper_2608_01467_amd.train_cost_model [--out DIR]

Times every candidate split near the Eq. (8) optimum (plus a few far ones)
on a set of training circuits drawn from the paper's families, with output
counts sized so that one evaluation is about 2e11 algorithmic int32 ops, trains the network on the device, writes
paper_2608_01467_amd/cost_model.json and a JSON report of the data and of the
regret on held-out circuits (exhaustive best vs model vs Eq. (8)).  Every
split is timed under one launch configuration (--launch; by default the
compiled consumer, whose modules are built in batches on host threads).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402

from . import Context, PART_EQ8, Program  # noqa: E402
from . import tune  # noqa: E402

TARGET_INT_OPS = 2e11      # algorithmic int32 ops per timed evaluation at the Eq. (8) split


def build(name: str, kw: dict, m_scale: float = 1.0):
    """(text, inputs, outputs) for one training or held-out case."""
    if name == "walk":
        c = w.quantum_walk(kw["n_pos"], kw["steps"])
        text = c.to_text()
        pool = lambda m: w.walk_outputs(kw["n_pos"], kw["steps"], m, seed=77)
    elif name == "qaoa":
        c = w.qaoa_maxcut(kw["nv"], kw["p"], kw.get("gseed", 401), kw.get("aseed", 402))[0]
        text = c.to_text()
        pool = lambda m: w.random_outputs(kw["nv"], min(m, 1 << kw["nv"]), seed=78)
    elif name == "aa":
        c = w.amplitude_amplification(kw["k"], kw["s"], 4, seed=kw.get("seed", 301))[0]
        text = c.to_text()
        pool = lambda m: w.random_outputs(c.n, min(m, 1 << c.n), seed=79)
    elif name == "clifford_t":
        c = w.random_clifford_t(kw["n"], kw["g"], seed=kw["seed"])
        text = c.to_text()
        pool = lambda m: w.random_outputs(kw["n"], min(m, 1 << kw["n"]), seed=80)
    else:
        raise ValueError(name)
    prog = Program(text)
    # int32 work per pair at the Eq. (8) split: prefix, root and suffix
    # evaluations (features 3, 5, 7 are their log2(1 + work)), folded
    # ladders included, so walks and gate-level circuits get similar times
    f = prog.split_features(*prog.choose_partition(PART_EQ8), 1, 1)
    per_pair = float(2 ** f[3] + 2 ** f[5] + 2 ** f[7])
    m = int(max(4, min(8192, round(m_scale * TARGET_INT_OPS / max(per_pair, 1.0)))))
    return text, [0], pool(m)


TRAIN = [
    ("walk", dict(n_pos=30, steps=12)), ("walk", dict(n_pos=60, steps=14)),
    ("walk", dict(n_pos=99, steps=16)), ("walk", dict(n_pos=80, steps=18)),
    ("walk", dict(n_pos=45, steps=17)),
    ("qaoa", dict(nv=8, p=2)), ("qaoa", dict(nv=10, p=2)), ("qaoa", dict(nv=12, p=1)),
    ("qaoa", dict(nv=10, p=2, gseed=7, aseed=8)),
    ("aa", dict(k=3, s=3)), ("aa", dict(k=4, s=2)), ("aa", dict(k=5, s=2)),
    ("clifford_t", dict(n=16, g=80, seed=5)), ("clifford_t", dict(n=24, g=120, seed=6)),
    ("walk", dict(n_pos=99, steps=18)), ("walk", dict(n_pos=50, steps=20)),
    ("qaoa", dict(nv=14, p=1)), ("qaoa", dict(nv=8, p=3)), ("qaoa", dict(nv=6, p=3)),
    ("aa", dict(k=6, s=2)), ("clifford_t", dict(n=20, g=100, seed=7)),
    ("clifford_t", dict(n=12, g=60, seed=9)),
    ("clifford_t", dict(n=18, g=90, seed=21)), ("clifford_t", dict(n=22, g=110, seed=22)),
    ("clifford_t", dict(n=14, g=70, seed=23)), ("qaoa", dict(nv=12, p=2, gseed=31, aseed=32)),
]
HELD_OUT = [
    ("walk", dict(n_pos=99, steps=20)), ("qaoa", dict(nv=12, p=2)), ("aa", dict(k=4, s=3)),
    ("walk", dict(n_pos=70, steps=19)), ("walk", dict(n_pos=40, steps=15)),
    ("qaoa", dict(nv=10, p=1, gseed=21, aseed=22)), ("aa", dict(k=3, s=4)),
    ("aa", dict(k=5, s=1)), ("clifford_t", dict(n=18, g=90, seed=11)),
    ("clifford_t", dict(n=16, g=80, seed=13)), ("clifford_t", dict(n=20, g=100, seed=14)),
]


def in_sample(blob, X, y, case, report) -> None:
    """Per training case: the measured time of the model's pick among the
    timed splits, against the best timed split and Eq. (8)'s split."""
    pred = tune.predict(blob, X)
    for k, entry in enumerate(report["train"]):
        idx = np.where(case == k)[0]
        t_best = float(np.exp(y[idx].min()))
        t_model = float(np.exp(y[idx[np.argmin(pred[idx])]]))
        entry["t_model"] = t_model
        entry["model_regret"] = t_model / t_best - 1.0
        if entry.get("t_eq8") is not None:
            entry["eq8_regret"] = entry["t_eq8"] / t_best - 1.0


def held_out(ctx, blob, args, report) -> None:
    for name, kw in HELD_OUT:
        text, ins, outs = build(name, kw, 1.0)
        wl = tune.Workload(ctx, text, ins, [1.0], outs)
        splits = tune.candidates(wl, max_cost_ratio=args.ratio, extra=0)
        r = tune.regret(wl, blob, splits, reps=3, log=lambda m: print(m, flush=True),
                        budget=args.heldout_budget)
        r["case"] = [name, kw]
        r["M"] = wl.M
        r["A"] = wl.prog.A
        report["held_out"].append(r)
        print(f"held-out {name} {kw}: best {r['best']} {r['t_best']*1e3:.2f} ms, model "
              f"({r['how']}) {r['model']} {r['t_model']*1e3:.2f} ms, shortlist "
              f"({r['how_shortlist']}) {r['shortlist']} {r['t_shortlist']*1e3:.2f} ms, eq8 "
              f"{r['eq8']} {r['t_eq8']*1e3:.2f} ms", flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "_build", "cost_model"))
    ap.add_argument("--epochs", type=int, default=4000)
    ap.add_argument("--ratio", type=float, default=16.0,
                    help="time every split whose Eq. (8) cost is within this factor of the best")
    ap.add_argument("--cases", type=int, default=len(TRAIN), help="use the first N training cases")
    ap.add_argument("--case-budget", type=float, default=30.0,
                    help="seconds of split timing per training case")
    ap.add_argument("--model-out", default=tune.MODEL_PATH)
    ap.add_argument("--heldout-budget", type=float, default=40.0,
                    help="seconds of exhaustive timing per held-out circuit (cheapest Eq. (8) first)")
    ap.add_argument("--evaluate", default=None,
                    help="skip training: measure the held-out regret of this saved model")
    ap.add_argument("--no-held-out", action="store_true",
                    help="train and save only (measure the regret later with --evaluate)")
    ap.add_argument("--launch", default="1,256,0,3",
                    help="launch configuration every split is timed under: histories per lane, "
                         "chunk, blocks per CU, dispatch (3: the compiled consumer)")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    ctx = Context(0)
    ctx.set_launch_config(*(int(v) for v in args.launch.split(",")))
    report = {"train": [], "held_out": []}
    if args.evaluate:
        blob = tune.load_model(args.evaluate)
        held_out(ctx, blob, args, report)
        with open(os.path.join(args.out, "report_held_out.json"), "w") as f:
            json.dump(report, f, indent=1, default=str)
        return 0
    Xs, ys, cid = [], [], []
    t0 = time.time()
    for name, kw in TRAIN[: args.cases]:
        last_m = None
        for scale, limit in ((1.0, None), (4.0, 48), (32.0, 16)):
            text, ins, outs = build(name, kw, scale)
            if len(outs) == last_m:
                continue            # the output count is capped: same workload again
            last_m = len(outs)
            wl = tune.Workload(ctx, text, ins, [1.0], outs)
            splits = tune.candidates(wl, max_cost_ratio=args.ratio, extra=6 if scale == 1.0 else 0,
                                     limit=limit)
            print(f"[{time.time()-t0:6.1f}s] {name} {kw} x{scale}: timing {len(splits)} splits",
                  flush=True)
            X, y, rows = tune.collect(wl, splits, log=lambda m: print(m, flush=True),
                                      budget=args.case_budget)
            Xs.append(X)
            ys.append(y)
            cid.append(np.full(len(y), len(report["train"])))
            best = min(rows, key=lambda r: r[1])
            eq8 = wl.prog.choose_partition(PART_EQ8)
            t_eq8 = dict(rows).get(eq8)
            report["train"].append({"case": [name, kw, scale], "M": wl.M, "A": wl.prog.A,
                                    "splits": len(rows), "best": best[0], "t_best": best[1],
                                    "eq8": eq8, "t_eq8": t_eq8})
            print(f"[{time.time()-t0:6.1f}s] {name} {kw} x{scale}: M={wl.M} A={wl.prog.A} "
                  f"{len(rows)} splits, best {best[0]} {best[1]*1e3:.2f} ms", flush=True)
    X = np.concatenate(Xs)
    y = np.concatenate(ys)
    case = np.concatenate(cid)
    np.savez(os.path.join(args.out, "dataset.npz"), features=X, log_seconds=y, case=case)
    blob, loss = tune.train(X, y, epochs=args.epochs, lr=3e-3)
    print(f"trained on {len(y)} rows, loss {loss:.4f}", flush=True)
    tune.save_model(blob, {"rows": int(len(y)), "loss": loss, "epochs": args.epochs,
                           "launch": args.launch,
                           "train": [[n, kw] for n, kw in TRAIN[: args.cases]]},
                    path=args.model_out)
    in_sample(blob, X, y, case, report)
    if not args.no_held_out:
        held_out(ctx, blob, args, report)
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1, default=str)
    return 0


if __name__ == "__main__":
    sys.exit(main())
