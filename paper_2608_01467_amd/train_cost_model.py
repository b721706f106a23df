"""Collect split timings with the autotuner and train the cost model.

    python -m paper_2608_01467_amd.train_cost_model [--out DIR]

Times every candidate split near the Eq. (8) optimum (plus a few far ones)
on a set of training circuits drawn from the paper's families at sizes that
take milliseconds per evaluation, trains the network on the device, writes
paper_2608_01467_amd/cost_model.json and a JSON report of the data and of the
regret on held-out circuits (exhaustive best vs model vs Eq. (8)).
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

TARGET_GATE_OPS = 1.5e10   # per timed evaluation at the Eq. (8) optimum


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
    best = min(prog.partition_cost(*x)[0] for x in prog.candidate_splits())
    m = int(max(4, min(8192, round(m_scale * TARGET_GATE_OPS / max(best, 1)))))
    return text, [0], pool(m)


TRAIN = [
    ("walk", dict(n_pos=30, steps=12)), ("walk", dict(n_pos=60, steps=14)),
    ("walk", dict(n_pos=99, steps=16)), ("walk", dict(n_pos=80, steps=18)),
    ("walk", dict(n_pos=45, steps=17)),
    ("qaoa", dict(nv=8, p=2)), ("qaoa", dict(nv=10, p=2)), ("qaoa", dict(nv=12, p=1)),
    ("qaoa", dict(nv=10, p=2, gseed=7, aseed=8)),
    ("aa", dict(k=3, s=3)), ("aa", dict(k=4, s=2)), ("aa", dict(k=5, s=2)),
    ("clifford_t", dict(n=16, g=80, seed=5)), ("clifford_t", dict(n=24, g=120, seed=6)),
]
HELD_OUT = [
    ("walk", dict(n_pos=99, steps=20)), ("qaoa", dict(nv=12, p=2)), ("aa", dict(k=4, s=3)),
    ("walk", dict(n_pos=70, steps=19)),
]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "gpurun_out", "cost_model"))
    ap.add_argument("--epochs", type=int, default=4000)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    ctx = Context(0)
    Xs, ys, report = [], [], {"train": [], "held_out": []}
    t0 = time.time()
    for name, kw in TRAIN:
        for scale in (1.0, 4.0):
            text, ins, outs = build(name, kw, scale)
            wl = tune.Workload(ctx, text, ins, [1.0], outs)
            splits = tune.candidates(wl, max_cost_ratio=64.0 if scale == 1.0 else 8.0,
                                     extra=8 if scale == 1.0 else 0)
            X, y, rows = tune.collect(wl, splits)
            Xs.append(X)
            ys.append(y)
            best = min(rows, key=lambda r: r[1])
            eq8 = wl.prog.choose_partition(PART_EQ8)
            report["train"].append({"case": [name, kw, scale], "M": wl.M, "A": wl.prog.A,
                                    "splits": len(rows), "best": best[0], "t_best": best[1],
                                    "eq8": eq8})
            print(f"[{time.time()-t0:6.1f}s] {name} {kw} x{scale}: M={wl.M} A={wl.prog.A} "
                  f"{len(rows)} splits, best {best[0]} {best[1]*1e3:.2f} ms", flush=True)
    X = np.concatenate(Xs)
    y = np.concatenate(ys)
    np.save(os.path.join(args.out, "features.npy"), X)
    np.save(os.path.join(args.out, "log_seconds.npy"), y)
    blob, loss = tune.train(X, y, epochs=args.epochs, lr=3e-3)
    print(f"trained on {len(y)} rows, loss {loss:.4f}", flush=True)
    tune.save_model(blob, {"rows": int(len(y)), "loss": loss, "epochs": args.epochs,
                           "train": [[n, kw] for n, kw in TRAIN]})
    for name, kw in HELD_OUT:
        text, ins, outs = build(name, kw, 1.0)
        wl = tune.Workload(ctx, text, ins, [1.0], outs)
        splits = tune.candidates(wl, max_cost_ratio=64.0, extra=0)
        r = tune.regret(wl, blob, splits)
        r["case"] = [name, kw]
        r["M"] = wl.M
        report["held_out"].append(r)
        print(f"held-out {name} {kw}: best {r['best']} {r['t_best']*1e3:.2f} ms, model "
              f"{r['model']} {r['t_model']*1e3:.2f} ms, eq8 {r['eq8']} {r['t_eq8']*1e3:.2f} ms",
              flush=True)
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1, default=str)
    return 0


if __name__ == "__main__":
    sys.exit(main())
