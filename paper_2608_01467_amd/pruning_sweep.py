"""Threshold-pruning sweep (Section V, QAOA): run time, fidelity and kept
histories against the threshold.

    python -m paper_2608_01467_amd.pruning_sweep [--workload qaoa_12v_p2]
        [--thresholds 0,1e-6,1e-4,1e-3] [--reps 3]

For each threshold t the batched evaluation (learned split: the cost
model's shortlist, timed on the workload) of every requested output is timed
by graph replay, and compared with t = 0:
  fidelity   F(t) = |sum_y conj(a_0(y)) a_t(y)|^2 / (sum |a_0|^2 sum |a_t|^2),
             0 when every amplitude is pruned;
  retained   sum |a_t|^2 / sum |a_0|^2;
  kept       valid histories (summed over outputs) at t over those at 0.
Prints one JSON object per threshold.  The paper defines neither the
fidelity nor the pruned quantity exactly; the reading used here is the one
the library implements (prune a history when the product of min(1, |U|)
over its branching factors falls below t).
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

from . import Context  # noqa: E402
from . import tune  # noqa: E402


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="qaoa_12v_p2")
    ap.add_argument("--thresholds", default="0,1e-6,1e-4,1e-3")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    cfg = w.CONFIGS[args.workload]()
    text = cfg["circuit"].to_text()
    ctx = Context(0)
    ctx.set_table_budget(32 << 30)
    launch = tune.model_launch()
    if launch is not None:
        ctx.set_launch_config(*launch)     # the configuration the cost model was trained under
    base = None
    for t in (float(x) for x in args.thresholds.split(",")):
        wl = tune.Workload(ctx, text, cfg["inputs"], [complex(*z) for z in cfg["coeffs"]],
                           cfg["outputs"], threshold=t)
        split, how = tune.choose(wl, tune.load_model(), reps=1, shortlist=5)
        sec = tune.time_split(wl, split, reps=args.reps)
        wl.run(split)
        torch.cuda.synchronize()
        a = wl.amps.cpu().numpy()
        amp = a[:, 0] + 1j * a[:, 1]
        valid = int(wl.stats.cpu().numpy()[:, 0].sum())
        if base is None:
            base = (amp, valid)
        a0, v0 = base
        n0, nt = float(np.sum(np.abs(a0) ** 2)), float(np.sum(np.abs(amp) ** 2))
        fid = 0.0 if nt == 0.0 else float(abs(np.vdot(a0, amp)) ** 2 / (n0 * nt))
        print(json.dumps({"workload": args.workload, "threshold": t, "split": list(split),
                          "launch_config": list(ctx.launch_config),
                          "split_mode": how, "ms_per_eval": sec * 1e3, "fidelity": fid,
                          "retained_norm": nt / n0 if n0 else 0.0, "norm": nt,
                          "valid_histories": valid, "kept_fraction": valid / v0 if v0 else 0.0,
                          "outputs": len(cfg["outputs"])}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
