"""Where the time goes across outputs (Section V: time against the number of
artificial sources on the quantum walk; time per requested bitstring).

    python -m paper_2608_01467_amd.profile_items items [--workload walk_99p_20s]
    python -m paper_2608_01467_amd.profile_items sources [--steps 10-20]
    python -m paper_2608_01467_amd.profile_items choice --workload aa_k16_s3

`items`: one batched evaluation of the workload in timing mode at its
Eq. (8) split (or --cuts); the persistent consumer's per-item clock stamps
(fhs_item_stamps) give each output's cost (the summed durations of its
items), their distribution, and how well the atomic work queue kept the
workgroups busy: the makespan against the summed item time divided by the
number of resident workgroups (the most items in flight at once), and how
long the tail after the last moment at that count lasts.  `sources`: the
walk at 10..20 steps (A = s-1 sources) with the same output count,
consumer time per output and per candidate history against A.  One JSON line per result.  Everything here
drives the C ABI; no computation of the method happens in Python.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402

from . import PART_EQ8, Context, Program  # noqa: E402


def _quantiles(x: np.ndarray) -> dict:
    if x.size == 0:
        return {}
    q = np.quantile(x, [0.0, 0.1, 0.5, 0.9, 0.99, 1.0])
    return {"min": float(q[0]), "p10": float(q[1]), "median": float(q[2]), "p90": float(q[3]),
            "p99": float(q[4]), "max": float(q[5]), "mean": float(x.mean()),
            "cv": float(x.std() / x.mean()) if x.mean() > 0 else 0.0}


def _histogram(x: np.ndarray, bins: int = 12) -> list:
    """Counts over log-spaced bins between the smallest and largest value."""
    x = x[x > 0]
    if x.size == 0:
        return []
    lo, hi = float(x.min()), float(x.max())
    if hi <= lo:
        return [{"from": lo, "to": hi, "count": int(x.size)}]
    edges = np.geomspace(lo, hi * (1 + 1e-12), bins + 1)
    counts, _ = np.histogram(x, bins=edges)
    return [{"from": float(edges[i]), "to": float(edges[i + 1]), "count": int(c)}
            for i, c in enumerate(counts)]


def _concurrency(start: np.ndarray, end: np.ndarray) -> dict:
    """Items in flight over the launch: the most at once (the workgroups the
    device kept resident), the mean (summed item time over the makespan),
    and when the count first fell below its maximum for good (the tail)."""
    ev = np.concatenate([np.stack([start, np.ones_like(start)], 1),
                         np.stack([end, -np.ones_like(end)], 1)])
    ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]          # ends before starts at equal times
    live = np.cumsum(ev[:, 1])
    peak = int(live.max())
    t0, t1 = float(start.min()), float(end.max())
    last_peak = float(ev[np.nonzero(live == peak)[0][-1], 0])
    mean = float((end - start).sum()) / max(t1 - t0, 1.0)
    return {"max_in_flight": peak, "mean_in_flight": mean, "busy_frac": mean / peak if peak else 0.0,
            "tail_frac": (t1 - last_peak) / max(t1 - t0, 1.0)}


def timed_evaluation(ctx: Context, prog: Program, cfg: dict, cuts, launch=None, reps: int = 2):
    """Evaluate in timing mode; returns (consumer ms per launch, stamps,
    items per pair, ticks per second, amps, stats) of the last repetition."""
    import torch
    if launch is not None:
        ctx.set_launch_config(*launch)
    ctx.load(prog)
    ctx.set_partition(*cuts)
    d_in = ctx.device_bits(cfg["inputs"])
    d_out = ctx.device_bits(cfg["outputs"])
    d_cf = ctx.device_coeffs([complex(*z) for z in cfg["coeffs"]])
    M = len(cfg["outputs"])
    amps = torch.empty((M, 2), dtype=torch.float64, device="cuda:0")
    stats = torch.empty((M, 4), dtype=torch.int64, device="cuda:0")
    ctx.evaluate(d_in, d_cf, d_out, threshold=cfg["threshold"], out=(amps, stats))   # compile, warm up
    torch.cuda.synchronize()
    ctx.set_kernel_timing(True)
    for _ in range(reps):
        ctx.evaluate(d_in, d_cf, d_out, threshold=cfg["threshold"], out=(amps, stats))
        torch.cuda.synchronize()
    ms = ctx.kernel_times()
    stamps, ipp, tps = ctx.item_stamps()
    ctx.set_kernel_timing(False)
    return (sum(ms) / len(ms), stamps, ipp, tps, amps.cpu().numpy(),
            stats.cpu().numpy().view(np.uint64))


def items(args) -> int:
    cfg = w.CONFIGS[args.workload]()
    text = cfg["circuit"].to_text()
    prog = Program(text)
    ctx = Context(0)
    ctx.set_table_budget(32 << 30)
    cuts = tuple(int(v) for v in args.cuts.split(",")) if args.cuts else prog.choose_partition(PART_EQ8)
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    if args.claim is not None:
        launch = (launch or ctx.launch_config) + (args.claim,)
    ms, stamps, ipp, tps, _, st = timed_evaluation(ctx, prog, cfg, cuts, launch)
    S = len(cfg["inputs"])
    ran = stamps[:, 0] > 0                 # items of pairs the precheck rejected are skipped (stamps 0)
    start = stamps[:, 0].astype(np.int64)
    dur = np.where(ran, (stamps[:, 1].astype(np.int64) - start) / tps * 1e6, 0.0)   # microseconds
    per_out = dur.reshape(-1, S * ipp).sum(axis=1)                       # outputs x (inputs x items)
    leaves = st[:, 3].astype(np.float64)
    makespan = (stamps[ran, 1].max() - stamps[ran, 0].min()) / tps * 1e6 if ran.any() else 0.0
    plan = ctx.plan(len(cfg["outputs"]), S)
    lc = ctx.launch_config
    valid = st[:, 0] > 0
    line = {"workload": args.workload, "partition": list(cuts), "launch_config": list(lc),
            "items_per_claim": plan["items_per_claim"],
            "regions": [plan["Ap"], plan["Ar"], plan["As"]], "items": int(stamps.shape[0]),
            "items_skipped": int((~ran).sum()), "root_parts": plan["root_parts"],
            "pair_filter": plan["pair_filter"],
            "items_per_pair": ipp, "consumer_ms": ms, "makespan_us": float(makespan),
            "item_us": _quantiles(dur[ran]), "output_us": _quantiles(per_out),
            "output_us_histogram": _histogram(per_out),
            "output_us_valid": _quantiles(per_out[valid]),
            "output_us_no_valid_history": _quantiles(per_out[~valid]),
            "leaves_per_output": _quantiles(leaves),
            # the queue's balance: summed item time over the workgroups that
            # ran it, against the makespan
            "sum_item_us": float(dur.sum()),
            "in_flight": _concurrency(start[ran].astype(np.float64), stamps[ran, 1].astype(np.float64))}
    print(json.dumps(line), flush=True)
    return 0


def sources(args) -> int:
    lo, hi = (int(v) for v in args.steps.split("-"))
    ctx = Context(0)
    ctx.set_table_budget(32 << 30)
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else (2, 256, 0, 3)
    for s in range(lo, hi + 1):
        c = w.quantum_walk(99, s)
        cfg = {"circuit": c, "inputs": [0], "coeffs": [(1.0, 0.0)],
               "outputs": w.walk_outputs(99, s, args.outputs, seed=501), "threshold": 0.0}
        prog = Program(c.to_text())
        cuts = prog.choose_partition(PART_EQ8)
        ms, stamps, ipp, tps, _, st = timed_evaluation(ctx, prog, cfg, cuts, launch)
        ran = stamps[:, 0] > 0
        dur = np.where(ran, (stamps[:, 1].astype(np.int64) - stamps[:, 0].astype(np.int64)) / tps * 1e6, 0.0)
        per_out = dur.reshape(-1, ipp).sum(axis=1)
        M = len(cfg["outputs"])
        print(json.dumps({"steps": s, "sources": prog.A, "outputs": M, "partition": list(cuts),
                          "consumer_ms": ms, "ms_per_output": ms / M,
                          "ns_per_candidate": ms * 1e6 / (M * (1 << prog.A)),
                          "output_us": _quantiles(per_out)}), flush=True)
    return 0


def choice(args) -> int:
    """The split choice for a workload the method cannot evaluate whole (the
    amplitude-amplification circuit with 16 search qubits and 14 ancillas:
    A = 96 sources, 2^96 histories per output): Eq. (8)'s argmin and cost,
    the plain cost, the cost model's predictions over the candidate splits
    (how many lie in its training range), its own choice, and what planning
    the evaluation returns."""
    import math
    from . import FhsError, PART_MODEL, tune
    cfg = w.CONFIGS[args.workload]()
    prog = Program(cfg["circuit"].to_text())
    M, S = len(cfg["outputs"]), len(cfg["inputs"])
    ctx = Context(0)
    line = {"workload": args.workload, "qubits": prog.n, "gates": prog.G, "sources": prog.A,
            "outputs": M, "inputs": S}
    e1, e2 = prog.choose_partition(PART_EQ8)
    cost, reg = prog.partition_cost(e1, e2)
    line["eq8"] = {"partition": [e1, e2], "gate_ops_per_pair": str(cost), "log2": math.log2(cost),
                   "regions": list(reg[3:])}
    plain = prog.partition_cost(0, 0)[0]
    line["plain"] = {"gate_ops_per_pair": str(plain), "log2": math.log2(plain), "eq8_gain": plain / cost}
    blob = tune.load_model()
    splits = prog.candidate_splits()
    line["candidate_splits"] = len(splits)
    if blob is not None:
        ctx.load_cost_model(blob)
        ctx.load(prog)
        pred = ctx.predict_splits(splits, M, S)
        ok = ~np.isnan(pred)
        line["model_in_range"] = int(ok.sum())
        if ok.any():
            i = int(np.nanargmin(pred))
            line["model_best_predicted"] = {"partition": list(splits[i]), "log_seconds": float(pred[i])}
        try:
            line["model_choice"] = list(ctx.choose_partition(PART_MODEL, M, S))
        except FhsError as e:
            line["model_choice"] = str(e)
    else:
        ctx.load(prog)
    ctx.set_partition(e1, e2)
    try:
        line["plan"] = ctx.plan(M, S)
    except FhsError as e:
        line["plan"] = str(e)
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    import torch
    if not torch.cuda.is_available():      # torch sets the device up before the library does
        print("profile_items: no GPU visible", file=sys.stderr)
        return 1
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["items", "sources", "choice"])
    ap.add_argument("--workload", default="walk_99p_20s")
    ap.add_argument("--cuts", default=None, metavar="C1,C2")
    ap.add_argument("--launch", default=None, metavar="H,CHUNK,BPC,DISPATCH")
    ap.add_argument("--claim", type=int, default=None, help="items per claim (0: automatic)")
    ap.add_argument("--steps", default="10-20")
    ap.add_argument("--outputs", type=int, default=8192)
    args = ap.parse_args()
    return {"items": items, "sources": sources, "choice": choice}[args.mode](args)


if __name__ == "__main__":
    sys.exit(main())
