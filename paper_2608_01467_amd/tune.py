"""Autotuner and learned split model.

The paper chooses the checkpoint split by minimising its gate-operation
estimate, Eq. (8) (Section IV-C).  On the GPU the run time also depends on
what Eq. (8) does not see: the prefix table's size and traffic, how many
root tasks there are to fill 256 compute units, and the mix of integer and
FP64 work per region.  This module

  * times evaluations on the device (`time_split`), sweeps the launch shape
    (`autotune_launch`) and searches every candidate split exhaustively
    (`exhaustive`): the ground truth;
  * turns (split features, measured time) pairs into a training set
    (`collect`), the features coming from the library (fhs_split_features);
  * trains the cost-model network on the device with the library's own
    forward/backward/Adam kernels (`train`), and packs it as the blob
    fhs_load_cost_model expects;
  * evaluates the trained model's regret against exhaustive search and
    Eq. (8) (`regret`).

Everything here drives the C ABI; no computation of the method happens in
Python.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import (N_FEATURES, PART_EQ8, PART_MODEL, Context, FhsError, Program, mlp_adam,
               mlp_backward, mlp_forward, mlp_param_count, mlp_workspace_size)

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_model.json")
SHAPE = (N_FEATURES, 32, 32)


class Workload:
    """A circuit plus resident device inputs for timing."""

    def __init__(self, ctx: Context, text: str, inputs, coeffs, outputs, threshold=0.0,
                 fuse: bool = True):
        import torch
        self.ctx = ctx
        self.prog = Program(text, fuse=fuse)
        ctx.load(self.prog)
        self.d_in = ctx.device_bits(inputs)
        self.d_cf = ctx.device_coeffs(coeffs)
        self.d_out = ctx.device_bits(outputs)
        self.M, self.S = len(outputs), len(inputs)
        self.thr = threshold
        self.amps = torch.empty((self.M, 2), dtype=torch.float64, device=self.d_out.device)
        self.stats = torch.empty((self.M, 4), dtype=torch.int64, device=self.d_out.device)

    def run(self, partition: Tuple[int, int], plain: bool = False) -> None:
        if self.ctx.program is not self.prog:
            self.ctx.load(self.prog)
        self.ctx.set_partition(*partition)
        self.ctx.evaluate(self.d_in, self.d_cf, self.d_out, threshold=self.thr, plain=plain,
                          out=(self.amps, self.stats))

    def table_bytes(self, partition) -> int:
        if self.ctx.program is not self.prog:
            self.ctx.load(self.prog)
        self.ctx.set_partition(*partition)
        return self.ctx.plan(self.M, self.S)["table_bytes"]


SHORT_STEP = 1e-3     # seconds: below this one evaluation is timed in batches
SHORT_BATCH = 32      # back-to-back evaluations per timing of a short step
CUTOFF_FLOOR = 0.05   # seconds: a first run (graph capture included) this fast is never cut off
TIE = 0.01            # timings within this fraction of the fastest are a tie


def first_within(rows, tie: float = TIE):
    """The first entry of [(key, seconds)], in the given order, whose time
    is within `tie` of the fastest: among timings the measurement cannot
    tell apart, the order decides (the cost model's ranking for splits, the
    sweep's order for launch shapes), so the same workload gets the same
    choice from run to run."""
    fastest = min(t for _, t in rows)
    return next(k for k, t in rows if t <= fastest * (1.0 + tie))


def time_split(wl: Workload, partition, reps: int = 3, plain: bool = False,
               cutoff: Optional[float] = None) -> float:
    """Time of one evaluation (graph replay), seconds: the best of `reps`
    timings.  The first run captures the graph; if it already took longer
    than `cutoff` seconds its time is returned as is (a split that slow is
    measured once, well enough to rank it last; never below CUTOFF_FLOOR,
    since a first run also captures the graph).  A second run tells a short
    step (under SHORT_STEP) from a long one: a short step is timed as the
    mean of SHORT_BATCH back-to-back evaluations between two
    synchronisations, best of at least 5 such batches (as the benchmark
    times its steps; a lone evaluation's launch and synchronisation latency
    would be most of its timing); a long one evaluation at a time."""
    import torch

    def timed(n: int) -> float:
        t0 = time.perf_counter()
        for _ in range(n):
            wl.run(partition, plain)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    first = timed(1)
    if cutoff is not None and first > max(cutoff, CUTOFF_FLOOR):
        return first
    one = timed(1)
    if one < SHORT_STEP:
        return min(timed(SHORT_BATCH) for _ in range(max(reps, 5)))
    return min([one] + [timed(1) for _ in range(reps - 1)])


def autotune_launch(wl: Workload, partition, reps: int = 2) -> Tuple[Tuple[int, int, int, int], List]:
    """Sweep histories per lane x chunk x blocks per CU (automatic dispatch),
    then the explicit dispatch modes (per run, per instruction, compiled) at
    the best shape, then histories per lane x chunk for the compiled
    consumer; keep the first of the fastest (first_within)."""
    log = []
    best, best_t = None, math.inf
    for h in (1, 2):
        for chunk in (64, 128, 256):
            for bpc in (0, 2, 4):
                cfg = (h, chunk, bpc, 0)
                wl.ctx.set_launch_config(*cfg)
                t = time_split(wl, partition, reps)
                log.append((cfg, t))
                if t < best_t:
                    best, best_t = cfg, t
    for dispatch in (1, 2, 3):
        cfg = best[:3] + (dispatch,)
        wl.ctx.set_launch_config(*cfg)
        t = time_split(wl, partition, reps)
        log.append((cfg, t))
        if t < best_t:
            best, best_t = cfg, t
    # the compiled consumer's own best lane shape and chunk
    done = {cfg for cfg, _ in log}
    for h in (1, 2):
        for chunk in (128, 256):
            cfg = (h, chunk, best[2], 3)
            if cfg in done:
                continue
            wl.ctx.set_launch_config(*cfg)
            t = time_split(wl, partition, reps)
            log.append((cfg, t))
            if t < best_t:
                best, best_t = cfg, t
    best = first_within(log)
    wl.ctx.set_launch_config(*best)
    return best, log


def candidates(wl: Workload, max_cost_ratio: float = 64.0, extra: int = 8,
               max_table_bytes: int = 8 << 30, seed: int = 0,
               limit: Optional[int] = None) -> List[Tuple[int, int]]:
    """Candidate splits worth timing: every one within max_cost_ratio of the
    Eq. (8) optimum (at most `limit`, cheapest first), plus a few random
    others, all with a table that fits."""
    cand = wl.prog.candidate_splits()
    costs = {c: wl.prog.partition_cost(*c)[0] for c in cand}
    best = min(costs.values())
    ranked = sorted(cand, key=lambda c: (costs[c], c))
    near = [c for c in ranked if costs[c] <= max_cost_ratio * best][:limit]
    far = [c for c in ranked if c not in near]
    rng = np.random.default_rng(seed)
    if far and extra:
        idx = rng.choice(len(far), size=min(extra, len(far)), replace=False)
        near += [far[i] for i in idx]
    keep = []
    for c in near:
        try:
            if wl.table_bytes(c) <= max_table_bytes:
                keep.append(c)
        except Exception:
            pass
    return keep


PRECOMPILE_BATCH = 32   # splits whose compiled consumers are built together


def exhaustive(wl: Workload, splits: Sequence[Tuple[int, int]], reps: int = 2, log=None,
               slow_factor: float = 8.0, budget: Optional[float] = None):
    """Time every split (in the given order, best guesses first); returns
    [(split, seconds)] and the first of the fastest (first_within).  A
    split whose first run is slower than `slow_factor` x the best so far is
    timed once; after `budget` seconds the remaining splits are skipped.
    `log`, if given, is called with a progress string every few splits."""
    rows = []
    t0 = time.perf_counter()
    best = math.inf
    splits = list(splits)
    compiled = wl.ctx.launch_config[3] == 3
    for i, c in enumerate(splits):
        if budget is not None and rows and time.perf_counter() - t0 > budget:
            if log is not None:
                log(f"  budget reached: {len(rows)}/{len(splits)} splits timed")
            break
        if compiled and i % PRECOMPILE_BATCH == 0:
            # compile the next batch's consumers in parallel, not one per timing
            wl.ctx.precompile(splits[i:i + PRECOMPILE_BATCH], wl.M, wl.S, wl.thr)
        t = time_split(wl, c, reps, cutoff=slow_factor * best if best < math.inf else None)
        rows.append((c, t))
        best = min(best, t)
        if log is not None and (i + 1) % 16 == 0:
            log(f"  {i + 1}/{len(splits)} splits timed, {time.perf_counter() - t0:.1f} s")
    return rows, first_within(rows)


def collect(wl: Workload, splits, reps: int = 2, log=None, budget: Optional[float] = None):
    """Feature rows and log-times for the given splits."""
    rows, _ = exhaustive(wl, splits, reps, log, budget=budget)
    X = np.array([wl.prog.split_features(c[0], c[1], wl.M, wl.S) for c, _ in rows])
    y = np.log(np.array([t for _, t in rows]))
    return X, y, rows


def train(X: np.ndarray, y: np.ndarray, epochs: int = 3000, lr: float = 3e-3, ensemble: int = 5,
          seed: int = 0, device: str = "cuda:0", log_every: int = 0):
    """Fit `ensemble` networks (different initialisations) on the device with
    fhs_mlp_backward / fhs_mlp_adam to the log times `y`; returns (blob,
    training loss of the averaged prediction).  Features are standardised
    here; the scaling and the per-feature training range travel in the
    blob."""
    import torch
    n_in, h1, h2 = SHAPE
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-9] = 1.0
    lo, hi = X.min(axis=0), X.max(axis=0)
    Xs = (X - mu) / sd
    dX = torch.tensor(Xs, dtype=torch.float64, device=device).contiguous()
    dT = torch.tensor(y, dtype=torch.float64, device=device).contiguous()
    B = dX.shape[0]
    ws = torch.empty(mlp_workspace_size(SHAPE, B), dtype=torch.uint8, device=device)
    loss = torch.zeros(1, dtype=torch.float64, device=device)
    nets = []
    for k in range(ensemble):
        rng = np.random.default_rng(seed + k)
        parts = []
        for fo, fi in ((h1, n_in), (h2, h1)):          # Glorot-uniform weights
            lim = math.sqrt(6.0 / (fi + fo))
            parts += [rng.uniform(-lim, lim, fo * fi), np.zeros(fo)]
        lim = math.sqrt(6.0 / (h2 + 1))
        parts += [rng.uniform(-lim, lim, h2), np.array([y.mean()])]
        p0 = np.concatenate(parts)
        assert p0.size == mlp_param_count(n_in, h1, h2)
        P = torch.tensor(p0, dtype=torch.float64, device=device)
        G = torch.zeros_like(P)
        m = torch.zeros_like(P)
        v = torch.zeros_like(P)
        for it in range(1, epochs + 1):
            mlp_backward(SHAPE, P, dX, dT, G, loss, ws)
            mlp_adam(P, G, m, v, it, lr)
            if log_every and it % log_every == 0:
                torch.cuda.synchronize()
                print(f"network {k} epoch {it} loss {loss.item():.5f}", flush=True)
        torch.cuda.synchronize()
        nets.append(P.cpu().numpy())
    blob = np.concatenate([[n_in, h1, h2], mu, sd, lo, hi] + nets)
    pred = predict(blob, X, device)
    return blob, float(np.mean((pred - y) ** 2))


def predict(blob: np.ndarray, X: np.ndarray, device: str = "cuda:0") -> np.ndarray:
    """Predicted log(seconds) for raw feature rows: fhs_mlp_forward per
    network of the blob, averaged."""
    import torch
    n_in, h1, h2 = (int(v) for v in blob[:3])
    mu = blob[3:3 + n_in]
    sd = blob[3 + n_in:3 + 2 * n_in]
    params = blob[3 + 4 * n_in:]
    npar = mlp_param_count(n_in, h1, h2)
    assert params.size % npar == 0
    dX = torch.tensor((X - mu) / sd, dtype=torch.float64, device=device).contiguous()
    dY = torch.empty(X.shape[0], dtype=torch.float64, device=device)
    out = np.zeros(X.shape[0])
    K = params.size // npar
    for k in range(K):
        P = torch.tensor(params[k * npar:(k + 1) * npar], dtype=torch.float64, device=device)
        mlp_forward((n_in, h1, h2), P, dX, dY)
        torch.cuda.synchronize()
        out += dY.cpu().numpy()
    return out / K


def save_model(blob: np.ndarray, meta: Dict, path: str = MODEL_PATH) -> None:
    with open(path, "w") as f:
        json.dump({"shape": list(SHAPE), "blob": [float(x).hex() for x in blob], "meta": meta},
                  f, indent=1)


def load_model(path: str = MODEL_PATH) -> Optional[np.ndarray]:
    """The saved blob, or None if there is none or it was trained on another
    feature set than this library's."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    blob = np.array([float.fromhex(x) for x in d["blob"]], dtype=np.float64)
    if blob.size < 3 or int(blob[0]) != N_FEATURES:
        return None
    return blob


def model_launch(path: str = MODEL_PATH) -> Optional[Tuple[int, int, int, int]]:
    """The launch configuration the saved model's timings were taken under
    (None if the file does not record one)."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        meta = json.load(f).get("meta", {})
    if "launch" not in meta:
        return None
    return tuple(int(v) for v in str(meta["launch"]).split(","))


def choose(wl: Workload, blob: Optional[np.ndarray], reps: int = 2, log=None,
           budget: Optional[float] = None, shortlist: int = 0) -> Tuple[Tuple[int, int], str]:
    """The split to run.  With a model whose training range covers the
    program: its argmin (shortlist = 0), or, with shortlist = k > 0, the
    fastest by measurement among the model's k best predictions and the
    Eq. (8) optimum.  Otherwise, or with no model, the fastest candidate by
    exhaustive timing.  Returns (split, "model" | "model+timed" | "timed")."""
    if blob is not None:
        wl.ctx.load_cost_model(blob)
        try:
            pick = wl.ctx.choose_partition(PART_MODEL, wl.M, wl.S)
        except FhsError as e:
            if e.status != 3:      # FHS_ERANGE: outside the training range
                raise
            pick = None
        if pick is not None and shortlist <= 0:
            return pick, "model"
        if pick is not None:
            cand = wl.prog.candidate_splits()
            pred = wl.ctx.predict_splits(cand, wl.M, wl.S)
            order = [cand[i] for i in np.argsort(np.where(np.isnan(pred), np.inf, pred), kind="stable")
                     if not np.isnan(pred[i])]
            short = list(dict.fromkeys(order[:shortlist] + [wl.prog.choose_partition(PART_EQ8)]))
            _, best = exhaustive(wl, short, reps, log)
            return best, "model+timed"
    _, best = exhaustive(wl, candidates(wl, extra=0), reps, log, budget=budget)
    return best, "timed"


def regret(wl: Workload, blob: np.ndarray, splits, reps: int = 2, log=None,
           shortlist: int = 5, budget: Optional[float] = None) -> Dict:
    """Time the model's choice, the model's shortlist verified by timing,
    Eq. (8)'s choice and the exhaustive best.  The best time is the minimum
    over every timing taken, so that a regret is never negative."""
    rows, best = exhaustive(wl, splits, reps, log, budget=budget)
    c_model, how = choose(wl, blob, reps)
    c_short, how_s = choose(wl, blob, reps, shortlist=shortlist)
    c_eq8 = wl.prog.choose_partition(PART_EQ8)
    t_model = time_split(wl, c_model, reps)
    t_short = time_split(wl, c_short, reps)
    t_eq8 = time_split(wl, c_eq8, reps)
    timed = dict(rows)
    for c, t in ((c_model, t_model), (c_short, t_short), (c_eq8, t_eq8)):
        if t < timed.get(c, math.inf):
            timed[c] = t
    best = min(timed, key=lambda c: (timed[c], c))
    t_best = timed[best]
    return {"best": best, "t_best": t_best, "model": c_model, "how": how, "t_model": t_model,
            "shortlist": c_short, "how_shortlist": how_s, "t_shortlist": t_short,
            "eq8": c_eq8, "t_eq8": t_eq8, "model_regret": t_model / t_best - 1.0,
            "shortlist_regret": t_short / t_best - 1.0,
            "eq8_regret": t_eq8 / t_best - 1.0, "gain_over_eq8": t_eq8 / t_model,
            "splits_timed": len(rows)}
