#!/usr/bin/env python3
"""Benchmark: reduced-history amplitude evaluation on one MI355X.

One step = one batched, checkpointed evaluation (precheck, prefix-table
build, persistent root/suffix consumer, deterministic reductions, Eq. (2))
of every requested output of the workload, inputs resident in HBM, replayed
from the library's captured HIP graph.

Default workload: the coined quantum walk with 100 qubits (1 coin + 99
position), 20 steps, 8192 requested outputs (42 reachable, 8150 seeded
unreachable), input |0>; 19 artificial sources, 2^19 candidate histories per
output.  `value` is candidate histories per second; the line also reports
amplitudes/s, leaf and valid histories/s, the plain Algorithm-1 form on the
same inputs, the dominant kernel against its roofline, and the CPU oracle
timed on a bounded sample on this host's cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "histories/s & amplitudes/s, batched+learned vs plain, 1 MI355X, |err|≤1e-12"

# MI355X peaks (AMD's published figures)
SHORTLIST = 5                # the learned split: model predictions timed before the run
PEAK_FP64 = 78.6e12          # FP64 vector FLOP/s
# 32-bit integer VALU ops/s: simple ops (add, xor, and, or, shifts, compares,
# selects) issue at the FP32 vector rate, 128 lanes per cycle per CU
# (157.3 TFLOP/s / 2 flops per FMA); 3-operand VOP3 forms issue at half that.
PEAK_INT32 = 256 * 128 * 2.4e9
PEAK_HBM = 8.0e12            # bytes/s


def kernels_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.hpp", "program.hpp", "device.hpp", "jit.hip"):
        with open(os.path.join(ROOT, "paper_2608_01467_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload: str, partition):
    """HBM bytes per launch of the consumer, from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, if it was taken on the current kernels
    with the same split (the summary holds the splits the learned shortlist
    picks for the workload)."""
    path = os.path.join(ROOT, "profiles", f"consume_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernels_hash") != kernels_hash():
        return None
    entry = d.get("splits", {}).get(f"{partition[0]},{partition[1]}")
    return entry.get("bytes_per_launch") if entry else None


def pmc_from_profile(workload: str, partition, launch):
    """Instructions the consumer issued per launch (rocprofv3 PMC summary
    committed under profiles/), if taken on the current kernels with the same
    split and launch configuration."""
    path = os.path.join(ROOT, "profiles", f"consume_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernels_hash") != kernels_hash():
        return None
    key = f"{partition[0]},{partition[1]}|{','.join(str(int(v)) for v in launch)}"
    return d.get("runs", {}).get(key)


def cpu_model() -> str:
    """The host CPU's model name (lscpu), for the CPU baseline's record."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# The oracle leg: the only part of this script that touches oracle/.  It
# checks the timed step's outputs against what the paper's mathematics fixes
# for the workload, and times the CPU oracle on a bounded sample.
# ---------------------------------------------------------------------------

_MIX = (0xBF58476D1CE4E5B9, 0x94D049BB133111EB)


def _all_history_stats(A: int):
    """(count, sum of h mod 2^64, xor of SplitMix64(h)) over every h < 2^A."""
    import numpy as np
    h = np.arange(1 << A, dtype=np.uint64)
    z = (h ^ (h >> np.uint64(30))) * np.uint64(_MIX[0])
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX[1])
    z = z ^ (z >> np.uint64(31))
    return 1 << A, int(h.sum(dtype=np.uint64)), int(np.bitwise_xor.reduce(z))


def oracle_check(workload, cfg, text, amps, stats, thr, partition, A, max_candidates=1 << 33):
    """Compare the benchmark's own outputs with references that do not come
    from the library: the position-space closed form and closed-form valid
    sets for the quantum walk (Eq. (7): every reachable output, padding
    outputs exactly zero), the 2^n state vector and the all-histories
    statistics for QAOA at t = 0, and otherwise the CPU oracle (Algorithm 2,
    same cuts) on a sample of outputs when its candidate count is small
    enough.  Returns a dict with max_abs_err, stats_exact and what was
    compared."""
    import numpy as np

    import oracle
    from oracle import closed_forms as cf
    from oracle import statevector as sv

    a = amps[:, 0] + 1j * amps[:, 1]
    st = stats.view(np.uint64) if stats.dtype != np.uint64 else stats
    outs = cfg["outputs"]
    if workload.startswith("walk_") and thr == 0.0 and all(b >> 1 == 0 for b in cfg["inputs"]):
        # inputs at position 0: the coin state is what their coefficients say
        c = cfg["circuit"]
        n_pos, steps = c.n - 1, sum(1 for g in c.gates if g.name == "H")
        coin = [0j, 0j]
        for b, z in zip(cfg["inputs"], cfg["coeffs"]):
            coin[b & 1] += complex(*z)
        dp = cf.walk_amplitudes(steps, tuple(coin))
        err, exact, n_reach = 0.0, True, 0
        for j, y in enumerate(outs):
            x = y >> 1
            x = x - (1 << n_pos) if x >= (1 << (n_pos - 1)) else x
            ref = dp.get((x, y & 1))
            if ref is None:          # unreachable: exactly zero, no valid history
                exact = exact and a[j] == 0 and all(int(v) == 0 for v in st[j, :3])
                continue
            n_reach += 1
            err = max(err, abs(a[j] - ref))
            # every input coin has the same valid set (the sources are the
            # later coin values); the statistics add over the inputs
            n1, s1, x1 = cf.walk_valid_stats(steps, x, y & 1)
            S = len(cfg["inputs"])
            want = (S * n1, (S * s1) % (1 << 64), x1 if S % 2 else 0)
            exact = exact and tuple(int(v) for v in st[j, :3]) == want
        return {"max_abs_err": float(err), "stats_exact": bool(exact), "checked_outputs": len(outs),
                "against": f"walk closed form ({n_reach} reachable outputs; {len(outs) - n_reach} "
                           "padding outputs exactly 0)"}
    if cfg["circuit"].n <= 16 and thr == 0.0:
        coeffs = [complex(*z) for z in cfg["coeffs"]]
        ref = sv.amplitudes(text, cfg["inputs"], coeffs, outs)
        err = float(np.abs(a - ref).max()) if len(outs) else 0.0
        res = {"max_abs_err": err, "checked_outputs": len(outs),
               "against": "state vector (every output)"}
        if workload.startswith("qaoa_") and A <= 30:
            # every history of a QAOA pair is valid at t = 0
            want = _all_history_stats(A)
            res["stats_exact"] = bool(all(tuple(int(v) for v in row[:3]) == want for row in st))
            res["against"] += "; valid sets: all 2^A histories"
        return res
    k = min(len(outs), 8)
    if len(outs) == 0 or k * len(cfg["inputs"]) * (1 << A) > max_candidates:
        return {"max_abs_err": None, "stats_exact": None, "checked_outputs": 0,
                "against": "not checked (the oracle would take too long)"}
    idx = np.linspace(0, len(outs) - 1, k).astype(int)
    sample = [outs[i] for i in idx]
    coeffs = [complex(*z) for z in cfg["coeffs"]]
    cores = len(os.sched_getaffinity(0))
    ref_a, ref_st = oracle.Feynman(text).evaluate(cfg["inputs"], coeffs, sample, threshold=thr,
                                                  partition=tuple(partition), threads=cores)
    err = float(np.abs(a[idx] - ref_a).max())
    exact = bool(np.array_equal(st[idx, :3], ref_st[:, :3].astype(np.uint64)))
    return {"max_abs_err": err, "stats_exact": exact, "checked_outputs": k,
            "against": f"CPU oracle (Algorithm 2, same cuts) on {k} sampled outputs"}


def cpu_baseline(text, inputs, outputs, partition, threshold, seconds_target=15.0):
    """The CPU oracle (Algorithm 2, same cuts) on a bounded sample: a slice of
    prefix assignments for several outputs, OpenMP over outputs on every
    core this process may use.  The rate is the sample's, projected to the
    whole workload's unit (candidate histories per second)."""
    import oracle

    cores = len(os.sched_getaffinity(0))
    o = oracle.Feynman(text)
    ap, ar, as_ = o.region_sources(*partition)
    per_prefix = 1 << (ar + as_)
    outs = list(outputs[: 2 * cores]) if len(outputs) >= 2 * cores else list(outputs)
    # calibrate the slice on one output, then size it for the target time
    hp = 1
    t0 = time.perf_counter()
    o.sample(inputs[0], outs[:1], partition, (0, hp), threshold, threads=1)
    dt = max(time.perf_counter() - t0, 1e-4)
    rounds = max(1, (len(outs) + cores - 1) // cores)
    hp = max(1, min(1 << ap, int(seconds_target / rounds / dt)))
    t0 = time.perf_counter()
    _, st = o.sample(inputs[0], outs, partition, (0, hp), threshold, threads=cores)
    wall = time.perf_counter() - t0
    cand = len(outs) * hp * per_prefix
    return {
        "value": cand / wall,
        "unit": "histories/s (projected from a timed sample)",
        "cores": cores,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"Algorithm 2 with the same cuts on {len(outs)} outputs, prefix assignments "
                   f"h_p < {hp} of {1 << ap} ({cand} candidate histories, {wall:.1f} s wall); "
                   f"the full workload would take "
                   f"{len(outputs) * len(inputs) * (1 << (ap + ar + as_)) / (cand / wall):.3g} s"),
    }


def sweep(args, cfg) -> int:
    """Threshold-pruning sweep (Section V, QAOA): for each threshold t the
    batched evaluation of every requested output, at the split the learned
    shortlist picks for that t (timed on the workload), timed by graph
    replay; its outputs compared with the oracle leg's references, and
    fidelity F(t) = |sum_y conj(a(y)) a_t(y)|^2 / (sum |a|^2 sum |a_t|^2)
    (0 when every amplitude is pruned) against the exact amplitudes a: the
    state vector when the circuit is small enough, else the t = 0 run.
    One JSON line per threshold."""
    import numpy as np
    import torch

    import paper_2608_01467_amd as fhs
    from paper_2608_01467_amd import tune

    text = cfg["circuit"].to_text()
    coeffs = [complex(*z) for z in cfg["coeffs"]]
    ctx = fhs.Context(0)
    ctx.set_table_budget(32 << 30)
    launch = tune.model_launch()
    if launch is not None:
        ctx.set_launch_config(*launch)     # the configuration the cost model was trained under
    exact = None
    if cfg["circuit"].n <= 16:
        from oracle import statevector as sv   # oracle leg: the exact amplitudes
        exact = sv.amplitudes(text, cfg["inputs"], coeffs, cfg["outputs"])
        exact_src = "state vector"
    base_valid = None
    for t in (float(x) for x in args.sweep.split(",")):
        wl = tune.Workload(ctx, text, cfg["inputs"], coeffs, cfg["outputs"], threshold=t)
        split, how = tune.choose(wl, tune.load_model(), reps=1, shortlist=SHORTLIST)
        sec = tune.time_split(wl, split, reps=max(1, args.steps))
        wl.run(split)
        torch.cuda.synchronize()
        a = wl.amps.cpu().numpy().copy()
        st = wl.stats.cpu().numpy()
        amp = a[:, 0] + 1j * a[:, 1]
        valid = int(st[:, 0].sum())
        leaves = int(st[:, 3].sum())
        if exact is None:
            exact, exact_src = amp.copy(), "t = 0 run"
        if base_valid is None:
            base_valid = valid
        n0, nt = float(np.sum(np.abs(exact) ** 2)), float(np.sum(np.abs(amp) ** 2))
        fid = 0.0 if nt == 0.0 else float(abs(np.vdot(exact, amp)) ** 2 / (n0 * nt))
        line = {"workload": cfg.get("name", args.workload), "threshold": t, "split": list(split),
                "split_mode": how, "launch_config": list(ctx.launch_config),
                "ms_per_eval": sec * 1e3, "fidelity": fid, "fidelity_against": exact_src,
                "retained_norm": nt / n0 if n0 else 0.0, "valid_histories": valid,
                "leaf_histories": leaves,
                "kept_fraction": valid / base_valid if base_valid else 0.0,
                "outputs": len(cfg["outputs"])}
        if not args.no_check:
            chk = oracle_check(args.workload, cfg | {"threshold": t}, text, a, st, t, split,
                               wl.prog.A)
            line["max_abs_err"] = chk.pop("max_abs_err")
            line["stats_exact"] = chk.pop("stats_exact", None)
            line["check"] = chk
        print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="walk_99p_20s")
    ap.add_argument("--partition", default="model", choices=["model", "eq8", "thirds", "none"],
                    help="model: the learned cost model's split (Eq. (8) if the workload lies "
                         "outside its training range)")
    ap.add_argument("--cuts", default=None, metavar="C1,C2",
                    help="fix the split (evaluation positions); overrides --partition")
    ap.add_argument("--cost-model", default=None, help="cost model file (default: the package's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true",
                    help="skip checking the timed step's outputs against the oracle leg's references")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shape instead of sweeping it")
    ap.add_argument("--no-fuse", action="store_true",
                    help="keep one instruction per gate (no add/subtract ladder folding)")
    ap.add_argument("--launch", default=None, metavar="H,CHUNK,BPC[,DISPATCH]",
                    help="fix the launch shape (histories per lane, chunk, blocks per CU)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison")
    ap.add_argument("--no-eq8", action="store_true",
                    help="skip timing the Eq. (8) split when the chosen split differs")
    ap.add_argument("--threshold", type=float, default=None,
                    help="pruning threshold t (default: the workload's own, 0 for every workload)")
    ap.add_argument("--sweep", default=None, metavar="T1,T2,...",
                    help="threshold sweep (Section V, QAOA): one JSON line per threshold with run "
                         "time, fidelity against the state vector and the oracle check; replaces "
                         "the single benchmark line")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (HBM-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(outputs are independent: N GPUs would each evaluate a slice of them)",
              file=sys.stderr)
        return 2

    import torch

    import paper_2608_01467_amd as fhs
    import workloads as w

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = w.CONFIGS[args.workload]()
    if args.threshold is not None:
        cfg["threshold"] = args.threshold
    if args.sweep:
        return sweep(args, cfg)
    text = cfg["circuit"].to_text()
    ctx = fhs.Context(0)
    M, S = len(cfg["outputs"]), len(cfg["inputs"])
    thr = cfg["threshold"]
    ctx.set_table_budget(32 << 30)          # one batch: the whole workload in HBM
    from paper_2608_01467_amd import tune
    wl = tune.Workload(ctx, text, cfg["inputs"], [complex(*z) for z in cfg["coeffs"]],
                       cfg["outputs"], thr, fuse=not args.no_fuse)
    prog = wl.prog              # loaded into ctx
    part_eq8 = prog.choose_partition(fhs.PART_EQ8)
    how = args.partition
    t_setup = time.perf_counter()
    blob = None
    model_launch = None
    if args.cuts:
        part = tuple(int(v) for v in args.cuts.split(","))
        how = "fixed"
    elif args.partition == "model":
        model_path = args.cost_model or tune.MODEL_PATH
        blob = tune.load_model(model_path)
        # the model's five best predictions and the Eq. (8) optimum, each
        # timed (best of 3) on this workload under the launch configuration
        # the model was trained under (or every candidate without a model)
        model_launch = tune.model_launch(model_path)
        if model_launch is not None and prog.A > 0:
            ctx.set_launch_config(*model_launch)
        part, how = tune.choose(wl, blob, reps=3, shortlist=SHORTLIST) if blob is not None else \
            (part_eq8, "eq8 (no cost model)")
    else:
        mode = {"eq8": fhs.PART_EQ8, "thirds": fhs.PART_THIRDS, "none": fhs.PART_NONE}
        part = prog.choose_partition(mode[args.partition])
    launch = None
    if args.launch:
        ctx.set_launch_config(*(int(v) for v in args.launch.split(",")))
    elif not args.no_autotune and prog.A > 0:
        # launch shape (histories per lane, chunk, blocks per CU) swept with
        # the chosen split on the workload (on its first 1024 outputs when
        # it has more than 8192); kept for the full run
        outs_t = cfg["outputs"] if len(cfg["outputs"]) <= 8192 else cfg["outputs"][:1024]
        sub = tune.Workload(ctx, text, cfg["inputs"], [complex(*z) for z in cfg["coeffs"]],
                            outs_t, thr, fuse=not args.no_fuse)
        launch, _ = tune.autotune_launch(sub, part, reps=2)
        ctx.load(prog)
        del sub
        if (args.partition == "model" and not args.cuts and blob is not None
                and launch != model_launch):
            # the shortlist again under the tuned launch configuration
            part, how = tune.choose(wl, blob, reps=3, shortlist=SHORTLIST)
    t_setup = time.perf_counter() - t_setup
    ctx.set_partition(*part)
    d_in, d_out, d_cf = wl.d_in, wl.d_out, wl.d_cf
    amps = torch.empty((M, 2), dtype=torch.float64, device="cuda:0")
    stats = torch.empty((M, 4), dtype=torch.int64, device="cuda:0")
    def step(plain=False):
        ctx.evaluate(d_in, d_cf, d_out, threshold=thr, plain=plain, out=(amps, stats))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    T = (time.perf_counter() - t0) / max(args.steps, 1)
    st = stats.cpu()
    amps_host = amps.cpu().numpy().copy()
    # Dominant-kernel durations: the same K steps again with HIP events
    # around every consumer launch (direct launches instead of the graph).
    ctx.set_kernel_timing(True)
    kt = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()
        kt += ctx.kernel_times()
    T_timed = (time.perf_counter() - t0) / max(args.steps, 1)
    n_entries, n_valid_entries = ctx.kernel_counts()
    ctx.set_kernel_timing(False)

    leaves = int(st[:, 3].sum())
    valid = int(st[:, 0].sum())
    cand = M * S * (1 << prog.A)
    plan = ctx.plan(M, S)
    # Algorithmic work of the consumer per step, summed over the gates that
    # must be evaluated: the root region once for each of the 2^Ar root
    # assignments of every prefix entry still consistent after the prefix
    # region, the suffix region's integer work once per leaf walked (2^As
    # per consistent root) and its factor products once per valid history
    # (a history's amplitude is needed only when it passes the final check).
    # The suffix's integer work whose inputs are only the suffix's own source
    # bits is the same for every root that shares the suffix assignment (the
    # consumer computes it once per assignment for a whole wave): it is not
    # counted per leaf.  Redundant evaluations the kernel makes for
    # parallelism (root re-runs by the lanes that share a root task, lanes
    # that idle inside a wave) do not count.
    root = prog.work(plan["c1"], plan["c2"])
    suffix = prog.work(plan["c2"], prog.G)
    launches = max(1, len(kt) // max(args.steps, 1))
    n_root = n_valid_entries << plan["Ar"]
    # The suffix instructions the compiled consumer evaluates once per root
    # (no suffix source influences them) count per root, not per leaf.
    hoist = ctx.launch_config[3] == 3 and thr == 0.0
    h_int = suffix["hoist_int_ops"] if hoist else 0
    h_fp = suffix["hoist_fp64_flops"] if hoist else 0
    suffix_leaf_int = suffix["int_ops"] - suffix["src_int_ops"] - h_int
    root_int, root_fp = root["int_ops"], root["fp64_flops"]
    suffix_valid_fp = suffix["fp64_flops"] - h_fp
    # Two-valued factors the compiled consumer counts instead of multiplying
    # (same condition): their integer steps join the int32 work, their
    # multiplies leave the FP64 work, and each valid history takes one
    # complex multiply per table group.
    groups = plan["count_groups"] if hoist else 0
    if groups:
        root_int += root["count_int_ops"]
        root_fp -= root["count_fp64_flops"]
        h_int += suffix["hoist_count_int_ops"]
        h_fp -= suffix["hoist_count_fp64_flops"]
        suffix_leaf_int += suffix["count_int_ops"] - suffix["hoist_count_int_ops"]
        suffix_valid_fp -= suffix["count_fp64_flops"] - suffix["hoist_count_fp64_flops"]
        suffix_valid_fp += 6 * groups
    int_ops = (n_root * (root_int + h_int) + leaves * suffix_leaf_int) / launches
    flops = (n_root * (root_fp + h_fp) + valid * suffix_valid_fp) / launches
    avg_launch = sum(kt) / len(kt) / 1e3
    int_rate = int_ops / avg_launch
    fp_rate = flops / avg_launch
    if int_rate / PEAK_INT32 >= fp_rate / PEAK_FP64:
        roof = {"bound": "alu", "achieved": int_rate / 1e12, "peak": PEAK_INT32 / 1e12,
                "unit": "Tops/s", "frac": int_rate / PEAK_INT32, "operand": "int32 VALU ops"}
    else:
        roof = {"bound": "alu", "achieved": fp_rate / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": fp_rate / PEAK_FP64, "operand": "FP64 flops"}
    tb = traffic_from_profile(args.workload, part)
    roof["traffic"] = tb
    # The work model counts operations; the hardware counters count issued
    # instructions.  Lane-instructions per second against the 128-lane VALU
    # issue rate (the int32 peak above), the FP64 share of them, and VALU
    # busy (wave-instructions per CU-cycle, rocprofv3's VALUBusy), from the
    # committed PMC summary over this launch's measured duration.
    pm = pmc_from_profile(args.workload, part, ctx.launch_config)
    if pm:
        lane_rate = pm["valu_insts"] * 64 / avg_launch
        roof["pmc"] = {"valu_lane_instr_per_s": lane_rate,
                       "valu_issue_frac": lane_rate / PEAK_INT32,
                       "fp64_instr_share": pm["fp64_insts"] / pm["valu_insts"],
                       "fp64_executed_tflops": pm["fp64_flops"] / avg_launch / 1e12,
                       "valu_busy": pm["valu_insts"] / (256 * 2.4e9 * avg_launch),
                       "salu_per_valu": pm["salu_insts"] / pm["valu_insts"]}
    else:
        roof["pmc"] = None
    roof["kernel"] = "fhs_consume_compiled" if ctx.launch_config[3] == 3 else "k_consume"
    roof["avg_launch_ms"] = avg_launch * 1e3
    roof["launches_per_step"] = launches
    roof["work"] = {"prefix_entries": n_entries, "prefix_entries_consistent": n_valid_entries,
                    "root_evaluations": n_root, "leaves": leaves,
                    "root_int_ops": root["int_ops"], "suffix_int_ops": suffix["int_ops"],
                    "suffix_src_int_ops": suffix["src_int_ops"],
                    "suffix_hoisted_int_ops": h_int, "suffix_hoisted_fp64_flops": h_fp,
                    "root_fp64_flops": root["fp64_flops"],
                    "suffix_fp64_flops": suffix["fp64_flops"],
                    "count_groups": groups, "count_entries": plan["count_entries"] if groups else 0,
                    "root_count_int_ops": root["count_int_ops"], "root_count_fp64_flops": root["count_fp64_flops"],
                    "suffix_count_int_ops": suffix["count_int_ops"],
                    "suffix_count_fp64_flops": suffix["count_fp64_flops"]}
    roof["ms_per_step_timed"] = T_timed * 1e3
    roof["fp64_tflops"] = fp_rate / 1e12
    roof["int32_tops"] = int_rate / 1e12
    # int32 and FP64 work share the same VALU issue slots: the fraction of
    # the launch the algorithmic work needs at both peaks together
    roof["frac_int32_plus_fp64"] = int_rate / PEAK_INT32 + fp_rate / PEAK_FP64

    out = {
        "metric": METRIC,
        "value": cand / T,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "qubits": prog.n, "gates": prog.G, "sources": prog.A,
            "outputs": M, "inputs": S, "threshold": thr,
            "fused_ladders": not args.no_fuse,
            "partition": list(part), "partition_mode": how, "partition_setup_s": t_setup,
            "launch_config": list(ctx.launch_config), "launch_autotuned": launch is not None,
            "regions": [plan["Ap"], plan["Ar"], plan["As"]],
        },
        "amplitudes_per_s": M * S / T,
        "leaf_histories_per_s": leaves / T,
        "valid_histories_per_s": valid / T,
        # Eq. (8) gate evaluations per second: the paper's work measure, counted gate
        # by gate (folded ladders count every gate they replace)
        "eq8_gate_ops_per_s": M * S * prog.partition_cost(*part)[0] / T,
        "roofline": roof,
    }
    if tuple(part) != tuple(part_eq8) and not args.no_eq8:
        # the paper's own choice, Eq. (8), on the same inputs, at its own best
        # chunk (the launch shape was tuned for the learned split)
        saved = ctx.launch_config
        ctx.set_partition(*part_eq8)
        best_e = None
        for chunk in dict.fromkeys((saved[1], 64, 128, 256)):
            ctx.set_launch_config(saved[0], chunk, saved[2], saved[3])
            step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(max(1, min(args.steps, 3))):
                step()
            torch.cuda.synchronize()
            te = (time.perf_counter() - t0) / max(1, min(args.steps, 3))
            if best_e is None or te < best_e[0]:
                best_e = (te, chunk)
        ctx.set_launch_config(*saved)
        ctx.set_partition(*part)
        Te = best_e[0]
        out["eq8_split"] = {"partition": list(part_eq8), "ms_per_step": Te * 1e3,
                            "chunk": best_e[1], "histories_per_s": cand / Te,
                            "learned_speedup": Te / T}
    if not args.no_plain:
        # Algorithm 1 (no checkpoint) in two code generations: the plain
        # kernel with the interpreted program on a static grid (the baseline
        # form, at its own best lane shape: 1 or 2 histories per lane), and
        # the same straight-line compiled regions as the batched form with
        # cuts (0, 0), so that the learned split's gain is also measured
        # like for like.  One timed pass each after a warm-up pass.
        saved = ctx.launch_config
        best = None
        for h in (1, 2):
            ctx.set_launch_config(h, saved[1], saved[2], 0)
            step(plain=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(plain=True)
            torch.cuda.synchronize()
            tp = time.perf_counter() - t0
            if best is None or tp < best[0]:
                best = (tp, h)
        Tp = best[0]
        out["plain"] = {"ms_per_step": Tp * 1e3, "histories_per_s": cand / Tp,
                        "amplitudes_per_s": M * S / Tp, "batched_speedup": Tp / T,
                        "histories_per_lane": best[1], "dispatch": "interpreted (k_plain)"}
        if saved[3] == 3 and prog.A > 0:
            ctx.set_launch_config(*saved)
            ctx.set_partition(0, 0)
            try:
                step()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                step()
                torch.cuda.synchronize()
                tc = time.perf_counter() - t0
                out["plain_compiled"] = {
                    "ms_per_step": tc * 1e3, "histories_per_s": cand / tc,
                    "batched_speedup": tc / T, "partition": [0, 0],
                    "dispatch": "compiled regions (fhs_consume_compiled), cuts (0, 0)"}
            except fhs.FhsError as e:      # a region too long to compile, or no table space
                out["plain_compiled"] = {"skipped": str(e)}
            ctx.set_partition(*part)
        ctx.set_launch_config(*saved)
    if not args.no_check:
        chk = oracle_check(args.workload, cfg, text, amps_host, st.numpy(), thr, part, prog.A)
        out["max_abs_err"] = chk.pop("max_abs_err")
        out["stats_exact"] = chk.pop("stats_exact", None)
        out["check"] = chk
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(text, cfg["inputs"], cfg["outputs"], part, thr)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
