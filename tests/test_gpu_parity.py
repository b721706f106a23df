"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Bar: valid-history count, index sum and index hash bit-exact; amplitudes
within |delta| <= 1e-12 (absolute, per output).  Every case runs both GPU
forms (plain Algorithm 1 and the batched, checkpointed Algorithm 2) on the
same seeded inputs.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as w
from oracle import closed_forms as cf
from oracle import statevector as sv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_01467_amd as fhs  # noqa: E402

TOL = 1e-12
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
THREADS = min(16, len(os.sched_getaffinity(0)))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fhs.Context(0)


def gpu_eval(ctx, text, inputs, coeffs, outputs, thr=0.0, partition=(0, 0), plain=False,
             prog=None):
    prog = prog or fhs.Program(text)
    ctx.load(prog)
    ctx.set_partition(*partition)
    amps, stats = ctx.evaluate(inputs, coeffs, outputs, threshold=thr, plain=plain)
    torch.cuda.synchronize()
    a = amps.cpu().numpy()
    return a[:, 0] + 1j * a[:, 1], stats.cpu().numpy().view(np.uint64)


def compare(ctx, text, inputs, coeffs, outputs, thr=0.0, partitions=None, ref=None):
    """Run plain + batched at each partition; compare with the oracle."""
    o = oracle.Feynman(text)
    if ref is None:
        ref_amps, ref_st = o.evaluate(inputs, coeffs, outputs, threshold=thr, threads=THREADS)
    else:
        ref_amps, ref_st = ref
    prog = fhs.Program(text)
    if partitions is None:
        partitions = [(0, 0), prog.choose_partition(fhs.PART_THIRDS),
                      prog.choose_partition(fhs.PART_EQ8), (prog.G, prog.G), (0, prog.G)]
    runs = [("plain", (0, 0), True)] + [(f"cut{p}", p, False) for p in partitions]
    for name, part, plain in runs:
        amps, st = gpu_eval(ctx, text, inputs, coeffs, outputs, thr, part, plain, prog=prog)
        err = np.abs(amps - ref_amps).max() if len(outputs) else 0.0
        assert err <= TOL, (name, err)
        assert np.array_equal(st[:, :3], ref_st[:, :3].astype(np.uint64)), name
    return ref_amps, ref_st


def test_eq6_and_fig2(ctx):
    t = "qubits 3\nH 0\nCX 0 1\nS 1\nCX 1 2\n"
    compare(ctx, t, [0], [1], list(range(8)))
    fig2 = ("qubits 4\nCX 1 0\nH 1\nSWAP 2 3\nH 3\nP 2 " + math.pi.hex() +
            "\nCX 0 1\nH 0\nSWAP 1 2\n")
    for i in range(16):
        compare(ctx, fig2, [i], [1], list(range(16)), partitions=[(0, 0), (2, 5), (1, 3)])


def test_clifford_t_config(ctx):
    cfg = w.CONFIGS["clifford_t_10q_40g"]()
    t = cfg["circuit"].to_text()
    coeffs = [complex(*z) for z in cfg["coeffs"]]
    ref = sv.amplitudes(t, cfg["inputs"], coeffs, cfg["outputs"])
    amps, _ = compare(ctx, t, cfg["inputs"], coeffs, cfg["outputs"])
    assert np.abs(amps - ref).max() <= TOL


@pytest.mark.parametrize("seed", range(24))
def test_random_mixed(ctx, seed):
    n = [2, 5, 9, 12, 31, 32, 33, 40, 64, 65, 99, 128][seed % 12]
    c = w.random_mixed(n, 12 + seed % 20, 4000 + seed, max_controls=4)
    t = c.to_text()
    rng = np.random.default_rng(seed)
    o = oracle.Feynman(t)
    if o.A > 14:
        pytest.skip("too many sources for the oracle in a quick test")
    S = 1 + seed % 3
    inputs = [int(rng.integers(0, 1 << min(n, 62))) for _ in range(S)]
    coeffs = [complex(rng.normal(), rng.normal()) for _ in range(S)]
    outs = [int(rng.integers(0, 1 << min(n, 62))) for _ in range(20)]
    # sprinkle outputs reachable from the first input (nonzero amplitudes)
    if n <= 12:
        psi = sv.evolve(t, inputs[0])
        outs += [int(x) for x in np.argsort(-np.abs(psi))[:8]]
    thr = [0.0, 0.0, 1e-3, 0.02][seed % 4]
    compare(ctx, t, inputs, coeffs, outs, thr=thr)


def test_qft20_closed_form(ctx):
    cfg = w.CONFIGS["qft_20q"]()
    t = cfg["circuit"].to_text()
    x = cfg["inputs"][0]
    ref = np.array([cf.qft_amplitude(20, x, y) for y in cfg["outputs"]])
    for plain in (False, True):
        amps, st = gpu_eval(ctx, t, [x], [1], cfg["outputs"], plain=plain)
        assert np.abs(amps - ref).max() <= TOL
        assert (st[:, 0] == 1).all()


def _all_h_stats(A):
    h = np.arange(1 << A, dtype=np.uint64)
    s = int(h.sum(dtype=np.uint64))
    z = h.copy()
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return s, int(np.bitwise_xor.reduce(z))


def test_aa_k4_closed_form(ctx):
    cfg = w.CONFIGS["aa_k4_s3"]()
    c, marked = cfg["circuit"], cfg["marked"]
    t = c.to_text()
    prog = fhs.Program(t)
    assert prog.A == 24
    outs = cfg["outputs"]
    ref = np.array([cf.aa_amplitude(4, 3, marked, y) for y in outs])
    s_all, x_all = _all_h_stats(24)
    for part, plain in [((0, 0), True), (prog.choose_partition(fhs.PART_EQ8), False),
                        (prog.choose_partition(fhs.PART_THIRDS), False)]:
        amps, st = gpu_eval(ctx, t, [0], [1], outs, partition=part, plain=plain, prog=prog)
        assert np.abs(amps - ref).max() <= TOL
        for y, row in zip(outs, st):
            if y >> 4:           # an ancilla bit set: no valid history
                assert row[0] == 0
            else:
                assert (int(row[0]), int(row[1]), int(row[2])) == (1 << 24, s_all, x_all)


def test_qaoa12_statevector_and_counts(ctx):
    """All 4096 outputs of the 12-vertex, p = 2 QAOA circuit against the
    state vector, every history valid: at Eq. (8)'s split in the default
    launch shape, and at the split the benchmark times, (35, 40), in the
    launch shapes its autotuner settles on (1 history per lane, chunk 256,
    4 blocks per CU or as many as fit; the compiled consumer with counted
    factors)."""
    cfg = w.CONFIGS["qaoa_12v_p2"]()
    t = cfg["circuit"].to_text()
    prog = fhs.Program(t)
    assert prog.A == 24
    outs = cfg["outputs"]
    ref = sv.amplitudes(t, [0], [1], outs)
    s_all, x_all = _all_h_stats(24)
    runs = [(prog.choose_partition(fhs.PART_EQ8), (0, 0, 0, 0)),
            ((35, 40), (1, 256, 0, 3)), ((35, 40), (1, 256, 4, 3))]
    for part, (h, chunk, bpc, dispatch) in runs:
        ctx.set_launch_config(h, chunk, bpc, dispatch)
        amps, st = gpu_eval(ctx, t, [0], [1], outs, partition=part, prog=prog)
        assert np.abs(amps - ref).max() <= TOL, (part, h, chunk, bpc, dispatch)
        assert abs(np.sum(np.abs(amps) ** 2) - 1.0) <= 1e-10
        assert (st[:, 0] == (1 << 24)).all()
        assert (st[:, 1] == s_all).all() and (st[:, 2] == x_all).all()
    ctx.set_launch_config(0, 0, 0, 0)


@pytest.mark.parametrize("thr", [1e-5, 3e-5, 1e-3])
def test_qaoa_pruning_sampled(ctx, thr):
    cfg = w.CONFIGS["qaoa_12v_p2"]()
    t = cfg["circuit"].to_text()
    prog = fhs.Program(t)
    rng = np.random.default_rng(7)
    outs = [int(x) for x in rng.choice(4096, size=2, replace=False)]
    part = prog.choose_partition(fhs.PART_EQ8)
    o = oracle.Feynman(t)
    ref = o.evaluate([0], [1], outs, threshold=thr, partition=part, threads=THREADS)
    for p, plain in [(part, False), ((0, 0), True)]:
        amps, st = gpu_eval(ctx, t, [0], [1], outs, thr=thr, partition=p, plain=plain, prog=prog)
        assert np.abs(amps - ref[0]).max() <= TOL
        assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64))


@pytest.mark.parametrize("thr", [1e-6, 1e-4])
def test_qaoa12_config_thresholds(ctx, thr):
    """The 12-vertex QAOA workload at its own pruning thresholds: 16 sampled
    outputs of the 4096, the plain form and the batched form at Eq. (8)'s
    split and at the cost model's three best predicted splits for the whole
    workload (the splits the benchmark's shortlist times), under the
    compiled consumer (one and two histories per lane) and the interpreter;
    amplitudes and valid sets against the oracle.  Pruning decisions are
    bit-exact: at 1e-6 about 85% of each output's 2^24 histories survive, at
    1e-4 none does (every amplitude exactly 0)."""
    from paper_2608_01467_amd import tune
    cfg = w.CONFIGS["qaoa_12v_p2"]()
    t = cfg["circuit"].to_text()
    prog = fhs.Program(t)
    rng = np.random.default_rng(11)
    outs = sorted(int(x) for x in rng.choice(4096, size=16, replace=False))
    eq8 = prog.choose_partition(fhs.PART_EQ8)
    ref_a, ref_st = oracle.Feynman(t).evaluate([0], [1], outs, threshold=thr, partition=eq8,
                                               threads=THREADS)
    if thr == 1e-4:
        assert (ref_st[:, 0] == 0).all() and (ref_a == 0).all()
    else:
        assert (ref_st[:, 0] > 0).all()
    splits = [eq8]
    blob = tune.load_model()
    if blob is not None:
        ctx.load(prog)
        ctx.load_cost_model(blob)
        cand = prog.candidate_splits()
        pred = ctx.predict_splits(cand, len(cfg["outputs"]), 1)
        order = [cand[i] for i in np.argsort(np.where(np.isnan(pred), np.inf, pred), kind="stable")
                 if not np.isnan(pred[i])]
        splits += [c for c in order[:3] if c != eq8]
    runs = [((0, 0), True, (0, 0, 0))]
    runs += [(p, False, launch) for p in splits for launch in ((1, 256, 3), (2, 256, 3))]
    runs += [(eq8, False, (2, 256, 0))]
    for part, plain, (h, chunk, dispatch) in runs:
        ctx.set_launch_config(h, chunk, 0, dispatch)
        amps, st = gpu_eval(ctx, t, [0], [1], outs, thr=thr, partition=part, plain=plain, prog=prog)
        assert np.abs(amps - ref_a).max() <= TOL, (thr, part, plain, h, dispatch)
        assert np.array_equal(st[:, :3], ref_st[:, :3].astype(np.uint64)), (thr, part, plain, h)
    ctx.set_launch_config(0, 0, 0, 0)


def test_qaoa8_pruning_all_partitions(ctx):
    t = w.qaoa_maxcut(8, 2, 411, 412)[0].to_text()
    for thr in (0.0, 1e-4, 3e-3):
        compare(ctx, t, [0], [1], list(range(0, 256, 5)), thr=thr)


@pytest.mark.parametrize("n_pos,steps", [(6, 5), (99, 7)])
def test_walk_small(ctx, n_pos, steps):
    t = w.quantum_walk(n_pos, steps).to_text()
    outs = w.walk_outputs(n_pos, steps, 40, seed=5)
    dp = cf.walk_amplitudes(steps)
    amps, st = compare(ctx, t, [0], [1], outs)
    for y, a in zip(outs, amps):
        x = (y >> 1)
        x = x - (1 << n_pos) if x >= (1 << (n_pos - 1)) else x
        assert abs(a - dp.get((x, y & 1), 0)) <= TOL


@pytest.mark.parametrize("n_pos", [10, 31, 32, 33, 63, 64])
def test_walk_field_widths(ctx, n_pos):
    """The compiled consumer ends the suffix by comparing the pending count of
    position steps with the position field's residue against the output
    rather than adding it.  Fields narrower than, as wide as and wider than a
    word, ending inside a word and crossing into the next; outputs reachable
    (negative positions: the residue wraps), one and two steps out of reach,
    and random (residues that no count reaches); cuts that put the whole run,
    part of it or none of it in the suffix; one and two histories per lane.
    Against the position-space closed form and the closed-form valid sets."""
    steps = 6
    t = w.quantum_walk(n_pos, steps).to_text()
    outs = w.walk_outputs(n_pos, steps, 2 * (steps + 1) + 12, seed=n_pos)
    outs += [y for y in (w.walk_state(n_pos, x, c) for x in (-steps - 2, -steps - 1, steps + 1, steps + 2)
                         for c in (0, 1)) if y not in outs]
    dp = cf.walk_amplitudes(steps)
    prog = fhs.Program(t)
    src = prog.source_eval_positions
    parts = [(0, 0), (0, src[2] + 1), (src[1] + 1, src[3] + 1), (src[0] + 1, src[-1]),
             prog.choose_partition(fhs.PART_EQ8), (prog.G, prog.G)]
    for h in (1, 2):
        ctx.set_launch_config(h, 0, 0, 3)
        for part in parts:
            amps, st = gpu_eval(ctx, t, [0], [1], outs, partition=part, prog=prog)
            for y, a, row in zip(outs, amps, st):
                x = y >> 1
                x = x - (1 << n_pos) if x >= (1 << (n_pos - 1)) else x
                assert abs(a - dp.get((x, y & 1), 0)) <= TOL, (n_pos, h, part, y)
                assert tuple(int(v) for v in row[:3]) == cf.walk_valid_stats(steps, x, y & 1), \
                    (n_pos, h, part, y)
    ctx.set_launch_config(0, 0, 0, 0)


@pytest.mark.gpu
@pytest.mark.parametrize("n_pos", [31, 40])
def test_walk_pass_filter(ctx, n_pos):
    """Leaves rejected before they are walked: the suffix ends with the
    position-count check, whose residue is the same for every leaf of a
    root, so a pass of leaves (or, with a long suffix walked one leaf at a
    time, a single leaf) whose source popcounts cannot reach it is skipped.
    16 steps (A = 15): suffixes of 2 to 15 sources, short (eight leaves per
    pass) and long (one), fields as wide as a word less one bit and wider;
    against the position-space closed form and the closed-form valid sets."""
    steps = 16
    t = w.quantum_walk(n_pos, steps).to_text()
    outs = w.walk_outputs(n_pos, steps, 2 * (steps + 1) + 10, seed=n_pos + 1)
    dp = cf.walk_amplitudes(steps)
    prog = fhs.Program(t)
    src = prog.source_eval_positions
    assert prog.A == 15
    parts = [(src[0] + 1, src[2]), (src[1], src[1]), (0, src[0]), (src[4], src[7]), (src[6], src[12]),
             (src[9], src[13])]
    for h in (1, 2):
        ctx.set_launch_config(h, 0, 0, 3)
        for part in parts:
            amps, st = gpu_eval(ctx, t, [0], [1], outs, partition=part, prog=prog)
            for y, a, row in zip(outs, amps, st):
                x = y >> 1
                x = x - (1 << n_pos) if x >= (1 << (n_pos - 1)) else x
                assert abs(a - dp.get((x, y & 1), 0)) <= TOL, (n_pos, h, part, y)
                assert tuple(int(v) for v in row[:3]) == cf.walk_valid_stats(steps, x, y & 1), \
                    (n_pos, h, part, y)
    ctx.set_launch_config(0, 0, 0, 0)


@pytest.mark.gpu
def test_walk_pair_filter_batches(ctx):
    """Pairs the precheck rejects with the residue test over the whole
    program (the walk's position count after the leading gates must be
    reachable by its sources' steps): reachable and unreachable outputs
    interleaved, two input bitstrings (coin 0 and 1 at position 0, complex
    coefficients), each batch listing its own accepted pairs (a table budget
    of 1 MiB: sixteen pairs per batch), and root parts (a pair's root tasks
    over several items); amplitudes and valid sets against the oracle."""
    n_pos, steps = 31, 14
    t = w.quantum_walk(n_pos, steps).to_text()
    rng = np.random.default_rng(77)
    outs = w.walk_outputs(n_pos, steps, 60, seed=78)
    outs = [outs[i] for i in rng.permutation(len(outs))]
    inputs = [w.walk_state(n_pos, 0, 0), w.walk_state(n_pos, 0, 1)]
    coeffs = [complex(0.6, 0.0), complex(0.0, 0.8)]
    ref = oracle.Feynman(t).evaluate(inputs, coeffs, outs, threads=THREADS)
    assert np.abs(ref[0]).max() > 1e-3
    prog = fhs.Program(t)
    src = prog.source_eval_positions
    assert prog.A == 13
    seen_batches = seen_parts = 0
    for part, budget in [((src[11], src[12]), 1 << 20), ((src[11], src[11]), 1 << 20),
                         ((src[1], src[12]), 1 << 30), ((0, src[6]), 1 << 30)]:
        ctx.set_table_budget(budget)
        for h in (1, 2):
            ctx.set_launch_config(h, 0, 0, 3)
            ctx.load(prog)
            ctx.set_partition(*part)
            plan = ctx.plan(len(outs), len(inputs))
            assert plan["pair_filter"] == 1
            seen_batches = max(seen_batches, plan["n_batches"])
            seen_parts = max(seen_parts, plan["root_parts"])
            amps, st = gpu_eval(ctx, t, inputs, coeffs, outs, partition=part, prog=prog)
            assert np.abs(amps - ref[0]).max() <= TOL, (part, budget, h)
            assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (part, budget, h)
    assert seen_batches >= 8 and seen_parts >= 8, (seen_batches, seen_parts)
    ctx.set_table_budget(1 << 30)
    ctx.set_launch_config(0, 0, 0, 0)


@pytest.mark.gpu
def test_walk_filters_with_pruning(ctx):
    """The residue tests (pair, root, pass) together with threshold pruning:
    a walk whose histories all have modulus 2^(-A/2) (one Hadamard factor
    per source), at thresholds below it (nothing pruned) and above it
    (everything pruned), interpreted and compiled consumers; against the
    oracle."""
    n_pos, steps = 20, 9
    t = w.quantum_walk(n_pos, steps).to_text()
    outs = w.walk_outputs(n_pos, steps, 40, seed=9)
    o = oracle.Feynman(t)
    prog = fhs.Program(t)
    src = prog.source_eval_positions
    for thr in (1e-3, 0.3):
        ref = o.evaluate([0], [1.0], outs, threshold=thr, threads=THREADS)
        for dispatch in (0, 3):
            ctx.set_launch_config(2, 0, 0, dispatch)
            for part in [(src[1], src[4]), (0, src[2]), prog.choose_partition(fhs.PART_EQ8)]:
                amps, st = gpu_eval(ctx, t, [0], [1], outs, thr=thr, partition=part, prog=prog)
                assert np.abs(amps - ref[0]).max() <= TOL, (thr, dispatch, part)
                assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (thr, dispatch, part)
        if thr > 0.1:
            assert not ref[1][:, 0].any()       # every history pruned
        else:
            assert ref[1][:, 0].any()
    ctx.set_launch_config(0, 0, 0, 0)


def test_walk_config_full(ctx):
    """100 qubits, 20 steps, the full 8192 outputs: the 42 reachable outputs
    against the position-space closed form and the closed-form valid sets
    (count, index sum, index hash); the padding outputs exactly zero.  Run
    in the launch shapes the benchmark times: the interpreting and the
    compiled consumer, one and two histories per lane, the Eq. (8) split and
    the learned splits; ladders paired (the default) and only folded."""
    cfg = w.CONFIGS["walk_99p_20s"]()
    t = cfg["circuit"].to_text()
    prog = fhs.Program(t)
    folded = fhs.Program(t, pair=False)
    outs = cfg["outputs"]
    dp = cf.walk_amplitudes(20)
    eq8 = prog.choose_partition(fhs.PART_EQ8)
    runs = [(prog, eq8, False, (0, 0, 0, 0)), (prog, (0, 0), True, (0, 0, 0, 0)),
            (prog, (2984, 3581), False, (1, 0, 0, 3)), (prog, (3183, 3581), False, (2, 0, 0, 3)),
            (prog, eq8, False, (2, 0, 0, 3)), (folded, (2984, 3581), False, (1, 0, 0, 3))]
    # the splits the learned shortlist picks for this workload, in the launch
    # shapes the benchmark's autotuner settles on (1 or 2 histories per lane,
    # chunk 256, 4 blocks per CU or as many as fit, compiled consumer and
    # prefix build): each split is its own compiled module
    shortlist = [(198, 2785), (596, 2785), (198, 2387), (1989, 2785), (2188, 2984)]
    runs += [(prog, p, False, (2, 256, 4, 3)) for p in shortlist]
    runs += [(prog, (198, 2785), False, (1, 256, 4, 3)), (prog, (596, 2785), False, (1, 256, 4, 3)),
             (prog, (198, 2785), False, (1, 256, 0, 3)), (prog, (198, 2387), False, (1, 128, 2, 3))]
    for pg, part, plain, (h, chunk, bpc, dispatch) in runs:
        ctx.set_launch_config(h, chunk, bpc, dispatch)
        amps, st = gpu_eval(ctx, t, [0], [1], outs, partition=part, plain=plain, prog=pg)
        for y, a, row in zip(outs[:42], amps[:42], st[:42]):
            x = y >> 1
            x = x - (1 << 99) if x >= (1 << 98) else x
            assert abs(a - dp.get((x, y & 1), 0)) <= TOL
            assert tuple(int(v) for v in row[:3]) == cf.walk_valid_stats(20, x, y & 1)
        assert abs(np.sum(np.abs(amps[:42]) ** 2) - 1.0) <= 1e-10
        assert (amps[42:] == 0).all() and (st[42:, 0] == 0).all()
    ctx.set_launch_config(0, 0, 0, 0)


def _reachable(circuit, count, seed):
    """Outputs reachable from |0>: follow the circuit forward with a random
    value at every H (permutations applied, phases ignored)."""
    rng = np.random.default_rng(seed)
    outs = set()
    for _ in range(count * 4):
        x = 0
        for g in circuit.gates:
            q = g.qubits
            negs = g.negs or (False,) * len(q)
            if g.name == "H":
                x = (x & ~(1 << q[0])) | (int(rng.integers(0, 2)) << q[0])
            elif g.name == "X":
                x ^= 1 << q[0]
            elif g.name == "CX":
                if (x >> q[0]) & 1:
                    x ^= 1 << q[1]
            elif g.name == "MCX":
                if all(((x >> c) & 1) != int(ng) for c, ng in zip(q[1:], negs[1:])):
                    x ^= 1 << q[0]
        outs.add(x)
        if len(outs) >= count:
            break
    return sorted(outs)


@pytest.mark.parametrize("n,seed", [(12, 1), (40, 2), (64, 3), (100, 4)])
def test_folded_ladders(ctx, n, seed):
    """Add/subtract-one ladders folded into one instruction (the default)
    and left gate by gate: both match the oracle at every cut, plain too."""
    c = w.random_ladders(n, 12, seed)
    t = c.to_text()
    outs = _reachable(c, 24, seed) + w.random_outputs(n, 8, seed + 50)
    o = oracle.Feynman(t)
    ref = o.evaluate([0], [1], outs, threads=THREADS)
    assert np.abs(ref[0]).max() > 0.0          # some amplitudes are nonzero
    for fuse, dispatch in ((True, 0), (False, 0), (True, 3), (False, 3)):
        ctx.set_launch_config(0, 0, 0, dispatch)
        prog = fhs.Program(t, fuse=fuse)
        parts = [prog.choose_partition(fhs.PART_EQ8), prog.choose_partition(fhs.PART_THIRDS),
                 (0, prog.G), (prog.G, prog.G)]
        # cuts inside a folded ladder: the next few positions after each source
        src = prog.source_eval_positions
        if src:
            parts += [(src[0] + 1, src[-1] + 2), (src[len(src) // 2] + 3, prog.G)]
        for part, plain in [((0, 0), True)] + [(p, False) for p in parts]:
            part = (min(part[0], prog.G), min(part[1], prog.G))
            amps, st = gpu_eval(ctx, t, [0], [1], outs, partition=part, plain=plain, prog=prog)
            assert np.abs(amps - ref[0]).max() <= TOL, (fuse, dispatch, part, plain)
            assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (fuse, dispatch, part)
    ctx.set_launch_config(0, 0, 0, 0)
    if n <= 12:
        sv_ref = sv.amplitudes(t, [0], [1], outs)
        assert np.abs(ref[0] - sv_ref).max() <= 1e-12


@pytest.mark.parametrize("n,seed", [(12, 11), (40, 12), (64, 13), (100, 14)])
def test_paired_ladders(ctx, n, seed):
    """Complementary ladder pairs merged into one add-or-subtract (the
    default), folded but unpaired, and gate by gate: all match the oracle at
    every cut (cuts inside a pair too), under the interpreted dispatches and
    the compiled consumer, plain too."""
    c = w.random_ladder_pairs(n, 10, seed)
    t = c.to_text()
    outs = _reachable(c, 24, seed) + w.random_outputs(n, 8, seed + 50)
    o = oracle.Feynman(t)
    ref = o.evaluate([0], [1], outs, threads=THREADS)
    assert np.abs(ref[0]).max() > 0.0
    paired = fhs.Program(t)
    assert paired.work(0, paired.G)["int_ops"] < fhs.Program(t, pair=False).work(0, paired.G)["int_ops"]
    for (fuse, pair), dispatch in [((True, True), 0), ((True, True), 2), ((True, True), 3),
                                   ((True, False), 3), ((False, False), 0)]:
        ctx.set_launch_config(0, 0, 0, dispatch)
        prog = fhs.Program(t, fuse=fuse, pair=pair)
        parts = [prog.choose_partition(fhs.PART_EQ8), prog.choose_partition(fhs.PART_THIRDS),
                 (0, prog.G), (prog.G, prog.G)]
        src = prog.source_eval_positions
        if src:
            parts += [(src[0] + 1, src[-1] + 2), (src[len(src) // 2] + 3, prog.G),
                      (src[0] + 2 + n // 2, prog.G)]
        for part, plain in [((0, 0), True)] + [(p, False) for p in parts]:
            part = (min(part[0], prog.G), min(part[1], prog.G))
            part = (min(part[0], part[1]), part[1])
            amps, st = gpu_eval(ctx, t, [0], [1], outs, partition=part, plain=plain, prog=prog)
            assert np.abs(amps - ref[0]).max() <= TOL, (fuse, pair, dispatch, part, plain)
            assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (fuse, pair, dispatch, part)
    ctx.set_launch_config(0, 0, 0, 0)
    if n <= 12:
        sv_ref = sv.amplitudes(t, [0], [1], outs)
        assert np.abs(ref[0] - sv_ref).max() <= 1e-12


def test_multi_input_and_edge_cases(ctx):
    t = w.random_mixed(7, 30, 77).to_text()
    inputs = [3, 17, 100]
    coeffs = [0.5 + 0.1j, -0.3j, 0.7]
    outs = list(range(128)) + [5, 5]          # duplicates allowed
    compare(ctx, t, inputs, coeffs, outs)
    # no outputs: nothing to do
    prog = fhs.Program(t)
    ctx.load(prog)
    amps, st = ctx.evaluate([0], [1], [], threshold=0.0)
    assert amps.shape[0] == 0
    # a circuit without gates: amplitude 1 iff output == input
    amps, st = gpu_eval(ctx, "qubits 3\n", [5], [1], list(range(8)))
    assert np.array_equal(amps, np.where(np.arange(8) == 5, 1.0, 0.0))


def test_bits_above_n_are_flagged(ctx):
    t = "qubits 3\nH 0\nCX 0 1\n"
    prog = fhs.Program(t)
    ctx.load(prog)
    bad = torch.tensor([[0], [8], [3]], dtype=torch.int64, device="cuda:0")
    for plain in (False, True):
        amps, st = ctx.evaluate([0], [1], bad, plain=plain)
        torch.cuda.synchronize()
        st = st.cpu().numpy().view(np.uint64)
        assert st[1, 3] == np.uint64(0xFFFFFFFFFFFFFFFF)
        assert amps[1].abs().sum().item() == 0.0
        assert st[0, 3] != np.uint64(0xFFFFFFFFFFFFFFFF)


def test_deterministic_and_graph_replay(ctx):
    cfg = w.CONFIGS["qaoa_12v_p2"]()
    t = cfg["circuit"].to_text()
    prog = fhs.Program(t)
    ctx.load(prog)
    ctx.set_partition(*prog.choose_partition(fhs.PART_EQ8))
    outs = cfg["outputs"][:512]
    d_in = ctx.device_bits([0])
    d_out = ctx.device_bits(outs)
    d_cf = ctx.device_coeffs([1])
    amps = torch.empty((512, 2), dtype=torch.float64, device="cuda:0")
    stats = torch.empty((512, 4), dtype=torch.int64, device="cuda:0")
    first = None
    for rep in range(4):
        amps.fill_(float("nan"))
        stats.fill_(-1)
        ctx.evaluate(d_in, d_cf, d_out, threshold=0.0, out=(amps, stats))
        torch.cuda.synchronize()
        cur = (amps.cpu().numpy().copy(), stats.cpu().numpy().copy())
        if first is None:
            first = cur
        assert np.array_equal(cur[0], first[0]) and np.array_equal(cur[1], first[1])
    # a different threshold re-captures and still matches the oracle on a sample
    ctx.evaluate(d_in, d_cf, d_out, threshold=1e-4, out=(amps, stats))
    torch.cuda.synchronize()
    ref = oracle.Feynman(t).evaluate([0], [1], outs[:4], threshold=1e-4,
                                     partition=ctx.partition, threads=THREADS)
    a = amps.cpu().numpy()[:4]
    assert np.abs(a[:, 0] + 1j * a[:, 1] - ref[0]).max() <= TOL


def test_errors(ctx):
    t = w.amplitude_amplification(16, 3, 4, 301)[0].to_text()
    prog = fhs.Program(t)
    ctx.load(prog)
    with pytest.raises(fhs.FhsError) as ei:
        ctx.evaluate([0], [1], [0])
    assert ei.value.status == 3          # A = 96 > 62
    ctx.load(fhs.Program("qubits 2\nH 0\n"))
    with pytest.raises(fhs.FhsError) as ei:
        ctx.set_partition(1, 0)
    assert ei.value.status == 1
    with pytest.raises(fhs.FhsError) as ei:
        ctx.evaluate([0], [1], [0], threshold=float("nan"))
    assert ei.value.status == 1
    with pytest.raises(fhs.FhsError) as ei:
        ctx.evaluate([0], [1], [0], threshold=-1.0)
    assert ei.value.status == 1
    fresh = fhs.Context(0)
    with pytest.raises(fhs.FhsError) as ei:
        fresh.set_partition(0, 0)
    assert ei.value.status == 6


def _phase_heavy(n_cp: int, seed: int):
    """6 qubits: a Hadamard on every wire, then n_cp random controlled-phase
    gates (a factor table of 8 doubles per gate) with six more Hadamards
    (artificial sources) spread through them, so that the regions' factors
    exceed what the kernels stage in LDS while their instructions stay short
    enough to be compiled."""
    rng = np.random.default_rng(seed)
    c = w.Circuit(6)
    for q in range(6):
        c.add("H", q)
    hs = {k * n_cp // 7: k - 1 for k in range(1, 7)}
    for i in range(n_cp):
        if i in hs:
            c.add("H", hs[i])
        a, b = (int(x) for x in rng.choice(6, size=2, replace=False))
        c.add("CP", a, b, angle=float(rng.uniform(-np.pi, np.pi)))
    return c


@pytest.mark.parametrize("family", ["clifford_t", "qaoa", "qaoa_pruned", "aa", "phase_heavy"])
def test_compiled_consumer_families(ctx, family):
    """The run-time compiled consumer and prefix build (dispatch mode 3, one
    and two histories per lane) against the oracle on each circuit family,
    at several splits: deferred suffix factors without pruning, factors as
    the walk goes with it, and factors read from HBM when the suffix's table
    is too large for LDS."""
    thr = 0.0
    if family == "clifford_t":
        c = w.random_clifford_t(10, 60, seed=31)
        outs = list(range(0, 1024, 17))
    elif family in ("qaoa", "qaoa_pruned"):
        c = w.qaoa_maxcut(8, 2, 41, 42)[0]
        outs = list(range(0, 256, 5))
        thr = 1e-3 if family == "qaoa_pruned" else 0.0
    elif family == "aa":
        c, _ = w.amplitude_amplification(3, 3)
        outs = list(range(0, 1 << c.n, max(1, (1 << c.n) // 48)))
    else:
        c = _phase_heavy(600, 51)
        outs = list(range(64))
    t = c.to_text()
    o = oracle.Feynman(t)
    ref = o.evaluate([0], [1], outs, threshold=thr, threads=THREADS)
    prog = fhs.Program(t)
    parts = [prog.choose_partition(fhs.PART_EQ8), prog.choose_partition(fhs.PART_THIRDS),
             (0, prog.G)]
    src = prog.source_eval_positions
    if len(src) >= 2:
        parts.append((src[0] + 1, src[-1] + 1))
    for h in (1, 2):
        ctx.set_launch_config(h, 0, 0, 3)
        for part in parts:
            amps, st = gpu_eval(ctx, t, [0], [1], outs, thr=thr, partition=part, prog=prog)
            assert np.abs(amps - ref[0]).max() <= TOL, (family, h, part)
            assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (family, h, part)
    ctx.set_launch_config(0, 0, 0, 0)


def _branchy(n: int, layers: int, seed: int):
    """Random layered circuit with a few branching gates per layer (H, RX,
    RY), diagonal two-qubit gates with conjugate-pair tables (RZZ) and
    without (CZ, CP), one-qubit phases (RZ, T, S, Z, P), and permutations
    (X, CX, SWAP, CCX): past the first layer most branching gates carry
    artificial sources."""
    rng = np.random.default_rng(seed)
    c = w.Circuit(n)
    for _ in range(layers):
        for q in rng.choice(n, size=min(n, 3), replace=False):
            g = str(rng.choice(["H", "H", "RX", "RY"]))
            if g == "H":
                c.add(g, int(q))
            else:
                c.add(g, int(q), angle=float(rng.uniform(-np.pi, np.pi)))
        for _ in range(n):
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            g = str(rng.choice(["RZZ", "RZZ", "CZ", "CP", "CX", "SWAP"]))
            if g in ("RZZ", "CP"):
                c.add(g, a, b, angle=float(rng.uniform(-np.pi, np.pi)))
            else:
                c.add(g, a, b)
        for q in rng.choice(n, size=min(n, 3), replace=False):
            g = str(rng.choice(["RZ", "T", "S", "Z", "X", "P"]))
            if g in ("RZ", "P"):
                c.add(g, int(q), angle=float(rng.uniform(-np.pi, np.pi)))
            else:
                c.add(g, int(q))
        if n >= 3:
            a, b, t3 = (int(x) for x in rng.choice(n, size=3, replace=False))
            c.add("CCX", a, b, t3)
    return c


@pytest.mark.parametrize("seed", range(8))
def test_compiled_random_mixed(ctx, seed):
    """The compiled consumer and prefix build on random layered circuits with
    random inputs: factors formed in registers from constant tables
    (conjugate pairs such as RZ and RZZ, real branching tables such as H
    with input bits 0 and 1, whose signs are applied at the region's end),
    the other tables read per lane, deferred and immediate suffix factors,
    with and without pruning, at several splits."""
    n = [4, 6, 7, 9, 12, 33, 64, 100][seed]
    c = _branchy(n, 3 + seed % 2, 9000 + seed)
    t = c.to_text()
    o = oracle.Feynman(t)
    assert 3 <= o.A <= 14, o.A
    rng = np.random.default_rng(100 + seed)
    S = 1 + seed % 3
    inputs = [int(rng.integers(0, 1 << min(n, 62))) for _ in range(S)]
    coeffs = [complex(rng.normal(), rng.normal()) for _ in range(S)]
    outs = [int(rng.integers(0, 1 << min(n, 62))) for _ in range(16)]
    if n <= 12:
        psi = sv.evolve(t, inputs[0])
        outs += [int(x) for x in np.argsort(-np.abs(psi))[:8]]
    prog = fhs.Program(t)
    parts = [prog.choose_partition(fhs.PART_EQ8), prog.choose_partition(fhs.PART_THIRDS),
             (0, prog.G), (prog.G, prog.G)]
    src = prog.source_eval_positions
    if len(src) >= 2:
        parts.append((src[0] + 1, src[-1] + 1))
    for thr in (0.0, 0.02):
        ref = o.evaluate(inputs, coeffs, outs, threshold=thr, threads=THREADS)
        for h in (1, 2):
            ctx.set_launch_config(h, 0, 0, 3)
            for part in parts:
                amps, st = gpu_eval(ctx, t, inputs, coeffs, outs, thr=thr, partition=part, prog=prog)
                assert np.abs(amps - ref[0]).max() <= TOL, (seed, thr, h, part)
                assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (seed, thr, h, part)
    ctx.set_launch_config(0, 0, 0, 0)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", [9112, 9128])
def test_compiled_uniform_suffix(ctx, seed):
    """Enough (pair, root) tasks that each lane holds its own root task:
    every suffix source then lives in the leaf loop's wave-uniform counter
    and the compiled consumer is built with that as a constant (scalar work
    over the suffix sources, unrolled passes when the suffix is short, the
    suffix instructions no suffix source influences once per root).  Random
    layered circuits on 12 qubits, 2048 outputs, against the oracle, with and
    without pruning, at splits with 2^8 or more root tasks per pair."""
    c = _branchy(12, 5, seed)
    t = c.to_text()
    o = oracle.Feynman(t)
    prog = fhs.Program(t)
    assert prog.A == 12
    src = list(prog.source_eval_positions)
    outs = w.random_outputs(12, 2048, seed=seed)
    # (Ap, Ar, As) = (9, 0, 3), (6, 3, 3), (6, 2, 4): 2^8 or more root tasks
    # per pair; (3, 3, 6) shares each root task among several lanes
    parts = [(src[8] + 1, src[9]), (src[5] + 1, src[9]), (src[5] + 1, src[8]), (src[2] + 1, src[5] + 1)]
    ctx.load(prog)
    uniform = 0
    for part in parts:
        ctx.set_launch_config(2, 0, 0, 3)
        ctx.set_partition(*part)
        plan = ctx.plan(len(outs), 1)
        uniform += plan["lanes_per_root_task"] == 1
    assert uniform == 3
    for thr in (0.0, 0.02):
        ref = o.evaluate([0], [1.0], outs, threshold=thr, threads=THREADS)
        for h in (1, 2):
            ctx.set_launch_config(h, 0, 0, 3)
            for part in parts:
                amps, st = gpu_eval(ctx, t, [0], [1.0], outs, thr=thr, partition=part, prog=prog)
                assert np.abs(amps - ref[0]).max() <= TOL, (seed, thr, h, part)
                assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (seed, thr, h, part)
    ctx.set_launch_config(0, 0, 0, 0)


def _counted(n: int, layers: int, seed: int):
    """Random layered circuit whose factors mostly take two values, with few
    distinct angles: RX on a few qubits (the first on each wire on its
    natural input, the later ones with sources), RZZ with +-gamma (both
    orientations of one class), CP, CZ, RZ with +-theta, T, TDG, S and Y."""
    rng = np.random.default_rng(seed)
    g1, g2, b1, th = (float(x) for x in rng.uniform(-np.pi, np.pi, 4))
    c = w.Circuit(n)

    def pick(k):
        return [int(x) for x in rng.choice(n, size=k, replace=False)]

    rxq = pick(4)
    for q in rxq:
        c.add("RX", q, angle=b1)
    for _ in range(layers):
        for _ in range(6):
            a, b = pick(2)
            c.add("RZZ", a, b, angle=g1 if rng.integers(0, 2) else -g1)
        for _ in range(2):
            a, b = pick(2)
            c.add("CP", a, b, angle=g2)
        a, b = pick(2)
        c.add("CZ", a, b)
        for q in pick(3):
            k = str(rng.choice(["RZ+", "RZ-", "T", "TDG", "S", "Y", "Y"]))
            if k.startswith("RZ"):
                c.add("RZ", q, angle=th if k == "RZ+" else -th)
            else:
                c.add(k, q)
        for q in rng.choice(rxq, size=3, replace=False):
            c.add("RX", int(q), angle=b1)
        a, b = pick(2)
        c.add("CX", a, b)
    return c


@pytest.mark.gpu
@pytest.mark.parametrize("n,seed", [(12, 1), (40, 2), (40, 3)])
def test_compiled_counted_factors(ctx, n, seed):
    """Two-valued factors counted by the compiled consumer instead of
    multiplied (without pruning): grouped population counts of each form
    (bits that differ, agree, are both set, a bit set or clear), single
    diagonal gates across state words, Y, RX on natural inputs and with
    sources, one to three table groups, with deferred suffix factors; against
    the oracle on reachable and random outputs, and with pruning (no
    counting) as well."""
    c = _counted(n, 3, seed)
    t = c.to_text()
    o = oracle.Feynman(t)
    prog = fhs.Program(t)
    assert prog.A == 9
    rng = np.random.default_rng(seed)
    outs = set()
    for _ in range(96):
        x = 0
        for g in c.gates:
            q = g.qubits
            if g.name == "RX":
                x = (x & ~(1 << q[0])) | (int(rng.integers(0, 2)) << q[0])
            elif g.name == "Y":
                x ^= 1 << q[0]
            elif g.name == "CX" and (x >> q[0]) & 1:
                x ^= 1 << q[1]
        outs.add(x)
    outs = sorted(outs)[:48] + [int(rng.integers(0, 1 << n)) for _ in range(8)]
    src = list(prog.source_eval_positions)
    parts = [(src[3] + 1, src[6] + 1), (src[0] + 1, src[4] + 1), (0, src[4]), (src[2] + 1, src[5] + 1)]
    for thr in (0.0, 0.02):
        ref = o.evaluate([0], [1.0], outs, threshold=thr, threads=THREADS)
        if thr == 0.0:
            assert np.abs(ref[0]).max() > 1e-3
        for h in (1, 2):
            ctx.set_launch_config(h, 0, 0, 3)
            for part in parts:
                amps, st = gpu_eval(ctx, t, [0], [1.0], outs, thr=thr, partition=part, prog=prog)
                assert np.abs(amps - ref[0]).max() <= TOL, (n, seed, thr, h, part)
                assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), (n, seed, thr, h, part)
    ctx.set_launch_config(0, 0, 0, 0)


@pytest.mark.parametrize("case", ["fig2", "qft8", "qaoa6", "walk_xcoin", "aa3", "branchy1", "branchy3"])
def test_forward_placement(ctx, case):
    """Sources placed by the forward sweep (FHS_REDUCE_FORWARD, Table I's
    other column): the plain form and the batched form (interpreted and
    compiled, cuts counted from the input) against the oracle's forward
    placement, valid sets included; the amplitudes also equal the backward
    program's."""
    rng = np.random.default_rng(sum(map(ord, case)))
    if case == "fig2":
        t = ("qubits 4\nCX 1 0\nH 1\nSWAP 2 3\nH 3\nP 2 " + math.pi.hex() +
             "\nCX 0 1\nH 0\nSWAP 1 2\n")
    elif case == "qft8":
        t = w.qft(8).to_text()
    elif case == "qaoa6":
        t = w.qaoa_maxcut(6, 2, 61, 62)[0].to_text()
    elif case == "walk_xcoin":
        t = w.quantum_walk_xcoin(12, 7).to_text()
    elif case == "aa3":
        t = w.amplitude_amplification(3, 1, 2, seed=9)[0].to_text()
    else:
        seed = int(case[-1])
        t = _branchy([4, 6, 7, 9][seed], 3 + seed % 2, 9000 + seed).to_text()
    of, ob = oracle.Feynman(t, "forward"), oracle.Feynman(t)
    n = of.n
    S = 1 + len(case) % 2
    inputs = [0] + [int(rng.integers(0, 1 << min(n, 62))) for _ in range(S - 1)]
    coeffs = [complex(rng.normal(), rng.normal()) for _ in range(S)]
    outs = list(range(1 << n)) if n <= 8 else [int(rng.integers(0, 1 << n)) for _ in range(48)]
    if case == "walk_xcoin":
        outs = w.walk_outputs(12, 7, 40, seed=3)
    ref_a, ref_st = of.evaluate(inputs, coeffs, outs, threads=THREADS)
    bwd_a, _ = ob.evaluate(inputs, coeffs, outs, threads=THREADS)
    assert np.abs(ref_a - bwd_a).max() <= TOL
    prog = fhs.Program(t, forward=True)
    assert prog.forward and prog.A == of.A
    parts = [(0, 0), prog.choose_partition(fhs.PART_EQ8), prog.choose_partition(fhs.PART_THIRDS),
             (prog.G, prog.G)]
    runs = [((0, 0), True, 0, 1)] + [(p, False, d, h) for p in parts for d, h in ((0, 2), (3, 1), (3, 2))]
    for part, plain, dispatch, h in runs:
        ctx.set_launch_config(h, 0, 0, dispatch)
        amps, st = gpu_eval(ctx, t, inputs, coeffs, outs, partition=part, plain=plain, prog=prog)
        assert np.abs(amps - ref_a).max() <= TOL, (case, part, plain, dispatch, h)
        assert np.array_equal(st[:, :3], ref_st[:, :3].astype(np.uint64)), (case, part, plain, dispatch)
    ctx.set_launch_config(0, 0, 0, 0)


REACH_CASES = ["fig3", "cnot5-optimal", "cnot8-optimal", "cnot11-greedy", "cnot14-greedy", "cnot51-optimal",
               "cnot103-optimal", "cnot107-optimal", "big-optimal"]


@pytest.mark.gpu
@pytest.mark.parametrize("case", REACH_CASES)
def test_reach_placement(ctx, case):
    """Sources placed by determinism reachability (FHS_REDUCE_OPTIMAL /
    GREEDY, Section IV-B): the plain form and the batched form at allowed
    cut pairs (interpreted, and compiled at three of them), with and without
    pruning, against the oracle's Algorithm 1 under the same placement,
    valid sets included; cuts that would separate an affine input from a
    source its form uses are refused."""
    import json
    rng = np.random.default_rng(sum(map(ord, case)))
    if case == "fig3":
        with open(os.path.join(ROOT, "tests", "golden", "fig3_three_qubit.json")) as f:
            t = json.load(f)["circuit"]
        placement = "optimal"
    elif case == "big-optimal":
        t = w.cnot_layers(10, 3, 4700).to_text()
        placement = "optimal"
    else:
        name, placement = case.split("-")
        seed = int(name[4:])
        t = w.cnot_layers(2 + seed % 6, 2 + seed % 4, 4400 + seed).to_text()
    o = oracle.Feynman(t, placement)
    prog = fhs.Program(t, placement=placement)
    assert prog.A == o.A and prog.source_eval_positions == o.source_eval_positions
    n = o.n
    S = 1 + len(case) % 2
    inputs = [int(rng.integers(0, 1 << n)) for _ in range(S)]
    coeffs = [complex(rng.normal(), rng.normal()) for _ in range(S)]
    outs = list(range(1 << n)) if n <= 8 else [int(rng.integers(0, 1 << n)) for _ in range(64)]
    allowed = [c for c in range(prog.L, prog.G + 1) if prog.cut_allowed(c)]
    refused = [c for c in range(prog.L, prog.G + 1) if not prog.cut_allowed(c)]
    splits = sorted({(a, b) for a in allowed for b in allowed if a <= b})
    pick = [splits[int(i)] for i in rng.choice(len(splits), size=min(10, len(splits)), replace=False)]
    # the allowed cuts on both sides of each refused run
    for c in refused:
        lo = max([a for a in allowed if a < c], default=None)
        hi = min([a for a in allowed if a > c], default=None)
        if lo is not None and hi is not None:
            pick += [(lo, hi), (lo, lo), (hi, hi)]
    pick.append(prog.choose_partition(fhs.PART_EQ8))
    for thr in (0.0, 0.05):
        ref_a, ref_st = o.evaluate(inputs, coeffs, outs, threshold=thr, threads=THREADS)
        runs = [((0, 0), True, 0)] + [(p, False, 0) for p in pick] + [(p, False, 3) for p in pick[-3:]]
        for part, plain, dispatch in runs:
            ctx.set_launch_config(2 if dispatch else 1, 0, 0, dispatch)
            amps, st = gpu_eval(ctx, t, inputs, coeffs, outs, thr=thr, partition=part, plain=plain, prog=prog)
            assert np.abs(amps - ref_a).max() <= TOL, (case, thr, part, plain, dispatch)
            assert np.array_equal(st[:, :3], ref_st[:, :3].astype(np.uint64)), (case, thr, part, plain, dispatch)
    ctx.load(prog)
    for c in refused[:3]:
        with pytest.raises(fhs.FhsError):
            ctx.set_partition(c, prog.G)
        with pytest.raises(fhs.FhsError):
            ctx.set_partition(prog.L, c)
    ctx.set_launch_config(0, 0, 0, 0)


@pytest.mark.gpu
def test_reach_depth_first_prefix(ctx):
    """A prefix holding every source, enumerated partly depth first inside a
    lane (many pairs, few lanes per pair), under a greedy placement whose
    affine inputs use sources that lie deeper than themselves: the depth-first
    part is cut back to sources no earlier affine input uses, and the results
    equal the oracle's Algorithm 1."""
    t = w.cnot_layers(14, 4, 5002).to_text()
    o = oracle.Feynman(t, "greedy")
    prog = fhs.Program(t, placement="greedy")
    assert prog.A == o.A == 14
    assert any(not prog.cut_allowed(c) for c in range(prog.G + 1))
    rng = np.random.default_rng(5002)
    outs = [int(rng.integers(0, 1 << 14)) for _ in range(256)]
    ref_a, ref_st = o.evaluate([0], [1.0], outs, threads=THREADS)
    ctx.set_launch_config(1, 0, 0, 0)
    ctx.load(prog)
    for part in ((prog.G, prog.G), (0, 0)):
        ctx.set_partition(*part)
        plan = ctx.plan(len(outs), 1)
        if part[0] == prog.G:
            assert plan["Ap"] == 14
        amps, st = gpu_eval(ctx, t, [0], [1.0], outs, partition=part, prog=prog)
        assert np.abs(amps - ref_a).max() <= TOL, (part, plan)
        assert np.array_equal(st[:, :3], ref_st[:, :3].astype(np.uint64)), part
    ctx.set_launch_config(0, 0, 0, 0)


def test_walk_paper_coin_s2(ctx):
    """The paper's large walk: 100 qubits, 16 steps, the coin starting in
    (|0> + i|1>)/sqrt2 as two input bitstrings (S = 2, A = 15 per pair),
    2000 requested outputs: the reachable ones against the position-space
    closed form with that coin (normalised), their valid sets summed over
    both inputs (count and index sum doubled, xor-hash cancelled), padding
    exactly zero; at Eq. (8)'s split and at splits around it, interpreted
    and compiled."""
    cfg = w.CONFIGS["walk_99p_16s_s2"]()
    t = cfg["circuit"].to_text()
    coeffs = [complex(*z) for z in cfg["coeffs"]]
    prog = fhs.Program(t)
    r = 1 / math.sqrt(2)
    dp = cf.walk_amplitudes(16, (r, 1j * r))
    outs = cfg["outputs"]
    eq8 = prog.choose_partition(fhs.PART_EQ8)
    src = prog.source_eval_positions
    parts = [eq8, (src[4], src[9]), (src[6], src[11]), (0, 0)]
    for part in parts:
        for launch in ((0, 0, 0, 0), (2, 256, 0, 3), (1, 128, 0, 3)):
            ctx.set_launch_config(*launch)
            amps, st = gpu_eval(ctx, t, cfg["inputs"], coeffs, outs, partition=part, prog=prog)
            total = 0.0
            for y, a, row in zip(outs, amps, st):
                x = y >> 1
                x = x - (1 << 99) if x >= (1 << 98) else x
                ref = dp.get((x, y & 1))
                if ref is None:
                    assert a == 0 and int(row[0]) == 0, (part, launch, y)
                    continue
                total += abs(a) ** 2
                assert abs(a - ref) <= TOL, (part, launch, x, y & 1)
                n, sh, _ = cf.walk_valid_stats(16, x, y & 1)
                assert (int(row[0]), int(row[1]), int(row[2])) == (2 * n, (2 * sh) % (1 << 64), 0)
            assert abs(total - 1.0) <= 1e-10
    ctx.set_launch_config(0, 0, 0, 0)


def test_qft_dense_signal(ctx):
    """A dense real signal on 12 qubits (every basis state an input,
    S = 4096 pairs per output, one history each): every frequency bin
    against the discrete Fourier transform of the signal; only the two
    tones and their mirror bins are nonzero."""
    cfg = w.CONFIGS["qft_12q_dense"]()
    t = cfg["circuit"].to_text()
    coeffs = [complex(*z) for z in cfg["coeffs"]]
    x = np.array([c.real for c in coeffs])
    ref = cf.qft_dense(12, x)
    for plain in (False, True):
        amps, st = gpu_eval(ctx, t, cfg["inputs"], coeffs, cfg["outputs"], plain=plain)
        assert np.abs(amps - ref).max() <= TOL, plain
        assert sorted(np.nonzero(np.abs(amps) > 1e-9)[0].tolist()) == [5, 2001, 2095, 4091]
        assert (st[:, 0] == 4096).all()          # one valid history per (input, output) pair
