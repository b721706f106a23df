"""Host checks of ladder folding and pairing (fhs_reduce_ex with
FHS_REDUCE_FUSE and FHS_REDUCE_PAIR): the folded program keeps every
position, source, final-bit mask and Eq. (8) count of the gate-by-gate
program and only its work per history drops."""
import ctypes

import numpy as np
import pytest

import paper_2608_01467_amd as fhs
import workloads as w

CASES = [w.quantum_walk(99, 20).to_text(), w.quantum_walk(20, 9).to_text(),
         w.random_ladders(12, 10, 1).to_text(), w.random_ladders(45, 10, 2).to_text(),
         w.random_ladders(100, 10, 3).to_text(), w.random_mixed(9, 60, 4).to_text(),
         w.qaoa_maxcut(8, 2, 5, 6)[0].to_text()]


@pytest.mark.parametrize("text", CASES)
def test_fused_program_keeps_positions_and_eq8(text):
    a, b = fhs.Program(text, fuse=False), fhs.Program(text)
    assert (a.n, a.G, a.A, a.L, a.W, a.n_branch) == (b.n, b.G, b.A, b.L, b.W, b.n_branch)
    assert a.source_eval_positions == b.source_eval_positions
    assert a.candidate_splits() == b.candidate_splits()
    for c in a.candidate_splits()[::5]:
        assert a.partition_cost(*c) == b.partition_cost(*c)
        fa, fb = a.split_features(*c, 64, 1), b.split_features(*c, 64, 1)
        same = [0, 1, 2, 9, 10, 11, 12, 13]             # everything but the work features
        assert np.array_equal(fa[same], fb[same])
        assert (fb[3:9] <= fa[3:9]).all() and fb[14] <= fa[14]   # runs may split
    for k in (PART for PART in (fhs.PART_NONE, fhs.PART_THIRDS, fhs.PART_EQ8)):
        assert a.choose_partition(k) == b.choose_partition(k)
    wa, wb = a.work(0, a.G), b.work(0, b.G)
    assert wa["gates"] == wb["gates"] and wa["fp64_flops"] == wb["fp64_flops"]
    assert wa["branch"] == wb["branch"] and wb["int_ops"] <= wa["int_ops"]


def test_walk_ladders_fold_to_one_instruction_each():
    n_pos, steps = 99, 20
    a = fhs.Program(w.quantum_walk(n_pos, steps).to_text(), fuse=False)
    b = fhs.Program(w.quantum_walk(n_pos, steps).to_text(), pair=False)
    c = fhs.Program(w.quantum_walk(n_pos, steps).to_text())
    # the coin's H: its source bit into the state (1);
    # unfolded: the X on position bit i has controls up to qubit i (w words): 3w+1;
    # folded: one add per ladder, 3*1+1 for the coin control + 1 for the step;
    # paired: one add per walk step, the coin bit added to the count: 2, except
    # that a step whose coin still holds the source bit the Hadamard before it
    # (in evaluation order) set costs nothing and the run sums those bits with
    # one popcount of the source index (2): only the first step, whose coin
    # comes from the output, pays 2.  Either way every step adds to the same
    # 4-word position field and only the coin's H (outside the field) lies
    # between them: one run.  The run is still pending at the end, where
    # every position bit is compared with the input, so it costs a compare of
    # its count with the field's residue (2), not a carry chain (3 * 4)
    words = lambda hi: hi // 32 + 1
    unfolded = steps * (1 + 2 * sum(3 * words(i) + 1 for i in range(n_pos)))
    assert a.work(0, a.G)["int_ops"] == unfolded
    assert b.work(0, b.G)["int_ops"] == steps * (1 + 2 * (4 + 1)) + 2
    assert c.work(0, c.G)["int_ops"] == steps * 1 + 2 + 2 + 2
    # the part that depends only on the range's own sources: the 19 source
    # bits into the state (the coin's first H takes the input bit) and the
    # popcount of the source index; the compare with the field's residue
    # reads the state
    assert c.work(0, c.G)["src_int_ops"] == (steps - 1) + 2
    assert b.work(0, b.G)["src_int_ops"] == steps - 1
    assert c.work(half0 := c.source_eval_positions[0], half0 + 1)["src_int_ops"] == 1
    # a range that starts inside the run pays its own popcount and compare,
    # and the range that holds the run's start but stops short of the end
    # applies its part with a carry chain
    half = c.source_eval_positions[len(c.source_eval_positions) // 2]
    assert c.work(half, c.G)["int_ops"] + c.work(0, half)["int_ops"] == \
        c.work(0, c.G)["int_ops"] + 3 * 4 + 2
    # one instruction per ladder when folded, one per step when paired
    fb = b.split_features(b.L, b.G, 64, 1)
    fc = c.split_features(c.L, c.G, 64, 1)
    assert fc[14] < fb[14]


def test_mixed_circuits_without_ladders_are_unchanged():
    for seed in range(5):
        t = w.random_clifford_t(10, 60, seed).to_text()
        a, b = fhs.Program(t, fuse=False), fhs.Program(t)
        assert a.work(0, a.G) == b.work(0, b.G)


def test_reduce_ex_rejects_unknown_flags():
    t = b"qubits 2\nH 0\n"
    h = ctypes.c_void_p()
    assert fhs.lib().fhs_reduce_ex(t, len(t), 32, ctypes.byref(h)) == 1
    assert fhs.lib().fhs_reduce_ex(t, len(t), 2, ctypes.byref(h)) == 1   # pair needs fuse
    assert fhs.lib().fhs_reduce_ex(t, len(t), 8 | 16, ctypes.byref(h)) == 1   # one placement
    assert fhs.lib().fhs_reduce_ex(t, len(t), 4 | 8, ctypes.byref(h)) == 1
    for flags in (0, 1, 3, 4, 7, 8, 11, 16, 19):
        assert fhs.lib().fhs_reduce_ex(t, len(t), flags, ctypes.byref(h)) == 0
        fhs.lib().fhs_program_free(h)


def test_hoisted_suffix_work_qaoa():
    """The suffix instructions the compiled consumer evaluates once per root
    (fhs_work.hoist_*): with the cut after the last two first-layer RX gates
    in evaluation order (vertices 0 and 1 in time order: the suffix's sources), the
    first-layer RZZ phases on edges that avoid both vertices and the
    Hadamards on vertices no remaining gate reads; counted here from the
    graph alone."""
    for nv, seed in ((12, 401), (12, 31), (8, 5)):
        c, edges, _, _ = w.qaoa_maxcut(nv, 2, seed, seed + 1)
        p = fhs.Program(c.to_text())
        c2 = p.G - (nv + len(edges) + 2)     # suffix: 2 RX, the first RZZ layer, the H layer
        src = {0, 1}
        stay_edges = [e for e in edges if src & set(e)]
        touched = src | {q for e in stay_edges for q in e}
        k = len(edges) - len(stay_edges)
        m = nv - len(touched)
        wk = p.work(c2, p.G)
        assert p.source_eval_positions[-2:] == [c2, c2 + 1]
        # a phase: 3 int ops, 6 flops; a Hadamard: its input bit (1 op) and a
        # sign, its magnitude being common to every history (0 flops)
        assert (wk["hoist_int_ops"], wk["hoist_fp64_flops"]) == (3 * k + m, 6 * k), (nv, seed)
        # counted (fhs_work.count_*): every RZZ (two values, e^{+-i gamma}) and
        # RX (cos on the diagonal, -i sin off it) of the suffix, one int op
        # per phase and two per branching gate; the Hadamards stay signs
        assert (wk["count_int_ops"], wk["count_fp64_flops"]) == (len(edges) + 2 * 2, 6 * len(edges) + 2 * 2)
        assert (wk["hoist_count_int_ops"], wk["hoist_count_fp64_flops"]) == (k, 6 * k)
    # the walk's suffix has nothing to hoist: every gate reads the coin or the field
    t = w.quantum_walk(20, 6).to_text()
    q = fhs.Program(t)
    for c2 in q.source_eval_positions:
        assert q.work(c2, q.G)["hoist_int_ops"] == 0
        assert q.work(c2, q.G)["count_int_ops"] == 0   # H and permutations: nothing two-valued


@pytest.mark.parametrize("gate,extra", [
    ("T", 1), ("TDG", 1), ("S", 1), ("SDG", 1), ("Z", 1), ("P 0.7", 1), ("RZ 0.7", 1), ("P 0.0", 0),
    ("RX 0.7", 2), ("RY 0.7", 0), ("H", 0), ("Y", 1), ("X", 0),
    ("CZ", 1), ("CP 0.7", 1), ("RZZ 0.7", 1), ("CX", 0), ("SWAP", 0)])
def test_two_valued_gates_counted(gate, extra):
    """Which gates the compiled consumer can count (fhs_work.count_int_ops):
    tables with exactly two distinct entries (P(0) has one value, RY three);
    the Hadamards around the gate are real-entry branches, whose signs are
    collected instead."""
    name, *ang = gate.split()
    qs = "0 1" if name in ("CZ", "CP", "RZZ", "CX", "SWAP") else "0"
    text = "qubits 2\nH 0\nH 1\nRX 0 0.3\n" + " ".join([name, qs] + ang) + "\nH 0\nH 1\n"
    p = fhs.Program(text)
    wk = p.work(0, p.G)
    assert wk["count_int_ops"] == extra + 2, gate     # + the RX 0.3 before it
