"""Seeded synthetic circuits and output lists.

This module only *describes* inputs: gate lists, angles drawn from a seeded
generator, input bitstrings and requested output bitstrings.  It holds none of
the simulation arithmetic (no gate matrices, no amplitudes); both the CPU
oracle and the GPU library consume what it writes, each parsing the same text
format on its own.

Circuit text format (one gate per line, time order, '#' starts a comment)::

    qubits <n>
    H q | X q | Y q | Z q | S q | SDG q | T q | TDG q
    P q <angle> | RX q <angle> | RY q <angle> | RZ q <angle>
    CX c t | CZ a b | SWAP a b | CP a b <angle> | RZZ a b <angle>
    CCX c1 c2 t | CSWAP c a b
    MCX t c1 c2 ...      (a control written ~c is active when qubit c is 0)
    MCZ q1 q2 ...        (phase -1 when every qubit matches its polarity)

Angles are written as C99 hex floats so both parsers see identical bits.
Qubit q is bit q of a basis index (little-endian).  Bitstrings cross the C
boundary as ceil(n/64) uint64 words, word w holding bits 64w..64w+63.

The families follow the circuits the paper evaluates (Section IV-F and
Section V): QFT, amplitude amplification, QAOA MaxCut and a coined quantum
walk, plus a random Clifford+T circuit used as a correctness case.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Gate", "Circuit", "random_clifford_t", "random_mixed", "random_ladders", "qft", "amplitude_amplification",
    "qaoa_maxcut", "quantum_walk", "quantum_walk_xcoin", "random_outputs", "bits_to_words",
    "words_to_bits", "n_words", "three_regular_graph", "reachable_outputs", "CONFIGS",
]


@dataclass(frozen=True)
class Gate:
    name: str
    qubits: Tuple[int, ...]
    negs: Tuple[bool, ...] = ()      # per qubit: negative-polarity control
    angle: Optional[float] = None

    def to_text(self) -> str:
        toks = [self.name]
        negs = self.negs or (False,) * len(self.qubits)
        for q, ng in zip(self.qubits, negs):
            toks.append(("~" if ng else "") + str(q))
        if self.angle is not None:
            toks.append(float(self.angle).hex())
        return " ".join(toks)


@dataclass
class Circuit:
    n: int
    gates: List[Gate] = field(default_factory=list)

    def add(self, name: str, *qubits: int, angle: Optional[float] = None,
            negs: Sequence[bool] = ()) -> None:
        for q in qubits:
            if not 0 <= q < self.n:
                raise ValueError(f"qubit {q} out of range for n={self.n}")
        if len(set(qubits)) != len(qubits):
            raise ValueError(f"repeated qubit in {name} {qubits}")
        self.gates.append(Gate(name, tuple(qubits), tuple(negs), angle))

    def to_text(self) -> str:
        lines = [f"qubits {self.n}"]
        lines += [g.to_text() for g in self.gates]
        return "\n".join(lines) + "\n"

    def __len__(self) -> int:
        return len(self.gates)


def n_words(n: int) -> int:
    return max(1, (n + 63) // 64)


def bits_to_words(values: Sequence[int], n: int) -> np.ndarray:
    """Python ints -> (len, ceil(n/64)) uint64 array, little-endian words."""
    w = n_words(n)
    out = np.zeros((len(values), w), dtype=np.uint64)
    mask = (1 << 64) - 1
    for i, v in enumerate(values):
        if v < 0 or v >> n:
            raise ValueError(f"bitstring {v:#x} does not fit in {n} bits")
        for j in range(w):
            out[i, j] = (v >> (64 * j)) & mask
    return out


def words_to_bits(words: np.ndarray) -> List[int]:
    words = np.asarray(words, dtype=np.uint64)
    res = []
    for row in words.reshape(len(words), -1):
        v = 0
        for j, x in enumerate(row):
            v |= int(x) << (64 * j)
        res.append(v)
    return res


def random_outputs(n: int, count: int, seed: int,
                   exclude: Sequence[int] = ()) -> List[int]:
    """`count` distinct uniform n-bit strings, none in `exclude`."""
    rng = np.random.default_rng(seed)
    seen = set(exclude)
    out: List[int] = []
    if count > (1 << n) - len(seen):
        raise ValueError("not enough distinct bitstrings")
    while len(out) < count:
        v = 0
        for j in range(0, n, 32):
            width = min(32, n - j)
            v |= int(rng.integers(0, 1 << width)) << j
        if v not in seen:
            seen.add(v)
            out.append(v)
    return out


# ---------------------------------------------------------------------------
# Circuit families
# ---------------------------------------------------------------------------

def random_mixed(n: int, n_gates: int, seed: int, max_controls: int = 3) -> Circuit:
    """Random circuit over the whole gate vocabulary (test coverage case):
    every fixed gate, random angles, MCX/MCZ with random polarities."""
    rng = np.random.default_rng(seed)
    one = ["H", "X", "Y", "Z", "S", "SDG", "T", "TDG"]
    one_a = ["P", "RX", "RY", "RZ"]
    two = ["CX", "CZ", "SWAP"]
    two_a = ["CP", "RZZ"]
    three = ["CCX", "CSWAP"]
    pool = one + one_a + (two + two_a if n >= 2 else []) + (three if n >= 3 else []) \
        + (["MCX", "MCZ"] if n >= 2 else [])
    c = Circuit(n)
    for _ in range(n_gates):
        k = pool[int(rng.integers(0, len(pool)))]
        if k in one:
            c.add(k, int(rng.integers(0, n)))
        elif k in one_a:
            c.add(k, int(rng.integers(0, n)), angle=float(rng.uniform(-math.pi, math.pi)))
        elif k in two or k in two_a:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            ang = float(rng.uniform(-math.pi, math.pi)) if k in two_a else None
            c.add(k, a, b, angle=ang)
        elif k in three:
            a, b, d = (int(x) for x in rng.choice(n, size=3, replace=False))
            c.add(k, a, b, d)
        else:
            m = int(rng.integers(2, min(n, max_controls + 1) + 1))
            qs = [int(x) for x in rng.choice(n, size=m, replace=False)]
            negs = [bool(rng.integers(0, 2)) for _ in qs]
            if k == "MCX":
                negs[0] = False
            c.add(k, *qs, negs=negs)
    return c


def random_ladders(n: int, n_ladders: int, seed: int, n_extra: int = 4) -> Circuit:
    """Random circuit built around add/subtract-one ladders (test coverage
    for ladder folding): each ladder is preceded by an H on a random qubit
    and a few random one- and two-qubit gates, then adds or subtracts one on
    a random block of consecutive qubits under 0-2 extra controls of random
    polarity, written as the walk writes it (MCX from the top bit down).
    Some ladders are broken on purpose (one gate with a wrong control) so
    that partial ladders occur too."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(n_ladders):
        c.add("H", int(rng.integers(0, n)))
        for _ in range(int(rng.integers(0, n_extra + 1))):
            k = ["T", "S", "CX", "CZ", "X"][int(rng.integers(0, 5))]
            if k in ("CX", "CZ"):
                a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
                c.add(k, a, b)
            else:
                c.add(k, int(rng.integers(0, n)))
        m = int(rng.integers(2, min(n - 1, 40) + 1))
        lo = int(rng.integers(0, n - m + 1))
        block = list(range(lo, lo + m))
        rest = [q for q in range(n) if q < lo or q >= lo + m]
        n_k = int(rng.integers(0, min(2, len(rest)) + 1))
        ks = [int(x) for x in rng.choice(rest, size=n_k, replace=False)] if n_k else []
        kneg = [bool(rng.integers(0, 2)) for _ in ks]
        neg = bool(rng.integers(0, 2))         # False: add one, True: subtract one
        broken = int(rng.integers(0, m)) if rng.random() < 0.25 else -1
        for i in range(m - 1, -1, -1):
            ctrls = ks + block[:i]
            negs = [False] + kneg + [neg] * i
            if i == broken and i > 0:
                negs[-1] = not neg
            c.add("MCX", block[i], *ctrls, negs=tuple(negs))
    return c


def random_ladder_pairs(n: int, n_pairs: int, seed: int, n_extra: int = 3) -> Circuit:
    """Random circuit built around pairs of add/subtract-one ladders on one
    block of consecutive qubits whose controls differ only in the polarity
    of a selector qubit outside the block (the shape of a coined walk's
    shift), under 0-2 further common controls of random polarity and with
    each ladder's direction random.  Every pair is preceded by an H on its
    selector qubit and a few random gates.  Some pairs are broken on purpose
    (the second ladder on a shifted block, or with its selector polarity
    equal to the first's) so that unpairable neighbours occur too."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)

    def ladder(block, ks, kneg, neg):
        for i in range(len(block) - 1, -1, -1):
            c.add("MCX", block[i], *(ks + block[:i]),
                  negs=tuple([False] + kneg + [neg] * i))

    for _ in range(n_pairs):
        m = int(rng.integers(2, min(n - 2, 40) + 1))
        lo = int(rng.integers(0, n - m + 1))
        block = list(range(lo, lo + m))
        rest = [q for q in range(n) if q < lo or q >= lo + m]
        sel = int(rng.choice(rest))
        c.add("H", sel)
        for _ in range(int(rng.integers(0, n_extra + 1))):
            k = ["T", "S", "CX", "CZ", "X"][int(rng.integers(0, 5))]
            if k in ("CX", "CZ"):
                a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
                c.add(k, a, b)
            else:
                c.add(k, int(rng.integers(0, n)))
        others = [q for q in rest if q != sel]
        n_k = int(rng.integers(0, min(2, len(others)) + 1))
        ks = [int(x) for x in rng.choice(others, size=n_k, replace=False)] if n_k else []
        kneg = [bool(rng.integers(0, 2)) for _ in ks]
        p0 = bool(rng.integers(0, 2))
        broken = rng.random() < 0.2
        block2 = block
        p1 = not p0
        if broken and lo + m < n and lo + m not in [sel] + ks:
            block2 = list(range(lo + 1, lo + m + 1))
        elif broken:
            p1 = p0
        ladder(block, [sel] + ks, [p0] + kneg, bool(rng.integers(0, 2)))
        ladder(block2, [sel] + ks, [p1] + kneg, bool(rng.integers(0, 2)))
    return c


def random_clifford_t(n: int = 10, n_gates: int = 40, seed: int = 101) -> Circuit:
    """Random Clifford+T circuit: H 30%, T 20%, S 10%, CNOT 30%, CZ 10%,
    qubits uniform, two-qubit gates on a distinct ordered pair."""
    rng = np.random.default_rng(seed)
    kinds = ["H", "T", "S", "CX", "CZ"]
    probs = [0.30, 0.20, 0.10, 0.30, 0.10]
    c = Circuit(n)
    for _ in range(n_gates):
        k = kinds[int(rng.choice(len(kinds), p=probs))]
        if k in ("CX", "CZ"):
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            c.add(k, a, b)
        else:
            c.add(k, int(rng.integers(0, n)))
    return c


def cnot_layers(n: int, layers: int, seed: int) -> Circuit:
    """Random circuit from the gate set the reachability placement covers:
    per layer, Hadamards and RX/RY on half the qubits (branching), n CNOTs
    or SWAPs on random pairs, then X/Z/T/P on a third of the qubits."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(layers):
        for q in rng.choice(n, size=max(1, n // 2), replace=False):
            g = str(rng.choice(["H", "H", "RX", "RY"]))
            if g == "H":
                c.add(g, int(q))
            else:
                c.add(g, int(q), angle=float(rng.uniform(-np.pi, np.pi)))
        for _ in range(n):
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            c.add(str(rng.choice(["CX", "CX", "CX", "SWAP"])), a, b)
        for q in rng.choice(n, size=max(1, n // 3), replace=False):
            g = str(rng.choice(["X", "Z", "T", "P"]))
            if g == "P":
                c.add(g, int(q), angle=float(rng.uniform(-np.pi, np.pi)))
            else:
                c.add(g, int(q))
    return c


def qft(n: int) -> Circuit:
    """Textbook QFT network in little-endian qubit order: for the most
    significant qubit down to qubit 0, a Hadamard followed by controlled phase
    R_k = P(2*pi/2^k) from every less significant qubit, then the qubit
    reversal by swaps.  It maps |x> to 2^{-n/2} sum_y e^{2 pi i x y / 2^n}|y>."""
    c = Circuit(n)
    for j in range(n - 1, -1, -1):
        c.add("H", j)
        for m in range(j - 1, -1, -1):
            k = j - m + 1
            c.add("CP", m, j, angle=2.0 * math.pi / float(1 << k))
    for i in range(n // 2):
        c.add("SWAP", i, n - 1 - i)
    return c


def _mcz_ladder(c: Circuit, qs: Sequence[int], anc: Sequence[int]) -> None:
    """Z on |1...1> of qubits `qs` using a Toffoli ladder over ancillas `anc`
    (len(qs) - 2 of them, all starting and ending in |0>)."""
    k = len(qs)
    if k == 1:
        c.add("Z", qs[0])
        return
    if k == 2:
        c.add("CZ", qs[0], qs[1])
        return
    assert len(anc) >= k - 2
    ladder = [(qs[0], qs[1], anc[0])]
    for i in range(2, k - 1):
        ladder.append((qs[i], anc[i - 2], anc[i - 1]))
    for a, b, t in ladder:
        c.add("CCX", a, b, t)
    c.add("CZ", qs[k - 1], anc[k - 3])
    for a, b, t in reversed(ladder):
        c.add("CCX", a, b, t)


def amplitude_amplification(k: int, iterations: int = 3, n_marked: int = 4,
                            seed: int = 301) -> Tuple[Circuit, List[int]]:
    """Grover-type amplitude amplification on k search qubits (0..k-1) with
    k-2 ancillas (k..2k-3).  Oracle: X-conjugated ladder-MCZ per marked state.
    Diffusion: H X MCZ X H on the search register.  Returns the circuit and
    the sorted marked states."""
    rng = np.random.default_rng(seed)
    marked = sorted(int(x) for x in rng.choice(1 << k, size=n_marked, replace=False))
    n = k + max(0, k - 2)
    qs = list(range(k))
    anc = list(range(k, n))
    c = Circuit(n)
    for q in qs:
        c.add("H", q)
    for _ in range(iterations):
        for m in marked:
            zeros = [q for q in qs if not (m >> q) & 1]
            for q in zeros:
                c.add("X", q)
            _mcz_ladder(c, qs, anc)
            for q in zeros:
                c.add("X", q)
        for q in qs:
            c.add("H", q)
        for q in qs:
            c.add("X", q)
        _mcz_ladder(c, qs, anc)
        for q in qs:
            c.add("X", q)
        for q in qs:
            c.add("H", q)
    return c, marked


def three_regular_graph(nv: int, seed: int) -> List[Tuple[int, int]]:
    """Random 3-regular simple graph by the pairing (configuration) model,
    rejecting matchings with loops or repeated edges."""
    if (3 * nv) % 2:
        raise ValueError("3-regular graph needs an even vertex count")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(nv), 3)
    for _ in range(100000):
        perm = rng.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        edges = set()
        ok = True
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in edges:
                ok = False
                break
            edges.add(e)
        if ok:
            return sorted(edges)
    raise RuntimeError("pairing model did not produce a simple graph")


def qaoa_maxcut(nv: int, p: int, graph_seed: int = 401, angle_seed: int = 402
                ) -> Tuple[Circuit, List[Tuple[int, int]], List[float], List[float]]:
    """QAOA for MaxCut on a random 3-regular graph: H on every vertex, then
    for each layer RZZ(2 gamma) per edge and RX(2 beta) per vertex; gamma and
    beta are uniform in [0, pi)."""
    edges = three_regular_graph(nv, graph_seed)
    rng = np.random.default_rng(angle_seed)
    gammas = [float(x) for x in rng.uniform(0.0, math.pi, size=p)]
    betas = [float(x) for x in rng.uniform(0.0, math.pi, size=p)]
    c = Circuit(nv)
    for v in range(nv):
        c.add("H", v)
    for layer in range(p):
        for a, b in edges:
            c.add("RZZ", a, b, angle=2.0 * gammas[layer])
        for v in range(nv):
            c.add("RX", v, angle=2.0 * betas[layer])
    return c, edges, gammas, betas


def quantum_walk(n_pos: int, steps: int) -> Circuit:
    """Coined walk on a cycle of 2^n_pos sites.  Qubit 0 is the coin, qubits
    1..n_pos the position register (qubit 1 least significant).  Each step:
    H on the coin, then +1 on the position when the coin is 1 and -1 when it
    is 0, each built as a cascade of multi-controlled X gates from the most
    significant position bit down."""
    n = n_pos + 1
    c = Circuit(n)
    pos = list(range(1, n))
    for _ in range(steps):
        c.add("H", 0)
        for i in range(n_pos - 1, -1, -1):
            ctrls = [0] + pos[:i]
            c.add("MCX", pos[i], *ctrls, negs=(False,) * (1 + len(ctrls)))
        for i in range(n_pos - 1, -1, -1):
            ctrls = [0] + pos[:i]
            c.add("MCX", pos[i], *ctrls, negs=(False,) + (True,) * len(ctrls))
    return c


def quantum_walk_xcoin(n_pos: int, steps: int) -> Circuit:
    """The same walk with the coin-0 shift written as X on the coin, the
    positively controlled decrement cascade, and X on the coin again (the
    same unitary as quantum_walk; the X gates are deterministic, so the coin
    wire's segments end at them)."""
    n = n_pos + 1
    c = Circuit(n)
    pos = list(range(1, n))
    for _ in range(steps):
        c.add("H", 0)
        for i in range(n_pos - 1, -1, -1):
            ctrls = [0] + pos[:i]
            c.add("MCX", pos[i], *ctrls, negs=(False,) * (1 + len(ctrls)))
        c.add("X", 0)
        for i in range(n_pos - 1, -1, -1):
            ctrls = [0] + pos[:i]
            c.add("MCX", pos[i], *ctrls, negs=(False, False) + (True,) * (len(ctrls) - 1))
        c.add("X", 0)
    return c


def walk_state(n_pos: int, x: int, coin: int) -> int:
    """Basis index of position x (mod 2^n_pos) with the given coin bit."""
    return ((x % (1 << n_pos)) << 1) | (coin & 1)


def walk_outputs(n_pos: int, steps: int, total: int, seed: int = 501) -> List[int]:
    """Every reachable (position, coin) after `steps` steps from position 0,
    in order of position then coin, padded with seeded random unreachable
    states up to `total`."""
    reach = []
    for x in range(-steps, steps + 1, 2):
        for coin in (0, 1):
            reach.append(walk_state(n_pos, x, coin))
    if total < len(reach):
        return reach[:total]
    pad = random_outputs(n_pos + 1, total - len(reach), seed, exclude=reach)
    return reach + pad


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def _cfg_clifford_t():
    c = random_clifford_t(10, 40, seed=101)
    return dict(circuit=c, inputs=[0], coeffs=[(1.0, 0.0)],
                outputs=random_outputs(10, 16, seed=102), threshold=0.0)


def reachable_outputs(c: Circuit, count: int, seed: int) -> List[int]:
    """Up to `count` distinct outputs reachable from |0...0>: the circuit
    followed forward with a random bit after every branching gate (H, RX,
    RY) and every permutation applied (phases ignored)."""
    rng = np.random.default_rng(seed)
    outs: List[int] = []
    seen = set()
    for _ in range(count * 8):
        x = 0
        for g in c.gates:
            q = g.qubits
            if g.name in ("H", "RX", "RY"):
                x = (x & ~(1 << q[0])) | (int(rng.integers(0, 2)) << q[0])
            elif g.name == "X":
                x ^= 1 << q[0]
            elif g.name == "CX" and (x >> q[0]) & 1:
                x ^= 1 << q[1]
            elif g.name == "SWAP" and ((x >> q[0]) ^ (x >> q[1])) & 1:
                x ^= (1 << q[0]) | (1 << q[1])
        if x not in seen:
            seen.add(x)
            outs.append(x)
            if len(outs) >= count:
                break
    return outs


def _cfg_clifford_t_large(n: int = 20, n_gates: int = 90, n_out: int = 4096):
    """A larger random Clifford+T circuit (same gate mix) for the cost
    distribution over outputs: half the outputs reachable from |0>, half
    uniform (most of which exact pruning rejects early)."""
    c = random_clifford_t(n, n_gates, seed=101)
    reach = reachable_outputs(c, n_out // 2, seed=103)
    outs = reach + random_outputs(n, n_out - len(reach), seed=102, exclude=reach)
    return dict(circuit=c, inputs=[0], coeffs=[(1.0, 0.0)], outputs=outs, threshold=0.0)


def _cfg_qft(n: int = 20, n_out: int = 256):
    rng = np.random.default_rng(201)
    x = int(rng.integers(0, 1 << n))
    return dict(circuit=qft(n), inputs=[x], coeffs=[(1.0, 0.0)],
                outputs=random_outputs(n, n_out, seed=202), threshold=0.0)


def _cfg_aa(k: int = 4, iterations: int = 3, n_out: Optional[int] = None):
    c, marked = amplitude_amplification(k, iterations, 4, seed=301)
    n = c.n
    if n_out is None:
        outs = list(range(1 << n))
    else:
        outs = list(marked) + random_outputs(n, n_out - len(marked), seed=302,
                                             exclude=marked)
    return dict(circuit=c, inputs=[0], coeffs=[(1.0, 0.0)], outputs=outs,
                threshold=0.0, marked=marked)


def _cfg_qaoa(nv: int = 12, p: int = 2, n_out: int = 4096, threshold: float = 0.0):
    c, edges, g, b = qaoa_maxcut(nv, p, 401, 402)
    if n_out >= (1 << nv):
        outs = list(range(1 << nv))
    else:
        outs = random_outputs(nv, n_out, seed=403)
    return dict(circuit=c, inputs=[0], coeffs=[(1.0, 0.0)], outputs=outs,
                threshold=threshold, edges=edges)


def _cfg_walk(n_pos: int = 99, steps: int = 20, total: int = 8192):
    c = quantum_walk(n_pos, steps)
    return dict(circuit=c, inputs=[0], coeffs=[(1.0, 0.0)],
                outputs=walk_outputs(n_pos, steps, total, seed=501), threshold=0.0)


def _cfg_walk_coin(n_pos: int = 99, steps: int = 16, total: int = 2000):
    """The paper's large walk (Section V): position 0 with the coin in
    (|0> + i|1>)/sqrt2, i.e. two input bitstrings (S = 2), 16 steps
    (A = 15 per pair), 2000 requested outputs (the reachable ones first)."""
    c = quantum_walk(n_pos, steps)
    r = 1.0 / math.sqrt(2.0)
    return dict(circuit=c, inputs=[walk_state(n_pos, 0, 0), walk_state(n_pos, 0, 1)],
                coeffs=[(r, 0.0), (0.0, r)], outputs=walk_outputs(n_pos, steps, total, seed=502),
                threshold=0.0)


def _cfg_qft_dense(n: int = 12):
    """QFT of a dense real signal on 12 qubits (every basis state an input,
    S = 4096), the shape of the paper's frequency-analysis example (its
    signal is not given): two tones at bins 5 and 2001, amplitudes
    normalised; every bin requested."""
    N = 1 << n
    t = np.arange(N)
    x = np.cos(2 * math.pi * 5 * t / N) + 0.5 * np.cos(2 * math.pi * 2001 * t / N)
    x = x / np.linalg.norm(x)
    return dict(circuit=qft(n), inputs=list(range(N)), coeffs=[(float(v), 0.0) for v in x],
                outputs=list(range(N)), threshold=0.0)


CONFIGS = {
    "clifford_t_10q_40g": _cfg_clifford_t,
    "clifford_t_20q_90g": _cfg_clifford_t_large,
    "qft_20q": _cfg_qft,
    "aa_k4_s3": lambda: _cfg_aa(4, 3),
    "aa_k5_s3": lambda: _cfg_aa(5, 3),
    "aa_k16_s3": lambda: _cfg_aa(16, 3, n_out=1024),
    "qaoa_12v_p2": lambda: _cfg_qaoa(12, 2, 4096),
    "qaoa_24v_p2": lambda: _cfg_qaoa(24, 2, 4096),
    "walk_99p_20s": _cfg_walk,
    "walk_99p_16s_s2": _cfg_walk_coin,
    "qft_12q_dense": _cfg_qft_dense,
}
