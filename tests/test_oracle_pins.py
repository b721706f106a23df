"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here runs GPU code.  Each test ties the oracle (state vector O1, the
C Feynman engine O2, the brute-force path sum) to something independent of
it: the paper's worked examples (tests/golden), textbook closed forms, gate
identities and invariants.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as w
from oracle import brute_force as bf
from oracle import closed_forms as cf
from oracle import statevector as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# gate matrices (O1) against identities that fix each convention
# --------------------------------------------------------------------------

def _u(text):
    return sv.unitary(text)


def test_gate_identities():
    I2 = np.eye(2)
    H = sv.gate_matrix("H", None)
    X = sv.gate_matrix("X", None)
    Y = sv.gate_matrix("Y", None)
    Z = sv.gate_matrix("Z", None)
    S = sv.gate_matrix("S", None)
    T = sv.gate_matrix("T", None)
    assert np.allclose(H @ H, I2)
    assert np.allclose(S @ S, Z)
    assert np.allclose(T @ T, S)
    assert np.allclose(sv.gate_matrix("SDG", None) @ S, I2)
    assert np.allclose(sv.gate_matrix("TDG", None) @ T, I2)
    assert np.allclose(H @ Z @ H, X)
    assert np.allclose(1j * X @ Z, Y)          # Y = i X Z
    th = 0.731
    # RX(pi) = -iX, RY(pi) = -iY, RZ(pi) = -iZ; RX = H RZ H
    assert np.allclose(sv.gate_matrix("RX", math.pi), -1j * X)
    assert np.allclose(sv.gate_matrix("RY", math.pi), -1j * Y)
    assert np.allclose(sv.gate_matrix("RZ", math.pi), -1j * Z)
    assert np.allclose(sv.gate_matrix("RX", th), H @ sv.gate_matrix("RZ", th) @ H)
    # exp(-i th/2 X) by its series definition
    assert np.allclose(sv.gate_matrix("RX", th), math.cos(th / 2) * I2 - 1j * math.sin(th / 2) * X)
    assert np.allclose(sv.gate_matrix("RY", th), math.cos(th / 2) * I2 - 1j * math.sin(th / 2) * Y)
    assert np.allclose(sv.gate_matrix("P", th), np.diag([1, np.exp(1j * th)]))
    for name, ang in [("H", None), ("RX", th), ("RY", th), ("RZ", th), ("P", th),
                      ("CP", th), ("RZZ", th), ("CX", None), ("SWAP", None), ("CCX", None),
                      ("CSWAP", None), ("CZ", None)]:
        u = sv.gate_matrix(name, ang)
        assert np.allclose(u.conj().T @ u, np.eye(len(u))), name


def test_two_qubit_conventions():
    th = 0.4137
    # CX a b: control a, target b (|a=1,b=0> -> |a=1,b=1>)
    u = _u("qubits 2\nCX 0 1\n")
    assert u[0b11, 0b01] == 1 and u[0b01, 0b01] == 0
    # RZZ(th) = CX . RZ(th) on the target . CX
    a = _u(f"qubits 2\nRZZ 0 1 {th.hex()}\n")
    b = _u(f"qubits 2\nCX 0 1\nRZ 1 {th.hex()}\nCX 0 1\n")
    assert np.allclose(a, b)
    # CP(pi) = CZ, symmetric in its qubits
    assert np.allclose(_u(f"qubits 2\nCP 0 1 {math.pi.hex()}\n"), _u("qubits 2\nCZ 0 1\n"))
    assert np.allclose(_u(f"qubits 2\nCP 1 0 {th.hex()}\n"), _u(f"qubits 2\nCP 0 1 {th.hex()}\n"))
    # SWAP = three CNOTs
    assert np.allclose(_u("qubits 2\nSWAP 0 1\n"), _u("qubits 2\nCX 0 1\nCX 1 0\nCX 0 1\n"))
    # CSWAP c a b = CX b a; CCX c a b; CX b a
    assert np.allclose(_u("qubits 3\nCSWAP 0 1 2\n"),
                       _u("qubits 3\nCX 2 1\nCCX 0 1 2\nCX 2 1\n"))
    # MCX with polarity = X-conjugated CCX; MCZ = H-conjugated MCX on the target
    assert np.allclose(_u("qubits 3\nMCX 2 ~0 1\n"), _u("qubits 3\nX 0\nCCX 0 1 2\nX 0\n"))
    assert np.allclose(_u("qubits 3\nMCZ 0 ~1 2\n"), _u("qubits 3\nX 1\nH 2\nCCX 0 1 2\nH 2\nX 1\n"))


# --------------------------------------------------------------------------
# the paper's worked examples
# --------------------------------------------------------------------------

def test_eq6_three_qubit_example():
    g = golden("eq6_three_qubit")
    F = oracle.Feynman(g["circuit"])
    assert F.A == g["A_backward"]
    for b, (re, im) in g["expected"].items():
        b = int(b)
        want = complex(re, im)
        amp, nv, *_ = F.pair(g["input"], b)
        assert abs(amp - want) <= 1e-15
        assert nv == g["n_valid"].get(str(b), 0)
        assert abs(sv.amplitudes(g["circuit"], [0], [1], [b])[0] - want) <= 1e-15
        assert abs(bf.path_sum(g["circuit"], 0, b)[0] - want) <= 1e-15


def test_fig2_four_qubit_example():
    g = golden("fig2_four_qubit")
    F = oracle.Feynman(g["circuit"])
    assert F.A == g["A_backward"]
    assert F.source_eval_positions == g["source_eval_positions"]
    assert [F.G - 1 - e for e in F.source_eval_positions] == g["source_time_index"]
    c1, c2 = g["partition"]
    assert (c1, c2 - c1, F.G - c2) == tuple(g["region_gates"])
    assert F.region_sources(c1, c2) == tuple(g["region_sources"])
    assert F.eq8(c1, c2) == g["eq8_partition"]
    assert F.eq8(0, 0) == g["eq8_plain"]
    b = lambda v, q: (v >> q) & 1
    for i in range(16):
        for o in range(16):
            a0, a1 = b(i, 0) ^ b(i, 1), b(i, 2)
            if b(o, 1) != b(i, 3):
                want, nv_want = 0.0, 0
            else:
                e = b(o, 0) * a0 + b(o, 3) * a1 + b(o, 1) + (b(o, 2) ^ a0) * b(i, 1)
                want, nv_want = (-1) ** e / (2 * math.sqrt(2)), 1
            for part in (None, (c1, c2)):
                amp, nv, sh, xh, _ = F.pair(i, o, partition=part)
                assert abs(amp - want) <= 1e-15
                assert nv == nv_want
                if nv:
                    assert sh == a0 | (a1 << 1)      # source k is bit k of h
                    assert xh == oracle.mix64(sh)


def test_fig3_backward_sources():
    g = golden("fig3_three_qubit")
    F = oracle.Feynman(g["circuit"])
    assert F.A == g["A_backward"]
    # the two sources are the final Hadamards (evaluation positions 0 and 1)
    assert sorted(F.source_eval_positions) == [0, 1]
    U = sv.unitary(g["circuit"])
    for i in range(8):
        amps, _ = F.evaluate([i], [1], list(range(8)))
        assert np.abs(amps - U[:, i]).max() <= 1e-15


def test_table1_backward_source_counts():
    g = golden("table1_sources")
    assert g["A_backward"]["qft"] == "0"
    for n in range(2, 13):
        assert oracle.Feynman(w.qft(n).to_text()).A == 0
    for k in (3, 4, 5, 6):
        for s in (1, 2, 3):
            c, _ = w.amplitude_amplification(k, s, 4 if k > 2 else 1, seed=7 + k)
            assert oracle.Feynman(c.to_text()).A == 2 * s * k
    for nv in (4, 6, 8, 12, 24):
        for p in (1, 2, 3):
            c, *_ = w.qaoa_maxcut(nv, p, 11, 12)
            assert oracle.Feynman(c.to_text()).A == p * nv
    for n_pos in (3, 8, 99):
        for s in (1, 2, 5, 20):
            assert oracle.Feynman(w.quantum_walk(n_pos, s).to_text()).A == s - 1


def test_table1_forward_source_counts():
    """Table I's forward column.  QFT: a source on the output side of every
    Hadamard whose qubit reaches the output through the final swaps (n for
    even n; for odd n the middle qubit is not swapped, its Hadamard's output
    segment is natural, n - 1).  Amplitude amplification and QAOA: the last
    layer of branching gates reaches the output directly, as the first layer
    reaches the input backward, so both columns agree.  Quantum walk: s when
    the coin-0 shift is written with X gates on the coin, which end the last
    Hadamard's output segment; with negatively controlled gates the coin
    reaches the output unchanged and the count is s - 1 both ways."""
    g = golden("table1_sources")
    assert g["A_forward"] == {"qft": "n", "amplitude_amplification": "2*s*n", "qaoa": "s*n",
                              "quantum_walk": "s"}
    for n in range(2, 13):
        assert oracle.Feynman(w.qft(n).to_text(), "forward").A == (n if n % 2 == 0 else n - 1)
    for k in (3, 4, 5, 6):
        for s in (1, 2, 3):
            c, _ = w.amplitude_amplification(k, s, 4, seed=7 + k)
            assert oracle.Feynman(c.to_text(), "forward").A == 2 * s * k
    for nv in (4, 6, 8, 12, 24):
        for p in (1, 2, 3):
            c, *_ = w.qaoa_maxcut(nv, p, 11, 12)
            assert oracle.Feynman(c.to_text(), "forward").A == p * nv
    for n_pos in (3, 8, 99):
        for s in (1, 2, 5, 20):
            xw = w.quantum_walk_xcoin(n_pos, s).to_text()
            assert oracle.Feynman(xw, "forward").A == s
            assert oracle.Feynman(xw).A == s - 1
            assert oracle.Feynman(w.quantum_walk(n_pos, s).to_text(), "forward").A == s - 1


def test_walk_constructions_agree():
    """The two walk constructions are the same unitary."""
    for n_pos, s in ((2, 3), (4, 4), (5, 2)):
        a = sv.unitary(w.quantum_walk(n_pos, s).to_text())
        b = sv.unitary(w.quantum_walk_xcoin(n_pos, s).to_text())
        assert np.abs(a - b).max() <= 1e-15


def test_forward_sources_on_output_side():
    """Forward placement on the paper's Fig. 2 circuit: sources sit on the
    output side of the Hadamards whose output segment does not reach the
    output, numbered from the input, and the amplitudes equal the backward
    placement's and the state vector's."""
    g = golden("fig2_four_qubit")
    t = g["circuit"]
    Fb, Ff = oracle.Feynman(t), oracle.Feynman(t, "forward")
    pos = Ff.source_eval_positions
    assert pos == sorted(pos)
    U = sv.unitary(t)
    for i in range(16):
        ab, _ = Fb.evaluate([i], [1], list(range(16)))
        af, _ = Ff.evaluate([i], [1], list(range(16)))
        assert np.abs(af - U[:, i]).max() <= 1e-15 and np.abs(af - ab).max() <= 1e-15


# --------------------------------------------------------------------------
# closed forms (pin O1 and O2 at sizes the state vector cannot reach)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_qft_closed_form_statevector(n):
    t = w.qft(n).to_text()
    U = sv.unitary(t)
    for x in range(1 << n):
        want = np.array([cf.qft_amplitude(n, x, y) for y in range(1 << n)])
        assert np.abs(U[:, x] - want).max() <= 1e-13


def test_qft20_closed_form_oracle():
    n = 20
    F = oracle.Feynman(w.qft(n).to_text())
    assert F.A == 0
    rng = np.random.default_rng(5)
    for _ in range(24):
        x, y = int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))
        amp, nv, *_ = F.pair(x, y)
        assert nv == 1
        assert abs(amp - cf.qft_amplitude(n, x, y)) <= 1e-12


@pytest.mark.parametrize("k,s", [(2, 1), (3, 1), (3, 2), (4, 3), (5, 3)])
def test_aa_closed_form_statevector(k, s):
    m = 1 if k == 2 else 4
    c, marked = w.amplitude_amplification(k, s, m, seed=3)
    t = c.to_text()
    psi = sv.evolve(t, 0)
    want = np.array([cf.aa_amplitude(k, s, marked, y) for y in range(1 << c.n)])
    assert np.abs(psi - want).max() <= 1e-12
    p = sum(abs(psi[y]) ** 2 for y in marked)
    assert abs(p - cf.aa_success_probability(k, s, m)) <= 1e-12


def test_aa_success_probabilities():
    # sin^2(7 theta), sin theta = sqrt(4/N): values quoted for N = 16, 32
    assert abs(cf.aa_success_probability(4, 3, 4) - 0.25) <= 1e-12
    assert abs(cf.aa_success_probability(5, 3, 4) - 0.330078125) <= 1e-9


def test_aa_closed_form_oracle_small():
    c, marked = w.amplitude_amplification(3, 2, 4, seed=3)
    F = oracle.Feynman(c.to_text())
    assert F.A == 12
    outs = list(range(1 << c.n))
    amps, st = F.evaluate([0], [1], outs, partition=F.eq8_argmin()[:2], threads=4)
    want = np.array([cf.aa_amplitude(3, 2, marked, y) for y in outs])
    assert np.abs(amps - want).max() <= 1e-12
    # every history is valid when the ancilla output bit is 0, none otherwise
    for y, s in zip(outs, st):
        assert int(s[0]) == ((1 << F.A) if (y >> 3) == 0 else 0)


def test_walk_closed_form_statevector():
    steps, n_pos = 5, 5
    t = w.quantum_walk(n_pos, steps).to_text()
    psi = sv.evolve(t, 0)
    dp = cf.walk_amplitudes(steps)
    for (x, c), a in dp.items():
        assert abs(psi[w.walk_state(n_pos, x, c)] - a) <= 1e-12
    assert abs(sum(abs(a) ** 2 for a in dp.values()) - 1) <= 1e-12


@pytest.mark.parametrize("n_pos,steps", [(6, 5), (99, 4), (99, 7)])
def test_walk_closed_form_oracle(n_pos, steps):
    F = oracle.Feynman(w.quantum_walk(n_pos, steps).to_text())
    assert F.A == steps - 1
    dp = cf.walk_amplitudes(steps)
    keys = [(x, c) for x in range(-steps - 2, steps + 3) for c in (0, 1)]
    outs = [w.walk_state(n_pos, x, c) for x, c in keys]
    for part in (None, F.eq8_argmin()[:2]):
        amps, st = F.evaluate([0], [1], outs, partition=part, threads=4)
        norm = 0.0
        for (x, c), a, s in zip(keys, amps, st):
            assert abs(a - dp.get((x, c), 0)) <= 1e-12
            assert int(s[0]) == cf.walk_n_valid(steps, x, c)
            assert tuple(int(v) for v in s[:3]) == cf.walk_valid_stats(steps, x, c)
            norm += abs(a) ** 2
        assert abs(norm - 1.0) <= 1e-12


# --------------------------------------------------------------------------
# O2 against O1 and the brute-force path sum
# --------------------------------------------------------------------------

def test_config_clifford_t_against_statevector():
    cfg = w.CONFIGS["clifford_t_10q_40g"]()
    t = cfg["circuit"].to_text()
    F = oracle.Feynman(t)
    amps, st = F.evaluate(cfg["inputs"], [complex(*z) for z in cfg["coeffs"]], cfg["outputs"])
    ref = sv.amplitudes(t, cfg["inputs"], [complex(*z) for z in cfg["coeffs"]], cfg["outputs"])
    assert np.abs(amps - ref).max() <= 1e-12


@pytest.mark.parametrize("seed", range(0, 600, 1))
def test_random_against_statevector(seed):
    n = 1 + seed % 6
    c = w.random_mixed(n, 4 + seed % 11, seed)
    t = c.to_text()
    F = oracle.Feynman(t)
    rng = np.random.default_rng(seed)
    S = 1 + seed % 3
    inputs = [int(v) for v in rng.choice(1 << n, size=min(S, 1 << n), replace=False)]
    coeffs = [complex(rng.normal(), rng.normal()) for _ in inputs]
    outs = list(range(1 << n))
    amps, _ = F.evaluate(inputs, coeffs, outs)
    ref = sv.amplitudes(t, inputs, coeffs, outs)
    assert np.abs(amps - ref).max() <= 1e-12


@pytest.mark.parametrize("seed", range(60))
def test_counts_and_threshold_against_brute_force(seed):
    n = 1 + seed % 4
    c = w.random_mixed(n, 3 + seed % 6, 1000 + seed)
    t = c.to_text()
    F = oracle.Feynman(t)
    rng = np.random.default_rng(seed)
    b_in = int(rng.integers(0, 1 << n))
    for thr in (0.0, 0.05, 0.3, 0.6):
        for b_out in range(1 << n):
            amp, nv, *_ = F.pair(b_in, b_out, threshold=thr)
            amp_b, nv_b = bf.path_sum(t, b_in, b_out, threshold=thr)
            assert nv == nv_b, (thr, b_out)
            assert abs(amp - amp_b) <= 1e-12


@pytest.mark.parametrize("seed", range(0, 300))
def test_forward_random_against_statevector(seed):
    """Forward placement (Table I's other column) reaches the same exact
    amplitudes on random circuits over the whole gate vocabulary."""
    n = 1 + seed % 6
    c = w.random_mixed(n, 4 + seed % 11, 7000 + seed)
    t = c.to_text()
    F = oracle.Feynman(t, "forward")
    rng = np.random.default_rng(seed)
    S = 1 + seed % 3
    inputs = [int(v) for v in rng.choice(1 << n, size=min(S, 1 << n), replace=False)]
    coeffs = [complex(rng.normal(), rng.normal()) for _ in inputs]
    outs = list(range(1 << n))
    amps, _ = F.evaluate(inputs, coeffs, outs)
    ref = sv.amplitudes(t, inputs, coeffs, outs)
    assert np.abs(amps - ref).max() <= 1e-12


@pytest.mark.parametrize("seed", range(40))
def test_forward_counts_and_threshold_against_brute_force(seed):
    """Valid-history counts and thresholded amplitudes under forward
    placement against the naive path sum with the modulus product taken from
    the input."""
    n = 1 + seed % 4
    c = w.random_mixed(n, 3 + seed % 6, 3000 + seed)
    t = c.to_text()
    F = oracle.Feynman(t, "forward")
    rng = np.random.default_rng(seed)
    b_in = int(rng.integers(0, 1 << n))
    for thr in (0.0, 0.05, 0.3, 0.6):
        for b_out in range(1 << n):
            amp, nv, *_ = F.pair(b_in, b_out, threshold=thr)
            amp_b, nv_b = bf.path_sum(t, b_in, b_out, threshold=thr, forward=True)
            assert nv == nv_b, (thr, b_out)
            assert abs(amp - amp_b) <= 1e-12


# --------------------------------------------------------------------------
# sparse and dense input states (Eq. (2) with S > 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_pos,steps", [(5, 4), (6, 5), (7, 6)])
def test_walk_complex_coin_statevector(n_pos, steps):
    """The walk from position 0 with the coin in (|0> + i|1>)/sqrt2 (the
    paper's large walk, Section V), as S = 2 basis inputs: the position-space
    recursion with that initial coin against the state vector of the
    superposition, and the oracle (Eq. (2)) against both."""
    r = 1 / math.sqrt(2)
    t = w.quantum_walk(n_pos, steps).to_text()
    ins = [w.walk_state(n_pos, 0, 0), w.walk_state(n_pos, 0, 1)]
    psi = np.zeros(1 << (n_pos + 1), dtype=complex)
    psi[ins[0]], psi[ins[1]] = r, 1j * r
    full = sv.evolve_state(t, psi)
    dp = cf.walk_amplitudes(steps, (r, 1j * r))
    assert abs(sum(abs(a) ** 2 for a in dp.values()) - 1.0) <= 1e-14
    for (x, c), a in dp.items():
        assert abs(full[w.walk_state(n_pos, x, c)] - a) <= 1e-14
    outs = list(range(1 << (n_pos + 1)))
    amps, _ = oracle.Feynman(t).evaluate(ins, [r, 1j * r], outs)
    assert np.abs(amps - full).max() <= 1e-13


def test_walk_complex_coin_large_closed_form():
    """The 100-qubit, 16-step walk from the paper's coin state: normalised
    over its reachable outputs; the oracle agrees on a sample of them, and
    each output's valid set (summed over the two inputs) is twice the
    single-input set: count and index sum doubled, xor-hash cancelled."""
    cfg = w.CONFIGS["walk_99p_16s_s2"]()
    t = cfg["circuit"].to_text()
    r = 1 / math.sqrt(2)
    dp = cf.walk_amplitudes(16, (r, 1j * r))
    assert len(dp) == 32 and abs(sum(abs(a) ** 2 for a in dp.values()) - 1.0) <= 1e-13
    F = oracle.Feynman(t)
    assert F.A == 15
    sample = [w.walk_state(99, x, c) for x, c in ((0, 0), (2, 1), (-6, 0), (14, 1), (16, 1))]
    amps, st = F.evaluate(cfg["inputs"], [complex(*z) for z in cfg["coeffs"]], sample, threads=4)
    for y, a, row in zip(sample, amps, st):
        x = y >> 1
        x = x - (1 << 99) if x >= (1 << 98) else x
        assert abs(a - dp[(x, y & 1)]) <= 1e-13
        n, sh, _ = cf.walk_valid_stats(16, x, y & 1)
        assert (int(row[0]), int(row[1]), int(row[2])) == (2 * n, (2 * sh) % (1 << 64), 0)


@pytest.mark.parametrize("n", [3, 6, 9, 12])
def test_qft_dense_input(n):
    """QFT of a dense real input: the state vector of the superposition
    against the discrete Fourier transform (FFT) of its amplitudes, and, at
    12 qubits, the workload's two tones at bins 5 and 2001 (with their
    mirror bins 4091 and 2095 for a real signal)."""
    rng = np.random.default_rng(n)
    psi = rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    t = w.qft(n).to_text()
    assert np.abs(sv.evolve_state(t, psi.astype(complex)) - cf.qft_dense(n, psi)).max() <= 1e-13
    if n == 12:
        cfg = w.CONFIGS["qft_12q_dense"]()
        x = np.array([z[0] for z in cfg["coeffs"]])
        a = cf.qft_dense(12, x)
        assert sorted(np.nonzero(np.abs(a) > 1e-12)[0].tolist()) == [5, 2001, 2095, 4091]
        assert abs(np.sum(np.abs(a) ** 2) - 1.0) <= 1e-13


# --------------------------------------------------------------------------
# source placement by reachability (Section IV-B, Fig. 3)
# --------------------------------------------------------------------------

def test_fig3_optimal_and_greedy_one_source():
    """Fig. 3: the backward sweep places two sources, the optimum one (on
    the merged node {w1, w2, w4, w5}; here the input segment of the final
    Hadamard on q1); both placements give the exact amplitudes and the same
    number of valid histories per pair (consistent wire assignments do not
    depend on where the sources sit)."""
    g = golden("fig3_three_qubit")
    t = g["circuit"]
    U = sv.unitary(t)
    Fb = oracle.Feynman(t)
    for pl in ("optimal", "greedy"):
        F = oracle.Feynman(t, pl)
        assert F.A == g["A_optimal"] == 1
        assert F.source_eval_positions == [0]
        for i in range(8):
            amps, st = F.evaluate([i], [1], list(range(8)))
            _, stb = Fb.evaluate([i], [1], list(range(8)))
            assert np.abs(amps - U[:, i]).max() <= 1e-15
            assert np.array_equal(st[:, 0], stb[:, 0])


@pytest.mark.parametrize("seed", range(40))
def test_reachability_placement_random(seed):
    """On random CNOT + one-qubit circuits: optimal <= greedy <= backward
    source counts, exact amplitudes against the state vector, and the
    valid-history counts of the backward placement and of the naive path
    sum."""
    n = 2 + seed % 4
    c = w.cnot_layers(n, 2 + seed % 3, 4400 + seed)
    t = c.to_text()
    Fb, Fo, Fg = (oracle.Feynman(t, p) for p in ("backward", "optimal", "greedy"))
    assert Fo.A <= Fg.A <= Fb.A
    rng = np.random.default_rng(seed)
    b_in = int(rng.integers(0, 1 << n))
    U = sv.evolve(t, b_in)
    outs = list(range(1 << n))
    ab, stb = Fb.evaluate([b_in], [1], outs)
    for F in (Fo, Fg):
        amps, st = F.evaluate([b_in], [1], outs)
        assert np.abs(amps - U).max() <= 1e-12
        assert np.array_equal(st[:, 0], stb[:, 0])
    if n <= 3 and len(c) <= 24:
        for y in outs:
            _, nv_b = bf.path_sum(t, b_in, y)
            assert int(stb[y, 0]) == nv_b


def test_reachability_placement_paper_families():
    """Section IV-B closes with backward propagation attaining the optimum
    on the paper's benchmark families; on the ones made of CNOT-like,
    diagonal and one-qubit gates (QFT, QAOA) the exhaustive search agrees."""
    for n in (3, 4, 6):
        assert oracle.Feynman(w.qft(n).to_text(), "optimal").A == 0
    for nv, p in ((4, 1), (4, 2), (6, 1), (6, 2)):
        t = w.qaoa_maxcut(nv, p, 11, 12)[0].to_text()
        assert oracle.Feynman(t, "optimal").A == oracle.Feynman(t).A == p * nv
        assert oracle.Feynman(t, "greedy").A == p * nv
