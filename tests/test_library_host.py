"""Host-side checks of the native library (no GPU needed).

  * libfhs.so loads and exports every function include/fhs.h declares;
  * the host reducer's placement (A, source positions, leading gates) and
    Eq. (8) agree with the independent C oracle;
  * argument and range errors come back as status codes.
"""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2608_01467_amd as fhs
import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fhs.h")).read()
    return sorted(set(re.findall(r"\b(fhs_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = fhs.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(fhs.EXPORTS)


def _circuits():
    yield "eq6", "qubits 3\nH 0\nCX 0 1\nS 1\nCX 1 2\n"
    for seed in range(80):
        n = [1, 3, 6, 12, 33, 64, 65, 100, 128][seed % 9]
        yield f"mixed{seed}", w.random_mixed(n, 10 + seed % 30, 900 + seed, max_controls=5).to_text()
    yield "qft12", w.qft(12).to_text()
    yield "aa4", w.amplitude_amplification(4, 3, 4, 301)[0].to_text()
    yield "aa16", w.amplitude_amplification(16, 3, 4, 301)[0].to_text()
    yield "qaoa12", w.qaoa_maxcut(12, 2)[0].to_text()
    yield "qaoa24", w.qaoa_maxcut(24, 2)[0].to_text()
    yield "walk", w.quantum_walk(99, 20).to_text()


@pytest.mark.parametrize("name,text", list(_circuits()), ids=[c[0] for c in _circuits()])
def test_reducer_matches_oracle_placement(name, text):
    p = fhs.Program(text)
    o = oracle.Feynman(text)
    assert (p.n, p.G, p.A) == (o.n, o.G, o.A)
    assert p.source_eval_positions == o.source_eval_positions
    assert p.L == (o.source_eval_positions[0] if o.A else o.G)
    rng = np.random.default_rng(len(text))
    for _ in range(20):
        c1, c2 = sorted(int(x) for x in rng.integers(0, p.G + 1, size=2))
        cost, reg = p.partition_cost(c1, c2)
        assert cost == o.eq8(c1, c2)
        assert reg[:3] == (c1, c2 - c1, p.G - c2)
        assert reg[3:] == o.region_sources(c1, c2)
    if p.G <= 1500:
        c1, c2, cost = o.eq8_argmin()
        assert p.choose_partition(fhs.PART_EQ8) == (c1, c2)
        assert p.partition_cost(c1, c2)[0] == cost
    assert p.choose_partition(fhs.PART_THIRDS) == (p.G // 3, 2 * p.G // 3)
    assert p.choose_partition(fhs.PART_NONE) == (0, 0)


def _forward_circuits():
    for seed in range(30):
        n = [1, 3, 6, 12, 33, 64, 65, 100, 128][seed % 9]
        yield f"mixed{seed}", w.random_mixed(n, 10 + seed % 30, 1900 + seed, max_controls=5).to_text()
    for n in (4, 7, 12):
        yield f"qft{n}", w.qft(n).to_text()
    yield "aa4", w.amplitude_amplification(4, 3, 4, 301)[0].to_text()
    yield "qaoa12", w.qaoa_maxcut(12, 2)[0].to_text()
    yield "walk_xcoin", w.quantum_walk_xcoin(20, 6).to_text()


@pytest.mark.parametrize("name,text", list(_forward_circuits()), ids=[c[0] for c in _forward_circuits()])
def test_forward_reducer_matches_oracle(name, text):
    """FHS_REDUCE_FORWARD places the same sources, at the same positions
    (counted from the input), as the oracle's forward sweep; Eq. (8) over
    time-order cuts agrees."""
    p = fhs.Program(text, forward=True)
    o = oracle.Feynman(text, "forward")
    assert p.forward
    assert (p.n, p.G, p.A) == (o.n, o.G, o.A)
    assert p.source_eval_positions == o.source_eval_positions
    rng = np.random.default_rng(len(text))
    for _ in range(10):
        c1, c2 = sorted(int(x) for x in rng.integers(0, p.G + 1, size=2))
        assert p.partition_cost(c1, c2)[0] == o.eq8(c1, c2)
        assert p.partition_cost(c1, c2)[1][3:] == o.region_sources(c1, c2)


def test_walk_eq8_argmin_matches_oracle():
    t = w.quantum_walk(99, 20).to_text()
    p, o = fhs.Program(t), oracle.Feynman(t)
    c1, c2, cost = o.eq8_argmin()
    assert p.choose_partition(fhs.PART_EQ8) == (c1, c2)
    assert p.partition_cost(c1, c2)[0] == cost
    assert cost < p.partition_cost(0, 0)[0] // 6


@pytest.mark.parametrize("text,status", [
    ("", 7),
    ("H 0\n", 7),
    ("qubits 0\n", 3),
    ("qubits 129\n", 3),
    ("qubits 2\nH 2\n", 3),
    ("qubits 2\nFOO 0\n", 2),
    ("qubits 2\nRX 0\n", 7),
    ("qubits 2\nH 0 0x1p+0\n", 7),
    ("qubits 2\nCX 0 0\n", 7),
    ("qubits 2\nCX ~0 1\n", 7),
    ("qubits 2\nMCX ~0 1\n", 7),
    ("qubits 2\nRX 0 nan\n", 7),
    ("qubits 2\nqubits 2\n", 7),
])
def test_reduce_errors(text, status):
    with pytest.raises(fhs.FhsError) as ei:
        fhs.Program(text)
    assert ei.value.status == status


def test_partition_cost_errors_and_large_A():
    p = fhs.Program(w.amplitude_amplification(16, 3, 4, 301)[0].to_text())
    assert p.A == 96
    assert p.partition_cost(0, 0)[0] == (2 ** 96) * p.G      # needs 128 bits
    with pytest.raises(fhs.FhsError) as ei:
        p.partition_cost(5, 4)
    assert ei.value.status == 1
    with pytest.raises(fhs.FhsError):
        p.partition_cost(0, p.G + 1)


def test_empty_circuit():
    p = fhs.Program("qubits 5\n")
    assert (p.G, p.A, p.L) == (0, 0, 0)
    assert p.partition_cost(0, 0)[0] == 0



def _reach_circuits():
    import json
    with open(os.path.join(ROOT, "tests", "golden", "fig3_three_qubit.json")) as f:
        yield "fig3", json.load(f)["circuit"]
    for seed in range(40):
        n = 2 + seed % 6
        yield f"cnot{seed}", w.cnot_layers(n, 2 + seed % 4, 4400 + seed).to_text()
    for n in (4, 6):
        yield f"qaoa{n}", w.qaoa_maxcut(n, 2, 11, 12)[0].to_text()
    yield "qft5", w.qft(5).to_text()


@pytest.mark.parametrize("placement", ["optimal", "greedy"])
@pytest.mark.parametrize("name,text", list(_reach_circuits()), ids=[c[0] for c in _reach_circuits()])
def test_reach_reducer_matches_oracle(name, text, placement):
    """FHS_REDUCE_OPTIMAL / GREEDY choose the same sources, at the same
    evaluation positions, as the oracle's placement by reachability; Eq. (8)
    agrees; every candidate split the library offers keeps 0 <= c1 <= c2 <= G
    and the full-range cuts (0 and G, which never separate an affine input
    from its sources) are always among the allowed ones."""
    p = fhs.Program(text, placement=placement)
    o = oracle.Feynman(text, placement)
    assert p.placement == placement
    assert (p.n, p.G, p.A) == (o.n, o.G, o.A)
    assert p.source_eval_positions == o.source_eval_positions
    assert p.A <= fhs.Program(text).A
    splits = p.candidate_splits()
    assert all(0 <= a <= b <= p.G for a, b in splits)
    for c1, c2 in splits[:: max(1, len(splits) // 8)]:
        assert p.partition_cost(c1, c2)[0] == o.eq8(c1, c2)
    assert p.cut_allowed(0) and p.cut_allowed(p.G)
    assert all(p.cut_allowed(a) and p.cut_allowed(b) for a, b in splits)
    c1, c2 = p.choose_partition(fhs.PART_EQ8)   # cuts below L act at L
    assert p.cut_allowed(max(c1, p.L)) and p.cut_allowed(max(c2, p.L))
    if placement == "optimal" and name.startswith("cnot"):
        # Eq. (8) over the allowed cuts is no better than over all of them
        assert p.partition_cost(c1, c2)[0] >= o.eq8_argmin()[2]


def test_reach_flag_errors():
    t = w.cnot_layers(4, 2, 4401).to_text()
    with pytest.raises(ValueError):
        fhs.Program(t, placement="sideways")
    lib = fhs.lib()
    import ctypes
    h = ctypes.c_void_p()
    b = t.encode()
    for flags in (fhs.REDUCE_OPTIMAL | fhs.REDUCE_GREEDY, fhs.REDUCE_OPTIMAL | fhs.REDUCE_FORWARD):
        assert lib.fhs_reduce_ex(b, len(b), flags, ctypes.byref(h)) == 1   # FHS_EINVAL
    # gates outside the analysed set
    t2 = "qubits 3\nH 0\nCCX 0 1 2\nH 2\n"
    with pytest.raises(fhs.FhsError):
        fhs.Program(t2, placement="optimal")
