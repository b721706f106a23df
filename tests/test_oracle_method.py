"""Method-level invariants of the C oracle (Algorithms 1 and 2, Eq. (8)).

  * Algorithm 2 returns Algorithm 1's amplitude and the identical valid set
    (count, sum and xor-hash of the history indices) for every cut pair;
  * with nothing pruned, the instrumented gate-evaluation count of
    Algorithm 2 equals Eq. (8) exactly, and Algorithm 1's equals 2^A G;
  * Eq. (8)'s argmin matches a brute-force scan in Python integers;
  * the valid set shrinks as the threshold grows, and t = 0 keeps every
    history the exact method keeps.
"""
import numpy as np
import pytest

import oracle
import workloads as w


def _all_splits(G):
    for c1 in range(G + 1):
        for c2 in range(c1, G + 1):
            yield c1, c2


@pytest.mark.parametrize("seed", range(40))
def test_alg2_equals_alg1_every_split(seed):
    n = 2 + seed % 4
    c = w.random_mixed(n, 5 + seed % 7, 500 + seed)
    F = oracle.Feynman(c.to_text())
    rng = np.random.default_rng(seed)
    b_in = int(rng.integers(0, 1 << n))
    thr = [0.0, 0.0, 0.1, 0.4][seed % 4]
    for b_out in range(1 << n):
        ref = F.pair(b_in, b_out, threshold=thr)
        for c1, c2 in _all_splits(F.G):
            got = F.pair(b_in, b_out, threshold=thr, partition=(c1, c2))
            assert abs(got[0] - ref[0]) <= 1e-12
            assert got[1:4] == ref[1:4], (c1, c2)


@pytest.mark.parametrize("seed", range(16))
def test_alg2_equals_alg1_every_split_forward(seed):
    """The same invariant under forward placement: cuts index time order."""
    n = 2 + seed % 4
    c = w.random_mixed(n, 5 + seed % 7, 800 + seed)
    F = oracle.Feynman(c.to_text(), "forward")
    rng = np.random.default_rng(seed)
    b_in = int(rng.integers(0, 1 << n))
    thr = [0.0, 0.1][seed % 2]
    for b_out in range(1 << n):
        ref = F.pair(b_in, b_out, threshold=thr)
        for c1, c2 in _all_splits(F.G):
            got = F.pair(b_in, b_out, threshold=thr, partition=(c1, c2))
            assert abs(got[0] - ref[0]) <= 1e-12
            assert got[1:4] == ref[1:4], (c1, c2)


def test_eq8_equals_gate_evaluations_qaoa():
    # QAOA has no exact-pruning failures: every history is valid at t = 0
    c, *_ = w.qaoa_maxcut(4, 1, 3, 4)
    F = oracle.Feynman(c.to_text())
    assert F.A == 4
    for c1, c2 in _all_splits(F.G):
        _, nv, _, _, evals = F.pair(0, 0b1010, partition=(c1, c2))
        assert nv == 1 << F.A
        assert evals == F.eq8(c1, c2), (c1, c2)
    _, _, _, _, evals = F.pair(0, 0b1010)
    assert evals == (1 << F.A) * F.G


def test_eq8_equals_gate_evaluations_aa():
    c, _ = w.amplitude_amplification(3, 1, 2, seed=9)
    F = oracle.Feynman(c.to_text())
    for c1, c2 in [(0, 0), (F.G // 3, 2 * F.G // 3), F.eq8_argmin()[:2], (F.G, F.G), (5, 17)]:
        _, nv, _, _, evals = F.pair(0, 0b101, partition=(c1, c2))
        assert nv == 1 << F.A
        assert evals == F.eq8(c1, c2)


def test_eq8_equals_gate_evaluations_forward():
    """Under forward placement QAOA's sources are the Hadamard layer and
    every RX layer but the last; with nothing pruned the instrumented count
    is again Eq. (8) at every cut pair (cuts in time order)."""
    c, *_ = w.qaoa_maxcut(4, 2, 3, 4)
    F = oracle.Feynman(c.to_text(), "forward")
    assert F.A == 8
    for c1, c2 in list(_all_splits(F.G))[::7]:
        _, nv, _, _, evals = F.pair(0, 0b0110, partition=(c1, c2))
        assert nv == 1 << F.A
        assert evals == F.eq8(c1, c2), (c1, c2)


def _eq8_py(G, pos, c1, c2):
    ap = sum(1 for e in pos if e < c1)
    ar = sum(1 for e in pos if c1 <= e < c2)
    as_ = len(pos) - ap - ar
    return 2 ** ap * (c1 + 2 ** ar * ((c2 - c1) + 2 ** as_ * (G - c2)))


@pytest.mark.parametrize("which", ["walk", "aa", "qaoa", "mixed"])
def test_eq8_argmin_brute_force(which):
    if which == "walk":
        t = w.quantum_walk(7, 6).to_text()
    elif which == "aa":
        t = w.amplitude_amplification(4, 2, 4, seed=1)[0].to_text()
    elif which == "qaoa":
        t = w.qaoa_maxcut(6, 2, 5, 6)[0].to_text()
    else:
        t = w.random_mixed(5, 40, 77).to_text()
    F = oracle.Feynman(t)
    pos = F.source_eval_positions
    best = None
    for c1, c2 in _all_splits(F.G):
        v = _eq8_py(F.G, pos, c1, c2)
        assert F.eq8(c1, c2) == v
        if best is None or v < best[0]:
            best = (v, c1, c2)
    c1, c2, cost = F.eq8_argmin()
    assert (cost, c1, c2) == best


def test_eq8_literal_aa_is_128bit():
    # 16 search qubits, 3 iterations: A = 96, the plain cost exceeds 2^64
    c, _ = w.amplitude_amplification(16, 3, 4, seed=301)
    F = oracle.Feynman(c.to_text())
    assert F.A == 96
    assert F.eq8(0, 0) == (2 ** 96) * F.G
    c1, c2, cost = F.eq8_argmin()
    assert cost == _eq8_py(F.G, F.source_eval_positions, c1, c2)
    assert cost < F.eq8(0, 0)
    with pytest.raises(oracle.OracleError):
        F.pair(0, 0)


@pytest.mark.parametrize("seed", range(12))
def test_threshold_monotone(seed):
    c, *_ = w.qaoa_maxcut(6, 1, 40 + seed, 50 + seed)
    F = oracle.Feynman(c.to_text())
    prev = None
    for thr in (0.0, 1e-4, 1e-3, 3e-3, 1e-2, 3e-2, 1.0):
        _, nv, *_ = F.pair(0, seed % 64, threshold=thr, partition=(3, 9))
        if prev is not None:
            assert nv <= prev
        prev = nv
    _, nv0, *_ = F.pair(0, seed % 64, threshold=0.0)
    assert nv0 == 1 << F.A
