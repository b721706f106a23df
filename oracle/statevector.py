"""O1: dense state-vector definition of the amplitudes (test infrastructure).

The paper defines what the method computes as the transition amplitude
<i_out| U^(m) ... U^(1) |i_in> (Eq. (1)) and, for a sparse input state, the
weighted sum of transition amplitudes over the input support (Eq. (2)).  At
threshold t = 0 the reduced-history sum reaches these values exactly (up to
rounding), so this module is the plain definition: apply every gate matrix to
a full 2^n vector in fp64 and read the requested entries.

It parses the circuit text itself and builds its own gate matrices; nothing is
shared with the C oracle or with the GPU library.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

MAX_QUBITS = 24


def parse(text: str):
    """Circuit text -> (n, [(name, qubits, negs, angle)])."""
    n = None
    gates = []
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        toks = line.split()
        if toks[0] == "qubits":
            n = int(toks[1])
            continue
        name = toks[0]
        qs, negs, angle = [], [], None
        for t in toks[1:]:
            neg = t.startswith("~")
            body = t[1:] if neg else t
            if body.isdigit():
                qs.append(int(body))
                negs.append(neg)
            else:
                angle = float.fromhex(body) if "x" in body.lower() else float(body)
        gates.append((name, tuple(qs), tuple(negs), angle))
    if n is None:
        raise ValueError("missing 'qubits' line")
    return n, gates


def gate_matrix(name: str, angle) -> np.ndarray:
    """Matrix U[out, in] of a fixed gate on its listed qubits; local index bit
    j belongs to the j-th listed qubit."""
    h = math.sqrt(0.5)
    if name == "H":
        return np.array([[h, h], [h, -h]], dtype=complex)
    if name == "X":
        return np.array([[0, 1], [1, 0]], dtype=complex)
    if name == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=complex)
    if name == "Z":
        return np.diag([1, -1]).astype(complex)
    if name == "S":
        return np.diag([1, 1j])
    if name == "SDG":
        return np.diag([1, -1j])
    if name == "T":
        return np.diag([1, complex(h, h)])
    if name == "TDG":
        return np.diag([1, complex(h, -h)])
    if name == "P":
        return np.diag([1, complex(math.cos(angle), math.sin(angle))])
    if name in ("RX", "RY", "RZ", "RZZ"):
        c, s = math.cos(0.5 * angle), math.sin(0.5 * angle)
    if name == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=complex)
    if name == "RY":
        return np.array([[c, -s], [s, c]], dtype=complex)
    if name == "RZ":
        return np.diag([complex(c, -s), complex(c, s)])
    if name in ("CX", "SWAP", "CCX", "CSWAP"):
        k = 2 if name in ("CX", "SWAP") else 3
        u = np.zeros((1 << k, 1 << k), dtype=complex)
        for x in range(1 << k):
            b = [(x >> j) & 1 for j in range(k)]
            if name == "CX" and b[0]:
                b[1] ^= 1
            elif name == "SWAP":
                b[0], b[1] = b[1], b[0]
            elif name == "CCX" and b[0] and b[1]:
                b[2] ^= 1
            elif name == "CSWAP" and b[0]:
                b[1], b[2] = b[2], b[1]
            y = sum(v << j for j, v in enumerate(b))
            u[y, x] = 1
        return u
    if name == "CZ":
        return np.diag([1, 1, 1, -1]).astype(complex)
    if name == "CP":
        return np.diag([1, 1, 1, complex(math.cos(angle), math.sin(angle))])
    if name == "RZZ":
        # e^{-i angle/2} when the two bits agree, e^{+i angle/2} otherwise
        return np.diag([complex(c, -s), complex(c, s), complex(c, s), complex(c, -s)])
    raise ValueError(f"no dense matrix for gate {name}")


def _apply_dense(psi: np.ndarray, n: int, u: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    k = len(qubits)
    t = psi.reshape([2] * n)            # axis a <-> qubit n-1-a
    ut = u.reshape([2] * (2 * k))       # (out_{k-1}..out_0, in_{k-1}..in_0)
    in_axes = list(range(k, 2 * k))     # in_{k-1} .. in_0
    psi_axes = [n - 1 - qubits[k - 1 - i] for i in range(k)]
    r = np.tensordot(ut, t, axes=(in_axes, psi_axes))
    r = np.moveaxis(r, list(range(k)), psi_axes)
    return r.reshape(-1)


def _match_mask(n: int, qubits: Sequence[int], negs: Sequence[bool]) -> np.ndarray:
    idx = np.arange(1 << n, dtype=np.int64)
    ok = np.ones(1 << n, dtype=bool)
    for q, ng in zip(qubits, negs):
        bit = (idx >> q) & 1
        ok &= bit == (0 if ng else 1)
    return ok


def apply_gate(psi: np.ndarray, n: int, gate) -> np.ndarray:
    name, qs, negs, angle = gate
    negs = negs or (False,) * len(qs)
    if name == "MCX":
        t = qs[0]
        ok = _match_mask(n, qs[1:], negs[1:])
        idx = np.arange(1 << n, dtype=np.int64)
        src = np.where(ok, idx ^ (1 << t), idx)
        return psi[src]
    if name == "MCZ":
        ok = _match_mask(n, qs, negs)
        out = psi.copy()
        out[ok] = -out[ok]
        return out
    return _apply_dense(psi, n, gate_matrix(name, angle), qs)


def evolve(text: str, b_in: int) -> np.ndarray:
    """C|b_in> as a dense vector (n <= MAX_QUBITS)."""
    n, gates = parse(text)
    if n > MAX_QUBITS:
        raise ValueError(f"state vector limited to {MAX_QUBITS} qubits")
    psi = np.zeros(1 << n, dtype=complex)
    psi[b_in] = 1.0
    for g in gates:
        psi = apply_gate(psi, n, g)
    return psi


def evolve_state(text: str, psi: np.ndarray) -> np.ndarray:
    """C|psi> for a dense input vector (Eq. (2) for every output at once)."""
    n, gates = parse(text)
    if n > MAX_QUBITS or psi.shape != (1 << n,):
        raise ValueError("state vector size")
    psi = np.asarray(psi, dtype=complex)
    for g in gates:
        psi = apply_gate(psi, n, g)
    return psi


def amplitudes(text: str, inputs: Sequence[int], coeffs: Sequence[complex],
               outputs: Sequence[int]) -> np.ndarray:
    """Eq. (2): <b_out|C|psi> for psi = sum_i coeff_i |b_in_i>."""
    n, _ = parse(text)
    acc = np.zeros(len(outputs), dtype=complex)
    outs = np.asarray(outputs, dtype=np.int64)
    for b, cf in zip(inputs, coeffs):
        cf = complex(*cf) if isinstance(cf, tuple) else complex(cf)
        psi = evolve(text, b)
        acc += cf * psi[outs]
    return acc


def unitary(text: str) -> np.ndarray:
    """Full 2^n x 2^n unitary, column b = C|b> (tiny circuits only)."""
    n, _ = parse(text)
    cols = [evolve(text, b) for b in range(1 << n)]
    return np.stack(cols, axis=1)
