"""Naive sum over histories (Eq. (3)-(5) of the paper) for tiny circuits.

TEST INFRASTRUCTURE ONLY.  A history is a sequence of full basis states
(i_in, i_1, ..., i_out); its contribution is the product of the gate
transition amplitudes along it.  Histories are walked in pure Python over
every intermediate basis state with a nonzero factor, so this is only for
circuits of a few qubits and gates.  It knows nothing of wire segments,
sources or propagation, which is what lets it pin the C oracle's counts.

Threshold rule (the same reading as the C oracle): a history is kept iff the
product, in evaluation order, of min(1, |factor|) over the gates that branch
(a matrix column with more than one nonzero) is >= t.  The evaluation order
runs from the output to the input (the backward sweep), or from the input to
the output when the sources are placed by the forward sweep.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from . import statevector as sv


def _gate_unitaries(text: str):
    n, gates = sv.parse(text)
    us = []
    branch = []
    for g in gates:
        cols = []
        for b in range(1 << n):
            psi = np.zeros(1 << n, dtype=complex)
            psi[b] = 1
            cols.append(sv.apply_gate(psi, n, g))
        u = np.stack(cols, axis=1)
        us.append(u)
        branch.append(bool(np.any(np.count_nonzero(u, axis=0) > 1)))
    return n, us, branch


def path_sum(text: str, b_in: int, b_out: int, threshold: float = 0.0, forward: bool = False
             ) -> Tuple[complex, int]:
    """(amplitude, number of kept histories) for one input/output pair;
    forward: evaluation order from the input."""
    n, us, branch = _gate_unitaries(text)
    m = len(us)
    total = 0j
    kept = 0
    path: List[int] = [b_in]

    def rec(t: int):
        nonlocal total, kept
        if t == m:
            if path[-1] != b_out:
                return
            amp = 1 + 0j
            M = 1.0
            for s in (range(m) if forward else range(m - 1, -1, -1)):   # evaluation order
                f = us[s][path[s + 1], path[s]]
                amp = amp * f
                if branch[s]:
                    mod = math.sqrt(f.real * f.real + f.imag * f.imag)
                    M = M * min(1.0, mod)
            if M >= threshold:
                total += amp
                kept += 1
            return
        col = us[t][:, path[-1]]
        for nxt in np.nonzero(col)[0]:
            path.append(int(nxt))
            rec(t + 1)
            path.pop()

    rec(0)
    return total, kept
