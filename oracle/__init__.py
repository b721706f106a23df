"""CPU oracle for the reduced-history Feynman method.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the product library never does, and the
two share no code.

Parts:
  * ``statevector`` -- O1, the plain definition: a dense state vector
    (Eq. (1)-(2) of the paper), exact up to rounding, for small circuits;
  * ``closed_forms`` -- textbook closed forms (QFT, amplitude amplification,
    quantum-walk position dynamics) that pin O1 and O2 at any size;
  * ``brute_force`` -- the naive path sum over all intermediate basis states
    (Eq. (3)-(5)) for tiny circuits, with the same threshold rule as O2;
  * ``Feynman`` -- O2, the method itself (Algorithms 1 and 2, backward source
    placement, Eq. (8)) in plain C (``feynman.c``), loaded through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "feynman.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ERRORS = {0: "ok", 1: "parse error", 2: "out of range", 3: "invalid argument",
          4: "internal error"}


def build(force: bool = True) -> str:
    """Compile feynman.c into liboracle.so (gcc, OpenMP, no FP contraction so
    products and moduli round exactly as written)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(P)]
        lib.orc_load_ex.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(P)]
        lib.orc_free.argtypes = [P]
        lib.orc_free.restype = None
        lib.orc_info.argtypes = [P] + [ctypes.POINTER(ctypes.c_int)] * 4
        lib.orc_sources.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
        lib.orc_gate_role.argtypes = [P, ctypes.c_int]
        lib.orc_pair.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P]
        lib.orc_evaluate.argtypes = [P, P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int]
        lib.orc_sample.argtypes = [P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, P, P, ctypes.c_int]
        lib.orc_eq8.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        lib.orc_eq8_argmin.argtypes = [P, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), P]
        _lib = lib
    return _lib


def _words(values: Sequence[int], n: int) -> np.ndarray:
    w = max(1, (n + 63) // 64)
    out = np.zeros((len(values), w), dtype=np.uint64)
    for i, v in enumerate(values):
        for j in range(w):
            out[i, j] = (int(v) >> (64 * j)) & ((1 << 64) - 1)
    return np.ascontiguousarray(out)


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what}: {ERRORS.get(rc, rc)}")


class Feynman:
    """O2: the paper's reduced-history method on the CPU (plain C).

    placement: "backward" (the paper's sweep from the output, Section IV-A)
    or "forward" (the sweep from the input, Table I's other column); the
    sweep direction is also the evaluation order that the cuts of
    Algorithm 2 index.  "optimal" and "greedy" (Section IV-B, Fig. 3):
    sources on the input segments of branching gates, as few as let
    determinism reach every internal wire (exhaustive search, or one
    candidate at a time by the most wires reached); CNOT, SWAP and one-qubit
    gates only; evaluated by Algorithm 1, propagation over the whole
    circuit."""

    ROLE_PRESERVE, ROLE_DET, ROLE_BRANCH = 0, 1, 2

    def __init__(self, circuit_text: str, placement: str = "backward"):
        lib = _load()
        h = ctypes.c_void_p()
        modes = {"backward": 0, "forward": 1, "optimal": 2, "greedy": 3}
        if placement not in modes:
            raise ValueError(f"unknown placement {placement!r}")
        _check(lib.orc_load_ex(circuit_text.encode(), modes[placement], ctypes.byref(h)), "orc_load")
        self._h = h
        n, G, A, ns = (ctypes.c_int() for _ in range(4))
        lib.orc_info(h, ctypes.byref(n), ctypes.byref(G), ctypes.byref(A), ctypes.byref(ns))
        self.n, self.G, self.A, self.n_segments = n.value, G.value, A.value, ns.value

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_free(self._h)
            self._h = None

    @property
    def source_eval_positions(self) -> list:
        arr = (ctypes.c_int * max(1, self.A))()
        _load().orc_sources(self._h, arr)
        return list(arr[: self.A])

    def role(self, t: int) -> int:
        return _load().orc_gate_role(self._h, t)

    def region_sources(self, c1: int, c2: int) -> Tuple[int, int, int]:
        pos = self.source_eval_positions
        ap = sum(1 for e in pos if e < c1)
        ar = sum(1 for e in pos if c1 <= e < c2)
        return ap, ar, self.A - ap - ar

    def pair(self, b_in: int, b_out: int, threshold: float = 0.0,
             partition: Optional[Tuple[int, int]] = None):
        """Transition amplitude alpha^{b_in,b_out}.  partition=None runs
        Algorithm 1, (c1, c2) runs Algorithm 2 with those evaluation cuts.
        Returns (complex amplitude, n_valid, sum_h, xor_h, gate_evals)."""
        bi = _words([b_in], self.n)
        bo = _words([b_out], self.n)
        amp = np.zeros(2, dtype=np.float64)
        st = np.zeros(4, dtype=np.uint64)
        c1, c2 = (-1, -1) if partition is None else partition
        _check(_load().orc_pair(self._h, bi.ctypes.data, bo.ctypes.data, float(threshold),
                                int(c1), int(c2), amp.ctypes.data, st.ctypes.data), "orc_pair")
        return complex(amp[0], amp[1]), int(st[0]), int(st[1]), int(st[2]), int(st[3])

    def evaluate(self, inputs: Sequence[int], coeffs: Sequence[complex], outputs: Sequence[int],
                 threshold: float = 0.0, partition: Optional[Tuple[int, int]] = None,
                 threads: int = 1):
        """Eq. (2) for every requested output.  Returns (amps complex[M],
        stats uint64[M,4] = n_valid, sum_h, xor_h, gate_evals)."""
        bi = _words(inputs, self.n)
        bo = _words(outputs, self.n)
        cf = np.zeros((len(inputs), 2), dtype=np.float64)
        for i, z in enumerate(coeffs):
            z = complex(*z) if isinstance(z, tuple) else complex(z)
            cf[i] = (z.real, z.imag)
        amps = np.zeros((len(outputs), 2), dtype=np.float64)
        st = np.zeros((len(outputs), 4), dtype=np.uint64)
        c1, c2 = (-1, -1) if partition is None else partition
        _check(_load().orc_evaluate(self._h, bi.ctypes.data, cf.ctypes.data, len(inputs),
                                    bo.ctypes.data, len(outputs), float(threshold), int(c1),
                                    int(c2), amps.ctypes.data, st.ctypes.data, int(threads)),
               "orc_evaluate")
        return amps[:, 0] + 1j * amps[:, 1], st

    def sample(self, b_in: int, outputs: Sequence[int], partition: Tuple[int, int],
               hp_range: Tuple[int, int], threshold: float = 0.0, threads: int = 1):
        """Algorithm 2 restricted to prefix assignments h_p in hp_range, for
        timing a bounded share of a workload.  Returns (amps, stats)."""
        bi = _words([b_in], self.n)
        bo = _words(outputs, self.n)
        amps = np.zeros((len(outputs), 2), dtype=np.float64)
        st = np.zeros((len(outputs), 4), dtype=np.uint64)
        _check(_load().orc_sample(self._h, bi.ctypes.data, bo.ctypes.data, len(outputs),
                                  float(threshold), int(partition[0]), int(partition[1]),
                                  int(hp_range[0]), int(hp_range[1]), amps.ctypes.data,
                                  st.ctypes.data, int(threads)), "orc_sample")
        return amps[:, 0] + 1j * amps[:, 1], st

    def eq8(self, c1: int, c2: int) -> int:
        out = np.zeros(2, dtype=np.uint64)
        _check(_load().orc_eq8(self._h, int(c1), int(c2), out.ctypes.data), "orc_eq8")
        return int(out[0]) | (int(out[1]) << 64)

    def eq8_argmin(self) -> Tuple[int, int, int]:
        c1, c2 = ctypes.c_int(), ctypes.c_int()
        out = np.zeros(2, dtype=np.uint64)
        _check(_load().orc_eq8_argmin(self._h, ctypes.byref(c1), ctypes.byref(c2),
                                      out.ctypes.data), "orc_eq8_argmin")
        return c1.value, c2.value, int(out[0]) | (int(out[1]) << 64)


def mix64(h: int) -> int:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014)."""
    m = (1 << 64) - 1
    z = h & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)
