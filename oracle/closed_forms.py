"""Textbook closed forms that pin the oracle at any size (test infrastructure).

  * QFT: <y|QFT_n|x> = 2^{-n/2} exp(2 pi i (x y mod 2^n) / 2^n), and for a
    dense input the discrete Fourier transform of its amplitudes (FFT);
  * amplitude amplification with the diffusion written as H X MCZ X H (which
    is I - 2|s><s|, the negative of the usual Grover reflection): after s
    iterations each of the m marked states holds (-1)^s sin((2s+1)theta)/sqrt(m)
    and each unmarked state (-1)^s cos((2s+1)theta)/sqrt(N-m), sin theta =
    sqrt(m/N); ancillas end in |0>;
  * coined Hadamard walk on a line (no wrap for few steps on a huge cycle):
    the position-space recursion, and the number of coin sequences that end at
    (x, c), which is the number of valid reduced histories when the coin
    values after the second..last coin flips are the artificial sources.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple


def qft_amplitude(n: int, x: int, y: int) -> complex:
    r = (x * y) % (1 << n)
    ang = 2.0 * math.pi * r / float(1 << n)
    s = 2.0 ** (-0.5 * n)
    return complex(s * math.cos(ang), s * math.sin(ang))


def aa_amplitude(k: int, iterations: int, marked: Sequence[int], y: int) -> complex:
    N = 1 << k
    m = len(marked)
    if y >> k:                      # an ancilla bit is set
        return 0j
    theta = math.asin(math.sqrt(m / N))
    sign = -1.0 if iterations % 2 else 1.0
    a = (2 * iterations + 1) * theta
    if y in set(marked):
        return complex(sign * math.sin(a) / math.sqrt(m), 0.0)
    return complex(sign * math.cos(a) / math.sqrt(N - m), 0.0)


def aa_success_probability(k: int, iterations: int, m: int) -> float:
    theta = math.asin(math.sqrt(m / (1 << k)))
    return math.sin((2 * iterations + 1) * theta) ** 2


def walk_amplitudes(steps: int, coin: Tuple[complex, complex] = (1.0, 0.0)
                    ) -> Dict[Tuple[int, int], complex]:
    """Hadamard walk from position 0 with coin state coin[0]|0> + coin[1]|1>
    (default |0>; the paper's large walk starts from (|0> + i|1>)/sqrt2):
    each step maps the coin (a0, a1) -> ((a0 + a1)/sqrt2, (a0 - a1)/sqrt2),
    then moves coin-1 amplitude to x+1 and coin-0 amplitude to x-1."""
    h = 1.0 / math.sqrt(2.0)
    amp = {(0, c): complex(coin[c]) for c in (0, 1) if coin[c] != 0}
    for _ in range(steps):
        nxt: Dict[Tuple[int, int], complex] = {}
        for (x, c), a in amp.items():
            # contribution of coin c to new coins 0 and 1
            for c2 in (0, 1):
                f = -h if (c == 1 and c2 == 1) else h
                x2 = x + (1 if c2 == 1 else -1)
                nxt[(x2, c2)] = nxt.get((x2, c2), 0j) + f * a
        amp = nxt
    return amp


def _splitmix64_np(h):
    import numpy as np
    z = h.astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def walk_valid_stats(steps: int, x: int, c: int) -> Tuple[int, int, int]:
    """(count, sum of h mod 2^64, xor of SplitMix64(h)) over the valid
    reduced histories of output (x, c).  Source k sits before the coin flip
    of step steps-k and carries the coin value after step steps-1-k, so a
    history is valid iff the coin values it assigns contain exactly
    (x+steps)/2 - c ones: the set is {h < 2^(steps-1) : popcount(h) = ones}."""
    import numpy as np
    if (x + steps) % 2:
        return 0, 0, 0
    ones = (x + steps) // 2 - c
    h = np.arange(1 << (steps - 1), dtype=np.uint64)
    pc = np.zeros(h.shape, dtype=np.int64)
    for b in range(steps - 1):
        pc += ((h >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    sel = h[pc == ones]
    if sel.size == 0:
        return 0, 0, 0
    return (int(sel.size), int(sel.sum(dtype=np.uint64)),
            int(np.bitwise_xor.reduce(_splitmix64_np(sel))))


def walk_n_valid(steps: int, x: int, c: int) -> int:
    """Coin sequences c_1..c_steps with c_steps = c and sum(2c_t - 1) = x."""
    if (x + steps) % 2:
        return 0
    ones = (x + steps) // 2 - c
    if ones < 0 or ones > steps - 1:
        return 0
    return math.comb(steps - 1, ones)


def qft_dense(n: int, psi):
    """<y|QFT_n|psi> for every y and a dense input psi (2^n entries):
    2^{-n/2} sum_x psi_x e^{2 pi i x y / 2^n}, which is 2^{n/2} times numpy's
    inverse FFT of psi."""
    import numpy as np
    psi = np.asarray(psi, dtype=complex)
    return np.fft.ifft(psi) * math.sqrt(float(1 << n))
