"""Rank-1 lattice main sequence and its toroidal per-pixel scrambling.

Sec. 3.2 defines the main sequence s^k = mod(Phi(k) d, 1) with Phi the van der
Corput radical inverse and d the direction (generator) vector, and the
per-pixel scrambling K(s^k, u_p) = mod(s^k + u_p, 1); Fig. 1a draws two
pixels' shifted point sets.  For N = 2**m points Phi(k) = bitrev_m(k) / N, so
Phi(k) d mod 1 = ((bitrev_m(k) * g) mod N) / N for an integer generator g.

All coordinates are Q0.16 fixed point (value v stands for v / 2**16), so the
modulo-one wrap is exact integer arithmetic (reading documented with the
oracle: offsets have resolution 2**-16 and N must divide 2**16).

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import numpy as np

Q16 = 1 << 16


def log2_exact(n: int) -> int:
    m = int(n).bit_length() - 1
    if n < 1 or (1 << m) != n:
        raise ValueError(f"N={n} is not a power of two")
    return m


def bitrev(k: int, m: int) -> int:
    """Reverse the low ``m`` bits of ``k`` (van der Corput index, base 2)."""
    out = 0
    for _ in range(m):
        out = (out << 1) | (k & 1)
        k >>= 1
    return out


def lattice_index(n: int, g) -> np.ndarray:
    """Integer lattice indices j_a(i) = (i * g_a) mod N for i = 0..N-1; int64 [N, 2]."""
    i = np.arange(n, dtype=np.int64)
    return np.stack([(i * int(g[0])) % n, (i * int(g[1])) % n], axis=1)


def lattice_q16(n: int, g) -> np.ndarray:
    """Lattice points in Q0.16: L_a(i) = j_a(i) * 2**16 / N; int64 [N, 2]."""
    m = log2_exact(n)
    if m > 16:
        raise ValueError("N must divide 2**16")
    return lattice_index(n, g) * (Q16 // n)


def sequence_q16(n: int, g) -> np.ndarray:
    """Main sequence s^k in van der Corput order: s^k = L(bitrev_m(k)); int64 [N, 2]."""
    m = log2_exact(n)
    L = lattice_q16(n, g)
    return np.stack([L[bitrev(k, m)] for k in range(n)], axis=0)


def scramble(points: np.ndarray, u) -> np.ndarray:
    """Toroidal shift mod(s + u, 1) in Q0.16: (s + u) mod 2**16."""
    return (np.asarray(points, dtype=np.int64) + np.asarray(u, dtype=np.int64)) % Q16


def to_unit(points_q16: np.ndarray) -> np.ndarray:
    return np.asarray(points_q16, dtype=np.float64) / Q16
