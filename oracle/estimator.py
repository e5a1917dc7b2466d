"""Per-pixel Monte Carlo estimates, hit counts and error vectors.

Sec. 2 defines the test-integrand map I_p = { (1/N) sum_k f_i(s_p^k) } (the
same estimator is drawn in Fig. 1b); the error vector of pixel p is
e_p = I_p - I_ref.  For a Heaviside the estimate is c / N with the integer
hit count c = #{k : f(s_p^k) = 1}.

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import numpy as np

from . import integrands, lattice

Q16 = 1 << 16
HALF = 1 << 15


def shifted_points(n: int, g, u) -> np.ndarray:
    """The N scrambled points of offsets ``u`` ([..., 2]): int64 [..., N, 2]."""
    L = lattice.lattice_q16(n, g)
    u = np.asarray(u, dtype=np.int64)
    return lattice.scramble(L, u[..., None, :])


def hit_counts(n: int, g, u, table: dict, chunk: int = 256) -> np.ndarray:
    """c[p, t] = #{i : n_t . (S_{p,i} - 2**15) > D'_t} for offsets ``u`` [P, 2]."""
    u = np.asarray(u, dtype=np.int64).reshape(-1, 2)
    nx = np.asarray(table["nx"], dtype=np.int64)
    ny = np.asarray(table["ny"], dtype=np.int64)
    d = integrands.heaviside_threshold(nx, ny, table["cx"], table["cy"])
    out = np.empty((u.shape[0], nx.shape[0]), dtype=np.int64)
    for lo in range(0, u.shape[0], chunk):
        s = shifted_points(n, g, u[lo:lo + chunk]) - HALF           # [p, N, 2]
        dots = s[..., 0, None] * nx + s[..., 1, None] * ny         # [p, N, T]
        out[lo:lo + chunk] = (dots > d).sum(axis=1)
    return out


def gauss_estimates(n: int, g, u, table: dict, chunk: int = 64) -> np.ndarray:
    """(1/N) sum_i f_t(S_{p,i} / 2**16) for Gaussian integrands, FP64 [P, T]."""
    u = np.asarray(u, dtype=np.int64).reshape(-1, 2)
    mx, my, s = (np.asarray(table[k], dtype=np.float64) for k in ("mx", "my", "s"))
    out = np.empty((u.shape[0], mx.shape[0]), dtype=np.float64)
    for lo in range(0, u.shape[0], chunk):
        x = shifted_points(n, g, u[lo:lo + chunk]).astype(np.float64) / Q16   # [p, N, 2]
        dx = x[..., 0, None] - mx
        dy = x[..., 1, None] - my
        out[lo:lo + chunk] = np.exp(-(dx * dx + dy * dy) / (2.0 * s * s)).mean(axis=1)
    return out


def errors_from_counts(counts: np.ndarray, n: int, areas: np.ndarray) -> np.ndarray:
    """e = c / N - A_t in FP64."""
    return np.asarray(counts, dtype=np.float64) / n - np.asarray(areas, dtype=np.float64)
