"""The screen-space sampler a renderer consumes (Sec. 2 and Sec. 3.1-3.2).

A screen-space sampler is the main sequence plus a tile of scrambling
offsets (Sec. 2); with dimension padding (Sec. 3.1) every pair of dimensions
(2d, 2d + 1) has its own 2-D main sequence and tile, and a 1-D effect takes
one dimension of a pair and discards the other.  With the rank-1 lattice of
Sec. 3.2 and the toroidal scrambling, sample k of screen pixel (x, y) in pair
d is
    s^k = mod(Phi(k) g_d / N_d + u_d[y mod H_d, x mod W_d], 1),
k taken modulo N_d, in Q0.16 (value v stands for v / 2**16).

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def sample_q16(pairs, x, y, k) -> np.ndarray:
    """pairs: list of dicts with n, g, width, height and offsets u (uint16
    [H, W, 2]); x, y, k: integer arrays of queries.  Returns int64
    [m, 2 * len(pairs)] Q0.16 values, dimension 2d + a = component a of
    pair d."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    k = np.asarray(k, dtype=np.int64)
    out = np.zeros((x.shape[0], 2 * len(pairs)), dtype=np.int64)
    for d, pr in enumerate(pairs):
        seq = lattice.sequence_q16(pr["n"], pr["g"])
        u = np.asarray(pr["u"], dtype=np.int64).reshape(pr["height"], pr["width"], 2)
        for j in range(x.shape[0]):
            s = lattice.scramble(seq[k[j] % pr["n"]], u[y[j] % pr["height"], x[j] % pr["width"]])
            out[j, 2 * d:2 * d + 2] = s
    return out
