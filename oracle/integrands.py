"""Test integrands and their exact integrals over the unit square.

Sec. 2 (the test-integrand map next to Eq. (1)) uses randomly oriented
Heaviside functions; Sec. 3.5 adds low-frequency integrands, here isotropic
Gaussians.  The optimiser only needs Monte Carlo estimates; the exact integrals
give the reference I_ref that the error vectors and the blur criterion of
Sec. 3.3 (Fig. 1c) are measured against.

Heaviside t (normal n_t: int16 pair, edge point C_t: Q0.16 pair):
    f_t(x) = 1  iff  n_t . (x - C_t / 2**16) > 0      (edge excluded)
In Q0.16 integer coordinates with centred values S' = S - 2**15 this is
    n_t . S' > D'_t,   D'_t = n_t . (C_t - 2**15),
which is exact in integers.  The integral is the area of the unit square
clipped by the half-plane, computed by clipping the square polygon against
the line (Sutherland-Hodgman, one plane) and the shoelace formula in FP64.

Gaussian t (centre mu, std s):
    f_t(x) = exp(-|x - mu|^2 / (2 s^2)),
    I_t = prod_a s sqrt(pi/2) [erf((1 - mu_a)/(s sqrt 2)) + erf(mu_a/(s sqrt 2))].

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox

Q16 = 1 << 16
HALF = 1 << 15


def heaviside_threshold(nx, ny, cx, cy) -> np.ndarray:
    """D'_t = n_t . (C_t - 2**15) as int64."""
    nx = np.asarray(nx, dtype=np.int64)
    ny = np.asarray(ny, dtype=np.int64)
    return nx * (np.asarray(cx, dtype=np.int64) - HALF) + ny * (np.asarray(cy, dtype=np.int64) - HALF)


def _clip_area(a: float, b: float, k: float) -> float:
    """Area of {x in [0,1]^2 : a x + b y >= k}."""
    square = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    poly = []
    for idx in range(4):
        p = square[idx]
        q = square[(idx + 1) % 4]
        fp = a * p[0] + b * p[1] - k
        fq = a * q[0] + b * q[1] - k
        if fp >= 0.0:
            poly.append(p)
        if (fp >= 0.0) != (fq >= 0.0):
            lam = fp / (fp - fq)
            poly.append((p[0] + lam * (q[0] - p[0]), p[1] + lam * (q[1] - p[1])))
    if len(poly) < 3:
        return 0.0
    twice = 0.0
    for idx in range(len(poly)):
        x0, y0 = poly[idx]
        x1, y1 = poly[(idx + 1) % len(poly)]
        twice += x0 * y1 - x1 * y0
    return abs(twice) * 0.5


def heaviside_area(nx: int, ny: int, cx: int, cy: int) -> float:
    """Exact integral of one Heaviside over the unit square (FP64).

    The half-plane is n . x > n . C / 2**16; the line itself has zero area,
    so clipping against n . x >= k gives the same value."""
    nx, ny, cx, cy = int(nx), int(ny), int(cx), int(cy)
    if nx == 0 and ny == 0:
        raise ValueError("degenerate Heaviside normal")
    k = (nx * cx + ny * cy) / Q16          # integer / 2**16: exact in FP64
    return _clip_area(float(nx), float(ny), k)


def heaviside_areas(table: dict) -> np.ndarray:
    return np.array([heaviside_area(a, b, c, d) for a, b, c, d in
                     zip(table["nx"], table["ny"], table["cx"], table["cy"])], dtype=np.float64)


def gaussian_integral(mx: float, my: float, s: float) -> float:
    """Integral of exp(-|x - mu|^2 / (2 s^2)) over [0,1]^2 via erf (separable)."""
    out = 1.0
    for mu in (mx, my):
        out *= s * math.sqrt(math.pi / 2.0) * (math.erf((1.0 - mu) / (s * math.sqrt(2.0)))
                                               + math.erf(mu / (s * math.sqrt(2.0))))
    return out


def gaussian_integrals(table: dict) -> np.ndarray:
    return np.array([gaussian_integral(a, b, c) for a, b, c in
                     zip(table["mx"], table["my"], table["s"])], dtype=np.float64)


def heaviside_table_philox(t: int, seed: int, problem: int = 0) -> dict:
    """Heavisides drawn from the counter stream S_INTEG at counters (t, 0,
    problem, S_INTEG): angle 2 pi w0 2**-32, normal rint(2**14 (cos, sin)),
    edge point (w1 >> 16, w2 >> 16)."""
    w = philox.draw(np.arange(t), 0, problem, philox.S_INTEG, seed)
    theta = 2.0 * math.pi * w[:, 0].astype(np.float64) * 2.0 ** -32
    nx = np.array([round(16384.0 * math.cos(a)) for a in theta], dtype=np.int16)
    ny = np.array([round(16384.0 * math.sin(a)) for a in theta], dtype=np.int16)
    return {"nx": nx, "ny": ny,
            "cx": (w[:, 1] >> np.uint32(16)).astype(np.uint16),
            "cy": (w[:, 2] >> np.uint32(16)).astype(np.uint16)}


def gaussian_table_philox(t: int, seed: int, problem: int = 0) -> dict:
    """Gaussians drawn from counters (t, 1, problem, S_INTEG): centre
    (w0, w1) 2**-32, standard deviation 0.05 + 0.25 w2 2**-32."""
    w = philox.draw(np.arange(t), 1, problem, philox.S_INTEG, seed).astype(np.float64)
    return {"mx": w[:, 0] * 2.0 ** -32, "my": w[:, 1] * 2.0 ** -32, "s": 0.05 + 0.25 * (w[:, 2] * 2.0 ** -32)}
