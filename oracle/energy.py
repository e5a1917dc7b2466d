"""Screen-space energy of Eq. (1) on a toroidal tile and its single-pixel change.

Eq. (1):  L = sum_p sum_{q != p} exp(-|p - q|^2 / 2.1^2) |I_p - I_q|^2.
Readings used here (each listed with the oracle's documentation):
  * the Gaussian weight is taken literally, w_o = exp(-|o|^2 / sigma^2) with
    sigma = 2.1 (no factor 2 in the denominator);
  * the sum over q runs over the window offsets o in [-r, r]^2 \\ {0}, with
    q = p + o wrapped on the torus; both orderings of each pair are counted;
  * I_p may be replaced by the error vector e_p = I_p - I_ref, since only
    differences enter.

Changing the vector of one pixel p from e to e' changes the energy by
    dE = 2 sum_o w_o sum_t [(e'_t - e_{q,t})^2 - (e_t - e_{q,t})^2]
(each pair appears once with p first and once with p second; the window is
symmetric).  For Heaviside rows, e = c/N - A with integer hit counts c, and
    dE = (2/N^2) sum_o w_o X_o,   X_o = sum_t (c'_t - c_t)(c'_t + c_t - 2 c_{q,t}),
with X_o integers.  Grouping offsets by d = |o|^2 gives integer class sums
X_d; the oracle then adds w(d) X_d in FP64 in increasing d starting from 0.0,
and a move is accepted iff that sum is negative.

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import math

import numpy as np


def window_offsets(r: int) -> list:
    """Offsets (ox, oy) of the (2r+1)^2 - 1 window, row-major."""
    return [(ox, oy) for oy in range(-r, r + 1) for ox in range(-r, r + 1) if (ox, oy) != (0, 0)]


def weight(d: int, sigma: float) -> float:
    """w = exp(-d / sigma^2) for squared pixel distance d (Eq. (1), literal)."""
    return math.exp(-d / (sigma * sigma))


def distance_classes(r: int) -> list:
    """Sorted distinct squared distances of the window offsets."""
    return sorted({ox * ox + oy * oy for ox, oy in window_offsets(r)})


def class_weights(r: int, sigma: float) -> np.ndarray:
    return np.array([weight(d, sigma) for d in distance_classes(r)], dtype=np.float64)


def weight_sum(r: int, sigma: float) -> float:
    """W = sum_o w_o over the window (direct sum)."""
    return sum(weight(ox * ox + oy * oy, sigma) for ox, oy in window_offsets(r))


def _neighbour(field: np.ndarray, ox: int, oy: int) -> np.ndarray:
    """field[(y + oy) mod H, (x + ox) mod W] at every (y, x)."""
    return np.roll(field, shift=(-oy, -ox), axis=(0, 1))


def energy_plain(e: np.ndarray, r: int, sigma: float) -> float:
    """E of an error field e [H, W, T] (FP64)."""
    e = np.asarray(e, dtype=np.float64)
    total = 0.0
    for ox, oy in window_offsets(r):
        diff = e - _neighbour(e, ox, oy)
        total += weight(ox * ox + oy * oy, sigma) * float(np.sum(diff * diff))
    return total


def energy_loops(e: np.ndarray, r: int, sigma: float) -> float:
    """E by explicit loops over pixels and offsets (small tiles only)."""
    h, w, _ = e.shape
    total = 0.0
    for y in range(h):
        for x in range(w):
            for ox, oy in window_offsets(r):
                q = e[(y + oy) % h, (x + ox) % w]
                total += weight(ox * ox + oy * oy, sigma) * float(np.sum((e[y, x] - q) ** 2))
    return total


def delta_plain(e: np.ndarray, y: int, x: int, e_new: np.ndarray, r: int, sigma: float) -> float:
    """dE of replacing e[y, x] by e_new (FP64)."""
    h, w, _ = e.shape
    e_old = np.asarray(e[y, x], dtype=np.float64)
    e_new = np.asarray(e_new, dtype=np.float64)
    total = 0.0
    for ox, oy in window_offsets(r):
        q = np.asarray(e[(y + oy) % h, (x + ox) % w], dtype=np.float64)
        total += weight(ox * ox + oy * oy, sigma) * float(np.sum((e_new - q) ** 2 - (e_old - q) ** 2))
    return 2.0 * total


def delta_class_sums(c: np.ndarray, ys, xs, c_new: np.ndarray, r: int) -> np.ndarray:
    """Integer X_d for moves of pixels (ys[j], xs[j]) to counts c_new[j].

    c: int64 [H, W, T]; c_new: int64 [M, T].  Returns int64 [M, n_classes]."""
    h, w, _ = c.shape
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    c_old = c[ys, xs].astype(np.int64)
    c_new = np.asarray(c_new, dtype=np.int64)
    dc = c_new - c_old
    s = c_new + c_old
    classes = distance_classes(r)
    out = np.zeros((ys.shape[0], len(classes)), dtype=np.int64)
    for ox, oy in window_offsets(r):
        cq = c[(ys + oy) % h, (xs + ox) % w].astype(np.int64)
        out[:, classes.index(ox * ox + oy * oy)] += np.sum(dc * (s - 2 * cq), axis=1)
    return out


def weighted_class_sum(xd: np.ndarray, r: int, sigma: float) -> np.ndarray:
    """sum_d w(d) X_d in FP64, added in increasing d from 0.0 (elementwise over rows)."""
    wd = class_weights(r, sigma)
    xd = np.asarray(xd)
    acc = np.zeros(xd.shape[:-1], dtype=np.float64)
    for j in range(wd.shape[0]):
        acc = acc + wd[j] * xd[..., j].astype(np.float64)
    return acc


def delta_exact(c: np.ndarray, ys, xs, c_new: np.ndarray, n: int, r: int, sigma: float) -> np.ndarray:
    """dE from integer hit counts: (2 / N^2) sum_d w(d) X_d (FP64)."""
    return weighted_class_sum(delta_class_sums(c, ys, xs, c_new, r), r, sigma) * (2.0 / (n * n))


def energy_class_sums(c: np.ndarray, r: int) -> np.ndarray:
    """Integer Y_d = sum_{o in class d} sum_{p, t} (c_p - c_{p+o})^2 (int64)."""
    c = np.asarray(c, dtype=np.int64)
    classes = distance_classes(r)
    out = np.zeros(len(classes), dtype=np.int64)
    for ox, oy in window_offsets(r):
        diff = c - _neighbour(c, ox, oy)
        out[classes.index(ox * ox + oy * oy)] += int(np.sum(diff * diff))
    return out


def energy_exact(c: np.ndarray, n: int, r: int, sigma: float) -> float:
    """E from integer hit counts: (1/N^2) sum_d w(d) Y_d, added in increasing d."""
    return float(weighted_class_sum(energy_class_sums(c, r), r, sigma)) / (n * n)


def swap_class_sums(c: np.ndarray, ay, ax, by, bx, r: int) -> np.ndarray:
    """Integer X_d of exchanging the vectors of pixels a and b (Sec. 3.4).

    The swap is the two moves c_a -> c_b and c_b -> c_a evaluated on the
    unmodified state, plus a correction for the pair itself: for every window
    offset o with a + o = b on the torus, each single move counted the pair
    term (c_a - c_b)^2 once with the partner's old vector, while the true
    pair term does not change.  Per such offset, X_{|o|^2} gains
    2 sum_t (c_a,t - c_b,t)^2.  Returns int64 [M, n_classes]."""
    h, w, _ = c.shape
    ay, ax, by, bx = (np.asarray(v, dtype=np.int64) for v in (ay, ax, by, bx))
    ca = c[ay, ax].astype(np.int64)
    cb = c[by, bx].astype(np.int64)
    out = delta_class_sums(c, ay, ax, cb, r) + delta_class_sums(c, by, bx, ca, r)
    d2 = np.sum((ca - cb) ** 2, axis=1)
    classes = distance_classes(r)
    for ox, oy in window_offsets(r):
        linked = ((ay + oy) % h == by) & ((ax + ox) % w == bx)
        out[linked, classes.index(ox * ox + oy * oy)] += 2 * d2[linked]
    return out


def swap_delta_plain(e: np.ndarray, ay: int, ax: int, by: int, bx: int, r: int, sigma: float) -> float:
    """dE of exchanging e[ay, ax] and e[by, bx], plain FP64 form with the
    pair correction of ``swap_class_sums``."""
    h, w, _ = e.shape
    ea = np.asarray(e[ay, ax], dtype=np.float64)
    eb = np.asarray(e[by, bx], dtype=np.float64)
    total = delta_plain(e, ay, ax, eb, r, sigma) + delta_plain(e, by, bx, ea, r, sigma)
    for ox, oy in window_offsets(r):
        if (ay + oy) % h == by and (ax + ox) % w == bx:
            total += 4.0 * weight(ox * ox + oy * oy, sigma) * float(np.sum((ea - eb) ** 2))
    return total
