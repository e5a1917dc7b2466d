"""The BF16 precision form of the energy change (matrix-core Gram products).

The paper is silent on arithmetic precision; the form checked here is the
reading used by the library (each step stated below), written plainly:

* Operands.  The error vector of a pixel, e_t = c_t/N - A_t for a Heaviside
  row and e_t = g_t - I_t for a Gaussian row, is formed in FP32 (c/N is exact
  in FP32; A_t and g_t - I_t are rounded to FP32 first) and then rounded to
  BF16 (8 significant bits, round to nearest, ties to even):  e^_q.  The
  change of a moved pixel, delta_t = e'_t - e_t (in FP32: (c' - c)/N exactly,
  or g' - g rounded to FP32), is rounded to BF16 the same way:  delta^_t.
* Energy change (Eq. (1) over the window, both orderings of each pair,
  split as in the exact form):
      dE = 2 [ W sum_t delta_t (e'_t + e_t)  -  2 sum_o w_o sum_t delta_t e_{p+o,t} ],
  W = sum_o w_o.  The BF16 form keeps the first (self) sum in full precision
  and evaluates every neighbour product of the second sum with the BF16
  operands:  G_o = sum_t delta^_t e^_{p+o,t}.  Products of two BF16 values are
  exact in FP64, so this oracle's G_o is the exact value of the BF16 sum.
* Decision (Sec. 3.4's strict rule on that value) and refinement: a move the
  BF16 value accepts is re-evaluated exactly (integer Heaviside part, FP64
  Gaussian part) and committed only if that value accepts it too; otherwise
  it is a veto.  Moves the BF16 value rejects stay rejected.

Where N <= 256 and there are no Gaussian rows, counts and count changes are
exact in BF16; the library then feeds the integer counts themselves (an exact
Gram) and this form is not used.

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import numpy as np

from . import energy


def round_bf16(x) -> np.ndarray:
    """Round FP32 values to the nearest BF16 value (ties to even), returned as
    FP64.  BF16 keeps the sign, the 8 exponent bits and the top 7 fraction
    bits of FP32.  Inputs are first converted to FP32."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = (rounded & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out).astype(np.float64)


def heaviside_errors_fp32(c, n: int, areas) -> np.ndarray:
    """e = c/N - A in FP32 arithmetic (c/N exact, A rounded to FP32 first)."""
    cn = np.asarray(c, dtype=np.float32) * np.float32(1.0 / n)
    return (cn - np.asarray(areas, dtype=np.float64).astype(np.float32)).astype(np.float32)


def gaussian_errors_fp32(g, gint) -> np.ndarray:
    """e = g - I with g in FP32 and the difference rounded to FP32."""
    g32 = np.asarray(g, dtype=np.float64).astype(np.float32).astype(np.float64)
    return (g32 - np.asarray(gint, dtype=np.float64)).astype(np.float32)


def delta_bf16(c, ys, xs, c_new, n: int, areas, r: int, sigma: float,
               g=None, g_new=None, gint=None) -> np.ndarray:
    """BF16-form dE of moving pixels (ys[j], xs[j]) to counts c_new[j] (and
    Gaussian estimates g_new[j]), against the state c [H, W, T] (and g
    [H, W, T_G]).  FP64 result per move."""
    c = np.asarray(c, dtype=np.int64)
    h, w, _ = c.shape
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    c_old = c[ys, xs]
    c_new = np.asarray(c_new, dtype=np.int64)
    # exact self term and the BF16 change operand, Heaviside rows
    e_old = c_old / n - np.asarray(areas, dtype=np.float64)
    e_new = c_new / n - np.asarray(areas, dtype=np.float64)
    d = (c_new - c_old) / n
    self_sum = np.sum(d * (e_new + e_old), axis=1)
    d_hat = round_bf16(d)
    e_hat = round_bf16(heaviside_errors_fp32(c, n, areas))            # [H, W, T]
    if g is not None and np.asarray(g).shape[-1] > 0:
        g = np.asarray(g, dtype=np.float64)
        g_old = g[ys, xs]
        g_new = np.asarray(g_new, dtype=np.float64)
        gd = g_new - g_old
        self_sum = self_sum + np.sum(gd * (g_new + g_old - 2.0 * np.asarray(gint, dtype=np.float64)), axis=1)
        d_hat = np.concatenate([d_hat, round_bf16(gd.astype(np.float32))], axis=1)
        e_hat = np.concatenate([e_hat, round_bf16(gaussian_errors_fp32(g, gint))], axis=2)
    wsum = energy.weight_sum(r, sigma)
    gram = np.zeros(ys.shape[0], dtype=np.float64)
    for ox, oy in energy.window_offsets(r):
        eq = e_hat[(ys + oy) % h, (xs + ox) % w]
        gram += energy.weight(ox * ox + oy * oy, sigma) * np.sum(d_hat * eq, axis=1)
    return 2.0 * (wsum * self_sum - 2.0 * gram)


def delta_bf16_scale(c, ys, xs, c_new, n: int, areas, r: int, sigma: float,
                     g=None, g_new=None, gint=None) -> np.ndarray:
    """Sum of the magnitudes of the terms of delta_bf16 (the size against
    which its rounding and accumulation errors are measured)."""
    c = np.asarray(c, dtype=np.int64)
    h, w, _ = c.shape
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    c_old = c[ys, xs]
    c_new = np.asarray(c_new, dtype=np.int64)
    a = np.asarray(areas, dtype=np.float64)
    d = (c_new - c_old) / n
    selfmag = np.sum(np.abs(d * ((c_new + c_old) / n - 2.0 * a)), axis=1)
    e = c / n - a
    dd, ee = d, e
    if g is not None and np.asarray(g).shape[-1] > 0:
        g = np.asarray(g, dtype=np.float64)
        gd = np.asarray(g_new, dtype=np.float64) - g[ys, xs]
        gi = np.asarray(gint, dtype=np.float64)
        selfmag = selfmag + np.sum(np.abs(gd * (np.asarray(g_new) + g[ys, xs] - 2.0 * gi)), axis=1)
        dd = np.concatenate([d, gd], axis=1)
        ee = np.concatenate([e, g - gi], axis=2)
    gram = np.zeros(ys.shape[0], dtype=np.float64)
    for ox, oy in energy.window_offsets(r):
        gram += energy.weight(ox * ox + oy * oy, sigma) * np.sum(np.abs(dd * ee[(ys + oy) % h, (xs + ox) % w]),
                                                                axis=1)
    return 2.0 * (energy.weight_sum(r, sigma) * selfmag + 2.0 * gram)


def energy_bf16(c, n: int, areas, r: int, sigma: float, g=None, gint=None) -> float:
    """Eq. (1) over the window with BF16 operands: sum_p sum_o w_o |e^_p - e^_q|^2."""
    e_hat = round_bf16(heaviside_errors_fp32(c, n, areas))
    if g is not None and np.asarray(g).shape[-1] > 0:
        e_hat = np.concatenate([e_hat, round_bf16(gaussian_errors_fp32(g, gint))], axis=2)
    return energy.energy_plain(e_hat, r, sigma)
