"""Quality criterion: RMSE of the test-integrand error tile after Gaussian
blurring, over a range of blur sizes (Sec. 3.3; Fig. 1c plots
|(I_N * k_sigma) - I_ref| against the kernel size, sigma in [0.25, 20]).

Readings used here: the blur is a Gaussian of standard deviation sigma_b,
periodised over the toroidal tile and normalised to unit sum, applied
separably along x and y as circular convolutions; the criterion is
Q(sigma_b) = sqrt(mean over pixels and integrands of the blurred error^2).

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULT_SIGMAS = (0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 20.0)


def periodic_kernel(n: int, sigma_b: float) -> np.ndarray:
    """k(d) = sum_m exp(-(d + m n)^2 / (2 sigma_b^2)), d = 0..n-1, |m| <= ceil(6 sigma_b / n) + 1,
    normalised to sum 1."""
    reps = int(math.ceil(6.0 * sigma_b / n)) + 1
    k = np.zeros(n, dtype=np.float64)
    for d in range(n):
        for m in range(-reps, reps + 1):
            k[d] += math.exp(-((d + m * n) ** 2) / (2.0 * sigma_b * sigma_b))
    return k / k.sum()


def circulant(k: np.ndarray) -> np.ndarray:
    """C[i, j] = k[(i - j) mod n]: (C v)[i] = sum_j k[i - j] v[j]."""
    n = k.shape[0]
    i = np.arange(n)
    return k[(i[:, None] - i[None, :]) % n]


def blur(e: np.ndarray, sigma_b: float) -> np.ndarray:
    """Separable circular Gaussian blur of an error field e [H, W, T]."""
    h, w, _ = e.shape
    cy = circulant(periodic_kernel(h, sigma_b))
    cx = circulant(periodic_kernel(w, sigma_b))
    tmp = np.einsum("xa,yat->yxt", cx, np.asarray(e, dtype=np.float64))
    return np.einsum("yb,bxt->yxt", cy, tmp)


def quality(e: np.ndarray, sigmas=DEFAULT_SIGMAS) -> np.ndarray:
    """Q(sigma_b) for each blur size."""
    return np.array([math.sqrt(float(np.mean(blur(e, s) ** 2))) for s in sigmas])


def radial_bin(u, v, w: int, h: int) -> np.ndarray:
    """Radial bin of DFT frequency (u, v) of a W x H torus: the frequency in
    cycles per pixel, (u', v') = (u/W or u/W - 1, v/H or v/H - 1) folded to
    [-1/2, 1/2), has radius rho; the bin is rho measured in units of
    1 / min(W, H), rounded to the nearest integer."""
    fu = np.where(np.asarray(u) * 2 < w, np.asarray(u) / w, np.asarray(u) / w - 1.0)
    fv = np.where(np.asarray(v) * 2 < h, np.asarray(v) / h, np.asarray(v) / h - 1.0)
    return np.rint(np.sqrt(fu * fu + fv * fv) * min(w, h)).astype(np.int64)


def error_spectrum(e: np.ndarray, nbins: int):
    """Radially averaged power spectrum of the error tile (the insets of
    Fig. 1b show |FFT(e)|^2 of one integrand's error): for every integrand t,
    |DFT2(e_t)(u, v)|^2 / P over the W x H torus; averaged over the
    integrands and over the frequencies of each radial bin (radial_bin).
    Returns (mean power [nbins], frequencies per bin [nbins]); bins with no
    frequency hold 0."""
    e = np.asarray(e, dtype=np.float64)
    h, w, t = e.shape
    power = np.zeros((h, w), dtype=np.float64)
    for k in range(t):
        power += np.abs(np.fft.fft2(e[:, :, k])) ** 2
    power /= (h * w) * t
    vv, uu = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    b = radial_bin(uu, vv, w, h)
    sums = np.zeros(nbins)
    counts = np.zeros(nbins, dtype=np.int64)
    keep = b < nbins
    np.add.at(sums, b[keep], power[keep])
    np.add.at(counts, b[keep], 1)
    return np.where(counts > 0, sums / np.maximum(counts, 1), 0.0), counts
