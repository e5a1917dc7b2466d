"""Pins of the oracle's radially averaged error spectrum (oracle/quality.py):
Parseval's identity, white noise (flat spectrum at the variance), a single
plane wave (all its power in its own bin), the bin of every frequency against
a direct loop, and a constant field (power only at the origin)."""
import math

import numpy as np

from oracle import quality


def test_parseval_and_bins_cover_all_frequencies():
    rng = np.random.default_rng(3)
    e = rng.standard_normal((12, 20, 5))
    nb = 20
    s, c = quality.error_spectrum(e, nb)
    assert c.sum() == 12 * 20
    # sum over frequencies of |F|^2 / P equals sum over pixels of e^2 (per integrand, averaged)
    assert math.isclose(np.sum(s * c), np.sum(e ** 2) / 5, rel_tol=1e-12)


def test_white_noise_is_flat_at_its_variance():
    rng = np.random.default_rng(5)
    e = rng.standard_normal((64, 64, 200)) * 0.3
    s, c = quality.error_spectrum(e, 40)
    ok = c >= 20
    assert np.all(np.abs(s[ok] / 0.09 - 1.0) < 0.1)


def test_plane_wave_lands_in_its_bin():
    h, w = 32, 48
    y, x = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    e = np.cos(2 * np.pi * (3 * x / w + 5 * y / h))[:, :, None]
    s, c = quality.error_spectrum(e, 30)
    want = int(round(math.hypot(3 / w, 5 / h) * min(w, h)))
    assert np.argmax(s * c) == want
    assert math.isclose(s[want] * c[want], np.sum(e ** 2), rel_tol=1e-9)
    assert np.sum(np.delete(s * c, want)) < 1e-18 * np.sum(e ** 2) + 1e-20


def test_bins_match_a_direct_loop():
    h, w = 10, 14
    for v in range(h):
        for u in range(w):
            fu = u / w if 2 * u < w else u / w - 1
            fv = v / h if 2 * v < h else v / h - 1
            assert quality.radial_bin(u, v, w, h) == round(math.sqrt(fu * fu + fv * fv) * min(w, h))


def test_constant_field_has_power_only_at_the_origin():
    e = np.full((8, 8, 3), 0.25)
    s, c = quality.error_spectrum(e, 8)
    assert math.isclose(s[0] * c[0], 0.25 ** 2 * 64)
    assert np.all(s[1:] == 0)
