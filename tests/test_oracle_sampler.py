"""Pins of the oracle's padded screen-space sampler (CPU only)."""
import numpy as np

from oracle import lattice, sampler
import synthgen


def pairs_fixture():
    shapes = [(16, (1, 5), 8, 8), (64, (1, 19), 4, 8), (4, (1, 3), 2, 2), (256, (1, 79), 16, 4)]
    return [dict(n=n, g=g, width=w, height=h, u=synthgen.offsets(w, h, seed=20 + i))
            for i, (n, g, w, h) in enumerate(shapes)]


def test_each_pixel_pair_is_stratified():
    """For every pixel of every pair, the N samples put exactly one point in
    each 1/N stratum of both dimensions (the shifted lattice's projections)."""
    pairs = pairs_fixture()
    for d, pr in enumerate(pairs):
        for yy in range(pr["height"]):
            for xx in range(pr["width"]):
                n = pr["n"]
                s = sampler.sample_q16(pairs, [xx] * n, [yy] * n, range(n))[:, 2 * d:2 * d + 2]
                for a in range(2):
                    strata = ((s[:, a] - int(pr["u"][yy, xx, a])) % 65536) // (65536 // n)
                    assert sorted(strata.tolist()) == list(range(n))


def test_tiles_repeat_and_sequence_repeats():
    """Screen pixels wrap modulo each pair's tile, sample indices modulo N."""
    pairs = pairs_fixture()
    g = np.random.default_rng(0)
    x, y, k = g.integers(0, 1000, 50), g.integers(0, 1000, 50), g.integers(0, 5000, 50)
    a = sampler.sample_q16(pairs, x, y, k)
    for d, pr in enumerate(pairs):
        b = sampler.sample_q16([pr], x % pr["width"] + pr["width"] * 7, y % pr["height"], k % pr["n"] + pr["n"])
        np.testing.assert_array_equal(a[:, 2 * d:2 * d + 2], b)


def test_fig1a_pixel_through_the_sampler():
    """A one-pixel pair with Fig. 1a's lattice (N = 16, generator (1, 5)):
    sample k of the pixel is frac(Phi(k) + u_x) along x (Fig. 1a's x
    coordinates), with Phi the base-2 radical inverse."""
    u = np.array([[[39654, 9000]]], dtype=np.uint16)
    pr = dict(n=16, g=(1, 5), width=1, height=1, u=u)
    s = sampler.sample_q16([pr], [0] * 16, [0] * 16, range(16))
    phi = np.array([lattice.bitrev(k, 4) / 16 for k in range(16)])
    np.testing.assert_array_equal(s[:, 0], np.round(((phi + 39654 / 65536) % 1.0) * 65536).astype(np.int64))
