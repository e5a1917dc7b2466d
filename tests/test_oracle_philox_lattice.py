"""Pins of the oracle's Philox, lattice and scrambling (CPU only)."""
import os
import subprocess

import numpy as np
import pytest

from oracle import estimator, lattice, philox
import synthgen

HERE = os.path.dirname(os.path.abspath(__file__))
Q16 = 1 << 16


# --------------------------------------------------------------------- Philox
@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("philox") / "ref")
    cmd = ["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    """Oracle Philox4x32-10 vs rocRAND's implementation of the same published
    generator, on random and structured counters/keys."""
    g = np.random.default_rng(7)
    rows = [(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0), (0, 0, 0, 0xC, 0, 0),
            (65535, 1999, 31, philox.S_PROP, 2, 0)]
    for _ in range(200):
        c = g.integers(0, 2 ** 32, size=4)
        c[1] %= 2 ** 30
        k = g.integers(0, 2 ** 32, size=2)
        rows.append(tuple(int(v) for v in (*c, *k)))
    text = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=text, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    got = np.stack([philox.philox4x32_10(r[:4], r[4:]) for r in rows]).astype(np.uint64)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)


def test_philox_vectorised_equals_scalar():
    ctr = np.array([[i, 3, 5, philox.S_INIT] for i in range(50)], dtype=np.uint64)
    vec = philox.philox4x32_10(ctr, (11, 12))
    for i in range(50):
        np.testing.assert_array_equal(vec[i], philox.philox4x32_10(ctr[i], (11, 12)))


def test_q16_pair_takes_top_bits():
    w = np.array([[0xABCD1234, 0x0001FFFF, 0, 0]], dtype=np.uint32)
    np.testing.assert_array_equal(philox.q16_pair(w), [[0xABCD, 0x0001]])


# -------------------------------------------------------------------- lattice
def load_fig1a():
    rows = []
    with open(os.path.join(HERE, "golden", "fig1a_points.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p, k, x, y = line.split()
                rows.append((int(p), int(k), float(x), float(y)))
    return rows


def test_fig1a_worked_example():
    """Fig. 1a: 16-point lattice with generator (1, 5), van der Corput order,
    additive mod-1 scrambling.  Both pixels' x coordinates match for all 16
    samples; the y coordinates match for the ten samples k in
    {1,3,5,6,7,9,11,13,14,15}; the six others are printed 0.004-0.008 below
    the lattice value (read as perturbed figure data)."""
    rows = load_fig1a()
    seq = lattice.sequence_q16(16, (1, 5))
    consistent_y = {1, 3, 5, 6, 7, 9, 11, 13, 14, 15}
    for pix in (0, 1):
        pts = [r for r in rows if r[0] == pix]
        u = (int(round(pts[0][2] * Q16)), int(round(0.5625 * Q16)))
        s = lattice.to_unit(lattice.scramble(seq, u))
        for _, k, x, y in pts:
            assert abs(s[k, 0] - x) <= 2.0 ** -16 + 1e-6, (pix, k)
            if k in consistent_y:
                assert abs(s[k, 1] - y) <= 1e-6, (pix, k)
            else:
                assert 0.003 < s[k, 1] - y < 0.008, (pix, k)


def test_fig1a_wrong_generator_or_order_fails():
    """The pin discriminates: generator (1, 3) or natural (non bit-reversed)
    order do not reproduce the printed points."""
    rows = [r for r in load_fig1a() if r[0] == 0]
    u = (int(round(rows[0][2] * Q16)), int(round(0.5625 * Q16)))
    natural = lattice.to_unit(lattice.scramble(lattice.lattice_q16(16, (1, 5)), u))
    wrong_g = lattice.to_unit(lattice.scramble(lattice.sequence_q16(16, (1, 3)), u))
    assert max(abs(natural[k, 0] - x) for _, k, x, _ in rows) > 0.1
    assert max(abs(wrong_g[k, 1] - y) for _, k, _, y in rows if k in (1, 3, 5)) > 0.1


def test_bitrev():
    assert [lattice.bitrev(k, 4) for k in range(16)] == [0, 8, 4, 12, 2, 10, 6, 14, 1, 9, 5, 13, 3, 11, 7, 15]


@pytest.mark.parametrize("n", [4, 16, 64, 256, 1024])
def test_one_point_per_stratum(n):
    """For generator components coprime to N each axis projection of the
    shifted lattice has exactly one point in every stratum [m/N, (m+1)/N)."""
    g = np.random.default_rng(n)
    for _ in range(20):
        gen = 2 * g.integers(0, 2 ** 15, size=2) + 1
        u = g.integers(0, Q16, size=2)
        pts = lattice.scramble(lattice.lattice_q16(n, gen), u)
        for a in range(2):
            strata = np.sort(pts[:, a] * n // Q16)
            np.testing.assert_array_equal(strata, np.arange(n))


def test_lattice_group_invariance():
    """The lattice is a group mod 1: shifting an offset by any lattice point
    permutes the point set and leaves every hit count unchanged."""
    n, gen = 64, (1, 19)
    table = synthgen.heaviside_table(40, seed=3)
    u = synthgen.offsets(5, 1, seed=4).reshape(-1, 2).astype(np.int64)
    L = lattice.lattice_q16(n, gen)
    base = estimator.hit_counts(n, gen, u, table)
    for k in (1, 7, 33, 63):
        moved = (u + L[k]) % Q16
        np.testing.assert_array_equal(estimator.hit_counts(n, gen, moved, table), base)


def test_lattice_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        lattice.lattice_q16(24, (1, 5))
