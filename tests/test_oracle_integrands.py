"""Pins of the oracle's integrands, integrals and hit counts (CPU only)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import estimator, integrands
import synthgen

Q16 = 1 << 16


def test_area_line_through_centre_is_half():
    g = np.random.default_rng(0)
    for _ in range(200):
        th = g.uniform(0, 2 * np.pi)
        nx, ny = int(round(16384 * math.cos(th))), int(round(16384 * math.sin(th)))
        assert abs(integrands.heaviside_area(nx, ny, 1 << 15, 1 << 15) - 0.5) < 1e-14


def test_area_axis_aligned():
    for c in (0, 1, 1000, 32768, 65535):
        assert integrands.heaviside_area(16384, 0, c, 77) == pytest.approx(1 - c / Q16, abs=1e-15)
        assert integrands.heaviside_area(-16384, 0, c, 77) == pytest.approx(c / Q16, abs=1e-15)
        assert integrands.heaviside_area(0, 16384, 5, c) == pytest.approx(1 - c / Q16, abs=1e-15)
        assert integrands.heaviside_area(0, -16384, 5, c) == pytest.approx(c / Q16, abs=1e-15)


def test_area_complement():
    t = synthgen.heaviside_table(300, seed=1)
    for nx, ny, cx, cy in zip(t["nx"], t["ny"], t["cx"], t["cy"]):
        a = integrands.heaviside_area(nx, ny, cx, cy)
        b = integrands.heaviside_area(-int(nx), -int(ny), cx, cy)
        assert 0.0 <= a <= 1.0
        assert a + b == pytest.approx(1.0, abs=1e-14)


def test_area_diagonal_triangles():
    """x + y > k: area 1 - k^2/2 for k <= 1, (2 - k)^2 / 2 for k >= 1."""
    for c in (0, 5000, 20000, 32768, 40000, 60000, 65535):
        k = 2 * c / Q16
        want = 1 - k * k / 2 if k <= 1 else (2 - k) ** 2 / 2
        assert integrands.heaviside_area(1000, 1000, c, c) == pytest.approx(want, abs=1e-14)


def test_area_midpoint_grid():
    """Dense midpoint-grid count of the strict predicate; only the cells cut
    by the edge can disagree, so the gap is below ~2 / grid."""
    m = 2048
    xs = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    t = synthgen.heaviside_table(12, seed=2)
    for nx, ny, cx, cy in zip(t["nx"], t["ny"], t["cx"], t["cy"]):
        nx, ny = float(nx), float(ny)
        inside = nx * (X - cx / Q16) + ny * (Y - cy / Q16) > 0
        assert abs(inside.mean() - integrands.heaviside_area(nx, ny, cx, cy)) < 2.0 / m


def test_axis_aligned_counts_closed_form():
    """n = (2**14, 0), generator x-component 1: the x coordinates are
    {m h + rho}, h = 2**16/N, rho = U_x mod h, so the hit count is the number
    of m with m h + rho > C_x."""
    g = np.random.default_rng(5)
    for n in (4, 16, 64, 256):
        h = Q16 // n
        for _ in range(30):
            cx = int(g.integers(0, Q16))
            u = g.integers(0, Q16, size=(1, 2))
            table = {"nx": np.array([16384], np.int16), "ny": np.array([0], np.int16),
                     "cx": np.array([cx], np.uint16), "cy": np.array([123], np.uint16)}
            rho = int(u[0, 0]) % h
            want = sum(1 for m in range(n) if m * h + rho > cx)
            assert estimator.hit_counts(n, (1, 3), u, table)[0, 0] == want
            table["nx"][0] = -16384
            want = sum(1 for m in range(n) if m * h + rho < cx)
            assert estimator.hit_counts(n, (1, 3), u, table)[0, 0] == want


def test_edge_point_is_not_a_hit():
    """A sample exactly on the edge is outside (strict inequality)."""
    table = {"nx": np.array([9000], np.int16), "ny": np.array([-4000], np.int16),
             "cx": np.array([0], np.uint16), "cy": np.array([0], np.uint16)}
    # N = 1: the only point is the offset itself; put it on the edge at C
    assert estimator.hit_counts(1, (1, 1), np.array([[0, 0]]), table)[0, 0] == 0
    assert estimator.hit_counts(1, (1, 1), np.array([[1, 0]]), table)[0, 0] == 1
    assert estimator.hit_counts(1, (1, 1), np.array([[0, 1]]), table)[0, 0] == 0


def test_mean_count_matches_area():
    """Averaged over uniformly random offsets the estimate c/N is unbiased:
    E[c/N] = A_t (checked statistically)."""
    t = synthgen.heaviside_table(8, seed=9)
    u = synthgen.offsets(64, 64, seed=10).reshape(-1, 2)
    c = estimator.hit_counts(16, (1, 7), u, t)
    np.testing.assert_allclose(c.mean(axis=0) / 16, integrands.heaviside_areas(t), atol=0.01)


def test_gaussian_integral_vs_quadrature():
    t = synthgen.gaussian_table(6, seed=3)
    for mx, my, s in zip(t["mx"], t["my"], t["s"]):
        ref, _ = integrate.dblquad(lambda y, x: math.exp(-((x - mx) ** 2 + (y - my) ** 2) / (2 * s * s)),
                                   0, 1, 0, 1, epsabs=1e-13, epsrel=1e-12)
        assert integrands.gaussian_integral(mx, my, s) == pytest.approx(ref, rel=1e-9, abs=1e-12)


def test_gaussian_integral_symmetry_and_limit():
    assert integrands.gaussian_integral(0.3, 0.8, 0.1) == pytest.approx(
        integrands.gaussian_integral(0.7, 0.2, 0.1), rel=1e-14)
    s = 0.01
    assert integrands.gaussian_integral(0.5, 0.5, s) == pytest.approx(2 * math.pi * s * s, rel=1e-12)


def test_gaussian_estimate_at_centre():
    """N = 1 and the offset at the centre: the estimate is exactly 1."""
    t = {"mx": np.array([0.25]), "my": np.array([0.5]), "s": np.array([0.1])}
    est = estimator.gauss_estimates(1, (1, 1), np.array([[16384, 32768]]), t)
    assert est[0, 0] == 1.0


def test_philox_heaviside_table_distribution():
    t = integrands.heaviside_table_philox(4000, seed=5)
    norm = np.hypot(t["nx"].astype(float), t["ny"].astype(float))
    assert np.all(np.abs(norm - 16384) < 1.0)
    ang = np.arctan2(t["ny"].astype(float), t["nx"].astype(float))
    hist, _ = np.histogram(ang, bins=8, range=(-np.pi, np.pi))
    assert hist.min() > 400 and hist.max() < 600
    assert abs(t["cx"].astype(float).mean() / Q16 - 0.5) < 0.02


def _one_point(mx, my, s, ux, uy):
    """Estimate of one Gaussian with N = 1: the single lattice point is the
    origin, so the only sample sits at the offset (ux, uy) / 2**16."""
    t = {"mx": np.array([mx]), "my": np.array([my]), "s": np.array([s])}
    return estimator.gauss_estimates(1, (1, 1), np.array([[ux, uy]]), t)[0, 0]


def test_gaussian_estimate_off_centre_levels():
    """Levels of an isotropic normal profile relative to its peak (Sec. 3.5's
    Gaussians have peak 1): one standard deviation away along an axis it is
    e^{-1/2}, two away e^{-2}, one along both axes e^{-1}, and at the half
    maximum radius s sqrt(2 ln 2) it is one half.  Centre (0.25, 0.5) and
    s = 1/16 are exact in Q0.16, so the sample distances are exact."""
    mx, my, s = 0.25, 0.5, 0.0625
    ux, uy, step = 16384, 32768, 4096          # Q0.16 of mx, my and of s
    assert _one_point(mx, my, s, ux + step, uy) == pytest.approx(0.6065306597126334, rel=1e-14)
    assert _one_point(mx, my, s, ux, uy - step) == pytest.approx(0.6065306597126334, rel=1e-14)
    assert _one_point(mx, my, s, ux + 2 * step, uy) == pytest.approx(0.1353352832366127, rel=1e-14)
    assert _one_point(mx, my, s, ux - step, uy + step) == pytest.approx(0.36787944117144233, rel=1e-14)
    # half maximum: distance 1/8 exactly, width chosen so that 1/8 is its HWHM
    s_half = 0.125 / math.sqrt(2.0 * math.log(2.0))
    assert _one_point(mx, my, s_half, ux + 8192, uy) == pytest.approx(0.5, rel=1e-13)


def test_gaussian_estimates_midpoint_grid_identity():
    """Shifting the N = 16 lattice by every offset of the midpoint grid
    ((a + 1/2) / G, (b + 1/2) / G), G = 512 a multiple of N, visits every
    point of that grid exactly N times (the lattice is a subgroup of the
    grid), so the mean estimate over those offsets is the midpoint rule of the
    integrand, within (h^2 / 24) (sup|f_xx| + sup|f_yy|) = 1 / (12 G^2 s^2) of
    the exact erf integral."""
    G = 512
    h = (1 << 16) // G
    a = np.arange(G) * h + h // 2
    ux, uy = np.meshgrid(a, a, indexing="xy")
    u = np.stack([ux.ravel(), uy.ravel()], axis=1)
    t = {"mx": np.array([0.5, 0.3, 0.8, 0.05]), "my": np.array([0.5, 0.6, 0.15, 0.9]),
         "s": np.array([0.1, 0.2, 0.3, 0.12])}
    est = estimator.gauss_estimates(16, (1, 7), u, t, chunk=8192).mean(axis=0)
    for k in range(4):
        exact = integrands.gaussian_integral(t["mx"][k], t["my"][k], t["s"][k])
        bound = 1.0 / (12.0 * G * G * t["s"][k] ** 2)
        assert abs(est[k] - exact) <= bound, (k, est[k], exact, bound)


def test_gaussian_estimates_unbiased_over_random_offsets():
    """Under a uniformly random shift every lattice point is uniform in the
    unit square, so the mean estimate over random offsets is the integral
    (checked to five standard errors of the sample mean)."""
    t = synthgen.gaussian_table(6, seed=21)
    u = synthgen.offsets(64, 64, seed=22).reshape(-1, 2)
    est = estimator.gauss_estimates(16, (1, 7), u, t)
    exact = integrands.gaussian_integrals(t)
    se = est.std(axis=0, ddof=1) / math.sqrt(est.shape[0])
    assert np.all(np.abs(est.mean(axis=0) - exact) <= 5.0 * se + 1e-12)


def test_philox_gaussian_table_distribution():
    """Drawn Gaussians (the config with 25 % Gaussians): centres uniform in
    [0, 1)^2, standard deviations uniform in [0.05, 0.3]."""
    t = integrands.gaussian_table_philox(20000, seed=5)
    for k in ("mx", "my"):
        assert t[k].min() >= 0.0 and t[k].max() < 1.0
        assert abs(t[k].mean() - 0.5) < 0.01
    s = t["s"]
    assert s.min() >= 0.05 and s.max() <= 0.3
    assert s.min() < 0.0501 and s.max() > 0.2999
    assert abs(s.mean() - 0.175) < 0.002
    hist, _ = np.histogram(s, bins=5, range=(0.05, 0.3))
    assert hist.min() > 3700 and hist.max() < 4300
    # the three parameters come from different words: no linear dependence
    assert abs(np.corrcoef(t["mx"], s)[0, 1]) < 0.03
    assert abs(np.corrcoef(t["mx"], t["my"])[0, 1]) < 0.03
