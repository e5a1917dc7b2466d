"""Pins of the oracle's energy, energy change, sweep and quality metric (CPU only)."""
import math

import numpy as np
import pytest

from oracle import energy, estimator, quality, sweep
import synthgen


def rand_field(h, w, t, seed):
    return np.random.default_rng(seed).normal(size=(h, w, t))


def rand_counts(h, w, t, n, seed):
    return np.random.default_rng(seed).integers(0, n + 1, size=(h, w, t)).astype(np.int64)


# --------------------------------------------------------------- energy (Eq. 1)
@pytest.mark.parametrize("h,w,r", [(4, 4, 3), (8, 8, 3), (8, 6, 2), (5, 7, 1)])
def test_energy_vectorised_equals_loops(h, w, r):
    e = rand_field(h, w, 3, h * w + r)
    assert energy.energy_plain(e, r, 2.1) == pytest.approx(energy.energy_loops(e, r, 2.1), rel=1e-12)


def test_energy_brute_force_literal_4x4():
    """Brute force straight from Eq. (1) on a 4x4 torus with a 7x7 window:
    pairs (p, q) weighted by the number of window offsets that reach q."""
    e = rand_field(4, 4, 2, 11)
    total = 0.0
    for py in range(4):
        for px in range(4):
            for qy in range(4):
                for qx in range(4):
                    for oy in range(-3, 4):
                        for ox in range(-3, 4):
                            if (ox, oy) == (0, 0):
                                continue
                            if (px + ox) % 4 == qx and (py + oy) % 4 == qy:
                                total += math.exp(-(ox * ox + oy * oy) / 2.1 ** 2) * float(
                                    np.sum((e[py, px] - e[qy, qx]) ** 2))
    assert energy.energy_plain(e, 3, 2.1) == pytest.approx(total, rel=1e-12)


@pytest.mark.parametrize("h,w,r", [(4, 4, 3), (8, 8, 3), (8, 8, 4), (6, 10, 2)])
def test_single_move_delta_equals_energy_difference(h, w, r):
    e = rand_field(h, w, 4, 100 + r)
    g = np.random.default_rng(r)
    for _ in range(5):
        y, x = int(g.integers(h)), int(g.integers(w))
        new = g.normal(size=4)
        e2 = e.copy()
        e2[y, x] = new
        want = energy.energy_plain(e2, r, 2.1) - energy.energy_plain(e, r, 2.1)
        assert energy.delta_plain(e, y, x, new, r, 2.1) == pytest.approx(want, rel=1e-10, abs=1e-10)


def test_exact_forms_match_plain_forms():
    n, r = 16, 3
    c = rand_counts(8, 8, 5, n, 1)
    areas = np.random.default_rng(2).uniform(0, 1, 5)
    e = estimator.errors_from_counts(c, n, areas)
    assert energy.energy_exact(c, n, r, 2.1) == pytest.approx(energy.energy_plain(e, r, 2.1), rel=1e-12)
    g = np.random.default_rng(3)
    ys, xs = g.integers(0, 8, 6), g.integers(0, 8, 6)
    c_new = g.integers(0, n + 1, size=(6, 5))
    d = energy.delta_exact(c, ys, xs, c_new, n, r, 2.1)
    for j in range(6):
        want = energy.delta_plain(e, ys[j], xs[j], c_new[j] / n - areas, r, 2.1)
        assert d[j] == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_energy_invariances():
    e = rand_field(8, 8, 4, 5)
    base = energy.energy_plain(e, 3, 2.1)
    assert base > 0
    assert energy.energy_plain(np.roll(e, (3, 5), axis=(0, 1)), 3, 2.1) == pytest.approx(base, rel=1e-12)
    assert energy.energy_plain(e + np.array([1.0, -2.0, 3.0, 0.5]), 3, 2.1) == pytest.approx(base, rel=1e-12)
    assert energy.energy_plain(e[..., ::-1], 3, 2.1) == pytest.approx(base, rel=1e-12)
    assert energy.energy_plain(np.broadcast_to(e[0, 0], e.shape), 3, 2.1) == 0.0


def test_window_weight_sum_closed_form():
    """sum_o exp(-|o|^2/sigma^2) is separable: (sum_d exp(-d^2/sigma^2))^2 - 1."""
    for r, want in ((3, 12.406706), (4, 12.798619), (5, 12.849952)):
        sep = sum(math.exp(-d * d / 2.1 ** 2) for d in range(-r, r + 1)) ** 2 - 1
        assert energy.weight_sum(r, 2.1) == pytest.approx(sep, rel=1e-14)
        assert sep == pytest.approx(want, abs=1e-6)
    assert [len(energy.distance_classes(r)) for r in (3, 4, 5)] == [9, 14, 19]
    assert len(energy.window_offsets(4)) == 80


# --------------------------------------------------------------------- sweeps
def small_problem(k=2, r=3, w=16, h=16, n=16, t=12, seed=0):
    table = synthgen.heaviside_table(t, seed=seed + 50)
    return sweep.Problem(n=n, g=(1, 7), width=w, height=h, radius=r, sigma=2.1, colour_k=k,
                         seed=seed, problem_id=0, table=table)


def test_sweep_deterministic_and_resumable():
    prob = small_problem()
    u0 = synthgen.offsets(16, 16, seed=1)
    a = sweep.run(prob, sweep.initial_state(prob, u0), 3)
    b = sweep.run(prob, sweep.initial_state(prob, u0), 3)
    np.testing.assert_array_equal(a.u, b.u)
    # resume: 1 sweep, rebuild the state from (offsets, sweep index), 2 more
    c = sweep.run(prob, sweep.initial_state(prob, u0), 1)
    d = sweep.initial_state(prob, c.u)
    d.sweep = c.sweep
    sweep.run(prob, d, 2)
    np.testing.assert_array_equal(a.u, d.u)
    np.testing.assert_array_equal(a.c, d.c)


def test_conflict_free_classes_are_additive_and_descend():
    """K >= r+1 dividing the tile: no two pixels of a class see each other, so
    each integer class sum of the energy moves by exactly twice the accepted
    moves' X_d, and the energy never rises."""
    prob = small_problem(k=4, r=3, w=16, h=16)
    st = sweep.initial_state(prob, synthgen.offsets(16, 16, seed=2))
    e_prev = sweep.energy_of(prob, st)
    for _ in range(2):
        for kappa in range(16):
            y_before = energy.energy_class_sums(st.c, prob.radius)
            ph = sweep.phase(prob, st, kappa)
            y_after = energy.energy_class_sums(st.c, prob.radius)
            np.testing.assert_array_equal(y_after - y_before, 2 * ph["xd"][ph["accept"]].sum(axis=0))
            e_now = sweep.energy_of(prob, st)
            assert e_now <= e_prev
            assert e_now == pytest.approx(e_prev + ph["delta"][ph["accept"]].sum(), rel=1e-10)
            e_prev = e_now
        st.sweep += 1


def test_accept_rule_matches_plain_delta():
    """Accepted exactly when the FP64 plain-form energy change is negative
    (checked away from ties)."""
    prob = small_problem()
    st = sweep.initial_state(prob, synthgen.offsets(16, 16, seed=3))
    e = sweep.errors(prob, st)
    ph = sweep.phase(prob, sweep.initial_state(prob, st.u), 0)
    for j in range(len(ph["ys"])):
        new = ph["c_new"][j] / prob.n - prob.areas
        d = energy.delta_plain(e, ph["ys"][j], ph["xs"][j], new, prob.radius, prob.sigma)
        assert d == pytest.approx(ph["delta"][j], rel=1e-10, abs=1e-12)
        if abs(d) > 1e-9:
            assert ph["accept"][j] == (d < 0)


def test_classes_partition_tile():
    seen = np.zeros(64, dtype=int)
    for kappa in range(4):
        ys, xs = sweep.class_pixels(8, 8, 2, kappa)
        assert len(ys) == 16
        seen[ys * 8 + xs] += 1
    assert np.all(seen == 1)


def test_descent_lowers_energy_ascent_raises_it():
    """Descending the sum of Eq. (1) lowers it; the ascending objective raises it."""
    prob = small_problem(w=32, h=32, t=16)
    u0 = synthgen.offsets(32, 32, seed=4)
    st = sweep.initial_state(prob, u0)
    e0 = sweep.energy_of(prob, st)
    sweep.run(prob, st, 8)
    assert sweep.energy_of(prob, st) < 0.9 * e0
    prob.objective = -1
    st = sweep.run(prob, sweep.initial_state(prob, u0), 8)
    assert sweep.energy_of(prob, st) > 1.1 * e0


def test_validation():
    with pytest.raises(ValueError):
        small_problem(n=12)
    with pytest.raises(ValueError):
        small_problem(k=3)
    with pytest.raises(ValueError):
        small_problem(r=16)
    with pytest.raises(ValueError):
        sweep.Problem(n=16, g=(2, 7), width=8, height=8, radius=2, sigma=2.1, colour_k=2, seed=0,
                      problem_id=0, table=synthgen.heaviside_table(3, seed=0))


# -------------------------------------------------------------------- quality
def test_quality_constant_field():
    e = np.full((8, 12, 3), 0.25)
    np.testing.assert_allclose(quality.quality(e), 0.25, rtol=1e-12)


def test_quality_impulse_closed_form():
    """Blurring a unit impulse gives the separable kernel itself."""
    h, w = 16, 20
    e = np.zeros((h, w, 1))
    e[3, 7, 0] = 1.0
    for s in (0.25, 1.0, 3.0, 20.0):
        kx, ky = quality.periodic_kernel(w, s), quality.periodic_kernel(h, s)
        want = math.sqrt(np.sum(kx ** 2) * np.sum(ky ** 2) / (h * w))
        assert quality.quality(e, (s,))[0] == pytest.approx(want, rel=1e-12)


def test_quality_matches_fft_convolution():
    e = rand_field(16, 12, 2, 8)
    for s in (0.5, 2.0, 8.0):
        kx, ky = quality.periodic_kernel(12, s), quality.periodic_kernel(16, s)
        k2 = np.outer(ky, kx)
        b = np.real(np.fft.ifft2(np.fft.fft2(e, axes=(0, 1)) * np.fft.fft2(k2)[..., None], axes=(0, 1)))
        np.testing.assert_allclose(quality.blur(e, s), b, atol=1e-12)


def test_quality_limits_and_white_noise():
    e = rand_field(64, 64, 8, 9)
    rmse = math.sqrt(np.mean(e ** 2))
    assert quality.quality(e, (0.05,))[0] == pytest.approx(rmse, rel=1e-9)
    big = quality.quality(e, (1000.0,))[0]
    assert big == pytest.approx(math.sqrt(np.mean(e.mean(axis=(0, 1)) ** 2)), rel=1e-6)
    # i.i.d. field: E[Q^2] = Q(0)^2 * sum_o k(o)^2
    for s in (1.0, 2.0):
        k2 = np.sum(quality.periodic_kernel(64, s) ** 2) ** 2
        assert quality.quality(e, (s,))[0] ** 2 == pytest.approx(rmse ** 2 * k2, rel=0.05)


def test_mixed_integrands_phase_consistent():
    """Heaviside + Gaussian rows: the phase's energy change equals the
    brute-force change of the full error field (both parts), and accepted
    moves are exactly the ones with a negative change."""
    prob = small_problem(w=12, h=12, t=6)
    prob.gauss = synthgen.gaussian_table(4, seed=5)
    prob.__post_init__()
    st = osw_initial = sweep.initial_state(prob, synthgen.offsets(12, 12, seed=6))
    e_before = sweep.errors(prob, st).copy()
    ph = sweep.phase(prob, sweep.initial_state(prob, st.u), 0)
    for j in range(0, len(ph["ys"]), 5):
        y, x = ph["ys"][j], ph["xs"][j]
        new = np.concatenate([ph["c_new"][j] / prob.n - prob.areas, ph["g_new"][j] - prob.gauss_integrals])
        want = energy.delta_plain(e_before, y, x, new, prob.radius, prob.sigma)
        assert ph["delta"][j] == pytest.approx(want, rel=1e-9, abs=1e-12)
        assert ph["accept"][j] == (ph["delta"][j] < 0)
    assert sweep.energy_of(prob, osw_initial) == pytest.approx(
        energy.energy_plain(e_before, prob.radius, prob.sigma), rel=1e-12)
