"""Pins of the oracle's swap mutation (Sec. 3.4: couples of pixels exchange
their offsets, evaluated on the unmodified state).  CPU only."""
import numpy as np
import pytest

from oracle import energy, estimator, philox, sweep
import synthgen


def rand_counts(h, w, t, n, seed):
    return np.random.default_rng(seed).integers(0, n + 1, size=(h, w, t)).astype(np.int64)


def swap_problem(w=16, h=16, n=16, g=(1, 7), t=12, r=3, k=2, seed=5, objective=1):
    return sweep.Problem(n=n, g=g, width=w, height=h, radius=r, sigma=2.1, colour_k=k, seed=seed,
                         problem_id=0, table=synthgen.heaviside_table(t, seed=seed), objective=objective,
                         move=1)


def couples_for(h, w, seed):
    """Random couples plus every partner inside the window of (1, 2), so the
    pair correction is exercised for each distance class."""
    g = np.random.default_rng(seed)
    out = [tuple(int(v) for v in g.integers(0, [h, w, h, w])) for _ in range(6)]
    out = [c for c in out if (c[0], c[1]) != (c[2], c[3])]
    for oy in range(-3, 4):
        for ox in range(-3, 4):
            if (ox, oy) != (0, 0):
                out.append((1, 2, (1 + oy) % h, (2 + ox) % w))
    return [c for c in out if (c[0], c[1]) != (c[2], c[3])]


@pytest.mark.parametrize("h,w,r", [(4, 4, 3), (8, 8, 3), (8, 8, 2), (6, 10, 3), (16, 8, 4)])
def test_swap_class_sums_equal_energy_class_differences(h, w, r):
    """Exchanging two pixels' counts changes the integer energy class sums
    Y_d (sum over offsets of class d, pixels and integrands of squared
    differences) by exactly 2 X_d, class by class, whether or not the two
    pixels are within each other's window (and on the 4x4 tile, where
    offsets alias)."""
    n = 16
    c = rand_counts(h, w, 5, n, h * w + r)
    for ay, ax, by, bx in couples_for(h, w, r):
        c2 = c.copy()
        c2[ay, ax], c2[by, bx] = c[by, bx], c[ay, ax]
        want = energy.energy_class_sums(c2, r) - energy.energy_class_sums(c, r)
        got = energy.swap_class_sums(c, [ay], [ax], [by], [bx], r)[0]
        np.testing.assert_array_equal(2 * got, want)


@pytest.mark.parametrize("h,w,r", [(4, 4, 3), (8, 8, 3), (6, 10, 2)])
def test_swap_delta_plain_equals_brute_force(h, w, r):
    """Real-valued vectors: the swap change equals the loop energy of the
    swapped field minus that of the original."""
    e = np.random.default_rng(r + h).normal(size=(h, w, 3))
    for ay, ax, by, bx in couples_for(h, w, 7 + r):
        e2 = e.copy()
        e2[ay, ax], e2[by, bx] = e[by, bx], e[ay, ax]
        want = energy.energy_loops(e2, r, 2.1) - energy.energy_loops(e, r, 2.1)
        assert energy.swap_delta_plain(e, ay, ax, by, bx, r, 2.1) == pytest.approx(want, rel=1e-9, abs=1e-9)


def test_swap_exact_matches_plain_form():
    n, r = 16, 3
    c = rand_counts(8, 8, 6, n, 3)
    e = c / n - 0.3
    cp = couples_for(8, 8, 1)
    ay, ax, by, bx = (np.array([q[i] for q in cp]) for i in range(4))
    exact = energy.weighted_class_sum(energy.swap_class_sums(c, ay, ax, by, bx, r), r, 2.1) * (2.0 / n ** 2)
    plain = [energy.swap_delta_plain(e, *q, r, 2.1) for q in cp]
    np.testing.assert_allclose(exact, plain, rtol=1e-10, atol=1e-12)


def test_permutation_and_passes():
    """pi is a permutation sorted by its Philox keys; every pass takes P/K^2
    distinct pixels in disjoint couples; masks stay in range."""
    prob = swap_problem(w=16, h=8)
    P = 128
    perm = prob.perm
    assert sorted(perm.tolist()) == list(range(P))
    w = philox.draw(np.arange(P), 0, 0, philox.S_PERM, prob.seed)
    keys = [(int(a) << 32) | int(b) for a, b in zip(w[:, 0], w[:, 1])]
    assert all(keys[perm[i]] <= keys[perm[i + 1]] for i in range(P - 1))
    seen_masks = set()
    for s in range(3):
        for kappa in range(4):
            a, b = sweep.swap_couples(prob, s, kappa)
            both = np.concatenate([a, b])
            assert len(a) == len(b) == P // 8
            assert len(set(both.tolist())) == P // 4 and both.min() >= 0 and both.max() < P
            seen_masks.add(sweep.swap_mask(prob, s, kappa))
    assert len(seen_masks) > 1


def test_swaps_permute_offsets_and_move_counts_with_them():
    """Swap sweeps only permute the tile (the multiset of offsets is kept)
    and the counts travel with the offsets: recounting the final offsets
    gives the state's counts."""
    prob = swap_problem(objective=-1)
    u0 = synthgen.offsets(16, 16, seed=9)
    st = sweep.run(prob, sweep.initial_state(prob, u0), 4)
    assert sum(st.accepts) > 0
    key = lambda u: sorted(map(tuple, u.reshape(-1, 2).tolist()))
    assert key(st.u) == key(np.asarray(u0, dtype=np.int64))
    recount = estimator.hit_counts(prob.n, prob.g, st.u.reshape(-1, 2), prob.table).reshape(st.c.shape)
    np.testing.assert_array_equal(recount, st.c)


def test_sequential_swaps_track_energy_exactly():
    """Applying the couples of a pass one at a time (each evaluated on the
    current state) changes the exact energy by exactly the swap change, and
    the descending objective never raises it."""
    prob = swap_problem(w=8, h=8, r=2)
    st = sweep.initial_state(prob, synthgen.offsets(8, 8, seed=2))
    y_prev = energy.energy_class_sums(st.c, prob.radius)
    moved = 0
    for kappa in range(4):
        a, b = sweep.swap_couples(prob, 0, kappa)
        for pa, pb in zip(a, b):
            (ay, ax), (by, bx) = divmod(int(pa), 8), divmod(int(pb), 8)
            xd = energy.swap_class_sums(st.c, [ay], [ax], [by], [bx], prob.radius)[0]
            d = energy.weighted_class_sum(xd, prob.radius, 2.1)
            if d < 0:
                st.c[ay, ax], st.c[by, bx] = st.c[by, bx].copy(), st.c[ay, ax].copy()
                moved += 1
                y_now = energy.energy_class_sums(st.c, prob.radius)
                np.testing.assert_array_equal(y_now - y_prev, 2 * xd)
                assert energy.weighted_class_sum(y_now, prob.radius, 2.1) < \
                    energy.weighted_class_sum(y_prev, prob.radius, 2.1)
                y_prev = y_now
    assert moved > 0


def test_swap_pass_decisions_follow_sign():
    prob = swap_problem()
    st = sweep.initial_state(prob, synthgen.offsets(16, 16, seed=3))
    ph = sweep.swap_pass(prob, st, 0)
    np.testing.assert_array_equal(ph["accept"], ph["delta"] < 0)
    prob.objective = -1
    ph = sweep.swap_pass(prob, st, 1)
    np.testing.assert_array_equal(ph["accept"], ph["delta"] > 0)


def test_swap_sweep_deterministic_and_resumable():
    prob = swap_problem()
    u0 = synthgen.offsets(16, 16, seed=6)
    a = sweep.run(prob, sweep.initial_state(prob, u0), 4)
    b = sweep.run(prob, sweep.initial_state(prob, u0), 2)
    b = sweep.run(prob, b, 2)
    np.testing.assert_array_equal(a.u, b.u)
    assert a.accepts == b.accepts


def test_ascending_swaps_lower_blurred_error():
    """Ascending the sum of Eq. (1) with swaps moves error energy to high
    frequencies: the blurred error (Sec. 3.3) drops below that of the random
    tile at moderate filter sizes."""
    from oracle import quality
    prob = swap_problem(w=32, h=32, t=16, objective=-1)
    u0 = synthgen.offsets(32, 32, seed=4)
    st0 = sweep.initial_state(prob, u0)
    q0 = quality.quality(sweep.errors(prob, st0), (1.0, 2.0))
    st = sweep.run(prob, sweep.initial_state(prob, u0), 10)
    q1 = quality.quality(sweep.errors(prob, st), (1.0, 2.0))
    assert np.all(q1 < 0.9 * q0)


def test_swap_validation():
    with pytest.raises(ValueError):
        swap_problem(w=12, h=8)            # P not a power of two
    with pytest.raises(ValueError):
        sweep.Problem(n=16, g=(1, 7), width=8, height=8, radius=2, sigma=2.1, colour_k=2, seed=0,
                      problem_id=0, table=synthgen.heaviside_table(3, seed=0), move=2)
    with pytest.raises(ValueError):
        sweep.Problem(n=16, g=(1, 7), width=8, height=8, radius=2, sigma=2.1, colour_k=2, seed=0,
                      problem_id=0, table=synthgen.heaviside_table(3, seed=0), move=1,
                      gauss=synthgen.gaussian_table(2, seed=0))
