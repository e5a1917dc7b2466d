"""Swap mutation (Sec. 3.4) on the GPU against the oracle: couples, exact
energy changes and decisions per pass, and whole trajectories, bit for bit."""
import numpy as np
import pytest

from oracle import energy, estimator, sweep as osw
import synthgen

from cases import gpu_problem, say, workload

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")

SWAP = {
    "n16": workload(move=1),
    "n16_ascend": workload(move=1, objective=-1),
    "tile4_alias": workload(move=1, width=4, height=4, radius=3, t_heaviside=9),
    "rect16x8": workload(move=1, width=16, height=8, radius=3, t_heaviside=70),
    "k1": workload(move=1, colour_k=1, width=8, height=8, radius=2),
    "k4": workload(move=1, colour_k=4, width=32, height=16, radius=3, t_heaviside=20),
    "n1": workload(move=1, n=1, g=(1, 1), t_heaviside=5),
    "n256_r4": workload(move=1, n=256, g=(1, 79), width=16, height=16, radius=4, t_heaviside=600,
                        objective=-1),
    "n1024_r5": workload(move=1, n=1024, g=(1, 381), width=16, height=16, radius=5, t_heaviside=66),
    "n4096_r6": workload(move=1, n=4096, g=(1, 1365), width=16, height=16, radius=6, t_heaviside=40),
    "r1": workload(move=1, width=8, height=32, radius=1, t_heaviside=130),
    # one colour class: every pixel is a pass member, so a workgroup's block
    # holds more members than one round of its member slots (three rounds at
    # r = 3, 32x8 blocks; two at r = 5, 32x4 blocks)
    "k1_rounds_r3": workload(move=1, colour_k=1, width=32, height=16, radius=3, t_heaviside=40),
    "k1_rounds_r5": workload(move=1, colour_k=1, width=32, height=16, radius=5, t_heaviside=40),
}


def oracle_swap(w, inp):
    return osw.Problem(n=w["n"], g=w["g"], width=w["width"], height=w["height"], radius=w["radius"],
                       sigma=w["sigma"], colour_k=w["colour_k"], seed=w["seed"],
                       problem_id=w.get("problem_id", 0), table=inp["heaviside"],
                       objective=w.get("objective", 1), move=1)


@pytest.mark.parametrize("name", list(SWAP))
def test_swap_passes_match_oracle(name):
    w = SWAP[name]
    say("case", name)
    inp = synthgen.problem_inputs(w)
    ref = oracle_swap(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    K2 = w["colour_k"] ** 2
    with gpu_problem(w, inp) as p:
        for s in range(2):
            for kappa in range(K2):
                p.phase_propose(kappa)
                p.phase_evaluate(kappa)
                got = p.get_swap_pass()
                ph = osw.swap_pass(ref, st, kappa)
                np.testing.assert_array_equal(got["a"], ph["a"])
                np.testing.assert_array_equal(got["b"], ph["b"])
                np.testing.assert_allclose(got["delta"], ph["delta"], rtol=1e-12, atol=0)
                np.testing.assert_array_equal(got["accept"], ph["accept"])
                p.phase_commit(kappa)
                np.testing.assert_array_equal(p.get_offsets(), st.u)
            p.phase_advance()
            st.sweep += 1
        np.testing.assert_array_equal(p.get_counts().reshape(st.c.shape), st.c)
        assert p.energy() == pytest.approx(osw.energy_of(ref, st), rel=1e-12)


@pytest.mark.parametrize("name,k", [("n16", 5), ("n256_r4", 3), ("k4", 2), ("tile4_alias", 4)])
def test_swap_sweeps_match_oracle(name, k):
    """bn_sweep's graph-replayed swap sweeps against the oracle's run; the
    accepted-couple count and the sweep index in the statistics."""
    w = SWAP[name]
    say("case", name, "sweeps", k)
    inp = synthgen.problem_inputs(w)
    ref = oracle_swap(w, inp)
    st = osw.run(ref, osw.initial_state(ref, inp["offsets"]), k)
    with gpu_problem(w, inp) as p:
        stats = p.sweep(k, stats=True)
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        np.testing.assert_array_equal(p.get_counts().reshape(st.c.shape), st.c)
        assert stats["accepts"] == sum(st.accepts)
        assert stats["proposals"] == k * w["width"] * w["height"] // 2
        assert stats["sweep_index"] == k
        e = p.get_errors()
        want = estimator.errors_from_counts(st.c, w["n"], ref.areas).reshape(e.shape)
        assert np.all(np.abs(e.astype(np.float64) - want) <= 1e-6 * np.maximum(np.abs(want), 1.0))


def test_swap_resume_and_profiled_schedule_agree():
    w = SWAP["n16_ascend"]
    inp = synthgen.problem_inputs(w)
    with gpu_problem(w, inp) as a:
        a.sweep(4)
        ua = a.get_offsets()
    with gpu_problem(w, inp) as b:
        b.sweep(1)
        b.set_profiling(True)
        b.sweep(2)
        prof = b.get_profile()
        b.set_profiling(False)
        b.sweep(1)
        np.testing.assert_array_equal(b.get_offsets(), ua)
    assert prof["phases"] == 2 * w["colour_k"] ** 2 and prof["recount_launches"] == 0


def test_full_size_tile256_swap_sampled():
    """256x256 tile, N=256, T=1024, 9x9 window: the first pass's couples
    (exact), and for sampled couples the energy change and decision, each
    computed by the oracle from the inputs around the couple."""
    w = workload("tile256_n256_t1024", move=1, objective=-1)
    inp = synthgen.problem_inputs(w)
    W, H, T, r = w["width"], w["height"], w["t_heaviside"], w["radius"]
    u0 = inp["offsets"].reshape(-1, 2).astype(np.int64)
    ref = oracle_swap(w, inp)
    with gpu_problem(w, inp) as p:
        p.phase_propose(0)
        p.phase_evaluate(0)
        got = p.get_swap_pass()
    a, b = osw.swap_couples(ref, 0, 0)
    np.testing.assert_array_equal(got["a"], a)
    np.testing.assert_array_equal(got["b"], b)
    # sampled couples, plus every couple whose members are window neighbours
    near = [i for i in range(len(a)) if abs(int(a[i]) // W - int(b[i]) // W) <= r
            and abs(int(a[i]) % W - int(b[i]) % W) <= r]
    idx = sorted(set(synthgen.pixel_sample(len(a), 6, seed=5).tolist()) | set(near[:4]))
    for i in idx:
        ay, ax = divmod(int(a[i]), W)
        by, bx = divmod(int(b[i]), W)
        win = {((yy + oy) % H, (xx + ox) % W) for yy, xx in ((ay, ax), (by, bx))
               for oy in range(-r, r + 1) for ox in range(-r, r + 1)}
        win = sorted(win)
        ids = np.array([yy * W + xx for yy, xx in win])
        local = np.zeros((H, W, T), dtype=np.int16)
        local[tuple(np.array(win).T)] = estimator.hit_counts(w["n"], w["g"], u0[ids], inp["heaviside"])
        xd = energy.swap_class_sums(local, [ay], [ax], [by], [bx], r)
        d = energy.weighted_class_sum(xd, r, w["sigma"])[0] * (2.0 / w["n"] ** 2)
        assert got["delta"][i] == pytest.approx(d, rel=1e-12)
        assert bool(got["accept"][i]) == bool(d > 0)



def test_full_size_tile256_swap_sweeps():
    """256x256 tile, N=256, T=1024, 9x9 window, two graph-replayed swap
    sweeps (ascent): the offsets are a permutation of the initial ones, the
    counts of sampled pixels are the oracle's estimator at their offsets, and
    the energy rose and equals the oracle's exact energy of all exported
    counts."""
    w = workload("tile256_n256_t1024", move=1, objective=-1)
    inp = synthgen.problem_inputs(w)
    W, H = w["width"], w["height"]
    u0 = inp["offsets"].reshape(-1, 2).astype(np.int64)
    with gpu_problem(w, inp) as p:
        e0 = p.energy()
        stats = p.sweep(2, stats=True)
        u = p.get_offsets().reshape(-1, 2).astype(np.int64)
        c = p.get_counts()
        e2 = p.energy()
    assert stats["accepts"] > 0 and e2 > e0
    key = lambda v: np.sort(v[:, 0] * 65536 + v[:, 1])
    np.testing.assert_array_equal(key(u), key(u0))
    assert np.any(u != u0)
    sample = synthgen.pixel_sample(W * H, 64, seed=6)
    np.testing.assert_array_equal(c[sample], estimator.hit_counts(w["n"], w["g"], u[sample], inp["heaviside"]))
    c3 = c.reshape(H, W, -1)
    xd = sum(energy.energy_class_sums(c3[:, :, t:t + 128], w["radius"]) for t in range(0, c3.shape[2], 128))
    e_ref = float(energy.weighted_class_sum(xd, w["radius"], w["sigma"])) / (w["n"] * w["n"])
    assert e2 == pytest.approx(e_ref, rel=1e-12)


def test_swap_call_order():
    w = SWAP["n16"]
    inp = synthgen.problem_inputs(w)
    with gpu_problem(w, inp) as p:
        with pytest.raises(bnlat.BnlatError):
            p.get_phase()
    w2 = workload()
    with gpu_problem(w2, synthgen.problem_inputs(w2)) as q:
        with pytest.raises(bnlat.BnlatError):
            q.get_swap_pass()


def test_swap_ascent_lowers_blurred_error_of_unseen_integrands():
    """The criterion of Sec. 3.3 (Fig. 1c) and the versatility claim of
    Sec. 3.5 on the GPU path, qualitatively (the paper's curves are not
    available): a 128x128 tile at 16 samples per pixel, generator (1, 5) as in
    Fig. 1a, optimised with the paper's swap mutation for 1000 sweeps on 256
    Heavisides (ascending the windowed energy), has a lower blurred error than
    the random tile it started from for blur sizes 1 to 8, on 1024 held-out
    Heavisides and on 1024 held-out Gaussians."""
    w = dict(n=16, g=(1, 5), width=128, height=128, t_heaviside=256, t_gauss=0, sigma=2.1, radius=3,
             colour_k=2, seed=11, problem_id=0)
    train = bnlat.draw_heavisides(11, 0, 256)
    held_h = bnlat.draw_heavisides(12, 0, 1024)
    held_g = bnlat.draw_gaussians(13, 0, 1024)
    u0 = synthgen.offsets(128, 128, seed=14)
    sig = [1.0, 2.0, 4.0, 8.0]

    def score(u):
        with bnlat.create_problem(dict(w, t_heaviside=1024), held_h) as q:
            q.init_offsets(u)
            q.compute_errors()
            qh = q.quality_metric(sig)
        with bnlat.create_problem(dict(w, t_heaviside=1, t_gauss=1024), held_h[:1], gaussians=held_g) as q:
            q.init_offsets(u)
            q.compute_errors()
            qg = q.quality_metric(sig, rows=bnlat.BN_ROWS_GAUSSIAN)
        return qh, qg

    with bnlat.create_problem(w, train, move=bnlat.BN_SWAP, objective=-1) as p:
        p.init_offsets(u0)
        p.compute_errors()
        e0 = p.energy()
        st = p.sweep(1000, stats=True)
        assert p.energy() > e0 and st["accepts"] > 0
        u = p.get_offsets()
    # swaps keep the multiset of offsets
    np.testing.assert_array_equal(np.sort(u.reshape(-1, 2).view(np.uint32).ravel()),
                                  np.sort(u0.reshape(-1, 2).view(np.uint32).ravel()))
    (h0, g0), (h1, g1) = score(u0), score(u)
    say("held-out Heaviside ratios", h1 / h0, "Gaussian ratios", g1 / g0)
    assert np.all(h1 < 0.8 * h0) and np.all(g1 < 0.8 * g0)
