"""Gaussian test integrands (Sec. 3.5) beside Heaviside rows.

Gaussian estimates are FP32 (exponent in FP64, exp2 in FP32, FP64 sums):
errors within 1e-6 of the larger of |e|, I and g; energy changes within 1e-5
of the oracle's FP64 values; decisions equal away from ties.  (The BF16
form with Gaussian rows, whose decisions come from BF16 values refined
exactly, is tested in test_gpu_bf16_approx.py.)"""
import numpy as np
import pytest

from oracle import energy, estimator, quality, sweep as osw
import synthgen

from cases import check_errors, gpu_problem, oracle_problem, say, workload

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")

MIX = {
    "mix_n64": workload(n=64, g=(1, 19), width=16, height=16, t_heaviside=20, t_gauss=70),
    "mix_n16_r2": workload(n=16, g=(1, 7), width=12, height=12, t_heaviside=9, t_gauss=10, radius=2),
    "mix_n256_r4": workload(n=256, g=(1, 79), width=12, height=12, t_heaviside=64, t_gauss=40, radius=4),
    "mix_ascend": workload(n=64, g=(1, 19), width=16, height=8, t_heaviside=16, t_gauss=24, objective=-1),
    # several LDS-staged workgroups, ragged Gaussian rows (130 of 192)
    "mix_r5_wide": workload(n=64, g=(1, 19), width=64, height=32, t_heaviside=16, t_gauss=130, radius=5),
    # region too large for the staged Gaussian kernel: per-pixel form
    "mix_k4_r6": workload(n=64, g=(1, 19), width=16, height=16, t_heaviside=8, t_gauss=20, radius=6,
                          colour_k=4),
    "mix_k1": workload(n=16, g=(1, 7), width=8, height=8, t_heaviside=6, t_gauss=12, radius=2, colour_k=1),
    # estimates over whole 512-sample chunks (smaller N take the masked tail)
    "mix_n1024": workload(n=1024, g=(1, 381), width=8, height=8, t_heaviside=8, t_gauss=40, radius=2),
}


def gauss_errors_ok(got, st, prob):
    ref = st.g.reshape(-1, st.g.shape[-1])
    e64 = ref - prob.gauss_integrals
    scale = np.maximum(np.maximum(np.abs(e64), prob.gauss_integrals), np.abs(ref))
    assert np.all(np.abs(got.astype(np.float64) - e64) <= 1e-6 * scale + 1e-12)


@pytest.mark.parametrize("name", list(MIX))
def test_gauss_estimates_and_phases(name):
    w = MIX[name]
    say("case", name)
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    T = w["t_heaviside"]
    with gpu_problem(w, inp) as p:
        _, _, g, gi = p.get_integrands(gaussians=True)
        np.testing.assert_allclose(gi, ref.gauss_integrals, rtol=1e-14)
        e = p.get_errors()
        check_errors(e[:, :T], st.c.reshape(-1, T), w["n"], ref.areas)
        gauss_errors_ok(e[:, T:], st, ref)
        for s in range(2):
            for kappa in range(w["colour_k"] ** 2):
                p.phase_propose(kappa)
                p.phase_evaluate(kappa)
                got = p.get_phase()
                ph = osw.phase(ref, st, kappa)
                np.testing.assert_array_equal(got["c_new"], ph["c_new"])
                d_ref = ph["delta"]
                tol = 1e-5 * (np.abs(d_ref) + np.median(np.abs(d_ref)))
                assert np.all(np.abs(got["delta"] - d_ref) <= tol)
                clear = np.abs(d_ref) > 1e-4 * np.median(np.abs(d_ref))
                np.testing.assert_array_equal(got["accept"][clear], ph["accept"][clear])
                assert np.array_equal(got["accept"], ph["accept"]), "decision differs at a near-tie"
                p.phase_commit(kappa)
            p.phase_advance()
            st.sweep += 1
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        e = p.get_errors()
        gauss_errors_ok(e[:, T:], st, ref)
        assert p.energy() == pytest.approx(osw.energy_of(ref, st), rel=1e-5)
        sig = (0.5, 2.0, 8.0)
        np.testing.assert_allclose(p.quality_metric(sig), quality.quality(osw.errors(ref, st), sig), rtol=1e-5)


def test_gauss_sweep_and_list_delta():
    w = MIX["mix_n64"]
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    P = w["width"] * w["height"]
    pix = synthgen.pixel_sample(P, 24, seed=11)
    prop = synthgen.proposals(24, seed=12)
    ys, xs = np.divmod(pix.astype(np.int64), w["width"])
    c_new = estimator.hit_counts(w["n"], w["g"], prop.astype(np.int64), inp["heaviside"])
    g_new = estimator.gauss_estimates(w["n"], w["g"], prop.astype(np.int64), inp["gauss"])
    want = energy.delta_exact(st.c, ys, xs, c_new, w["n"], w["radius"], w["sigma"])
    want = want + np.array([energy.delta_plain(st.g, y, x, g_new[j], w["radius"], w["sigma"])
                            for j, (y, x) in enumerate(zip(ys, xs))])
    with gpu_problem(w, inp) as p:
        de = p.delta_energy(pix, prop)
        np.testing.assert_allclose(de, want, rtol=1e-5, atol=1e-5 * np.median(np.abs(want)))
        p.sweep(3)
        stt = osw.run(ref, osw.initial_state(ref, inp["offsets"]), 3)
        np.testing.assert_array_equal(p.get_offsets(), stt.u)
        assert p.energy() == pytest.approx(osw.energy_of(ref, stt), rel=1e-5)


def test_drawn_gaussians_used_when_none_given():
    w = MIX["mix_n16_r2"]
    with bnlat.create_problem(w, None) as p:
        _, _, g, _ = p.get_integrands(gaussians=True)
    np.testing.assert_array_equal(g, bnlat.draw_gaussians(w["seed"], 0, w["t_gauss"]))


def test_quality_metric_per_family():
    """The criterion over Heaviside rows only and Gaussian rows only, against
    the oracle's criterion of each family's error field; the all-rows value
    is their count-weighted root mean square."""
    w = MIX["mix_n64"]
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    e = osw.errors(ref, st)
    T, TG = w["t_heaviside"], w["t_gauss"]
    sig = (0.5, 2.0, 8.0)
    with gpu_problem(w, inp) as p:
        qh = p.quality_metric(sig, rows=bnlat.BN_ROWS_HEAVISIDE)
        qg = p.quality_metric(sig, rows=bnlat.BN_ROWS_GAUSSIAN)
        qa = p.quality_metric(sig)
    np.testing.assert_allclose(qh, quality.quality(e[..., :T], sig), rtol=1e-5)
    np.testing.assert_allclose(qg, quality.quality(e[..., T:], sig), rtol=1e-5)
    np.testing.assert_allclose(qa, np.sqrt((T * qh ** 2 + TG * qg ** 2) / (T + TG)), rtol=1e-6)
    wh = workload(n=16, g=(1, 7), width=8, height=8, t_heaviside=5, radius=2)
    with gpu_problem(wh, synthgen.problem_inputs(wh)) as q:
        with pytest.raises(bnlat.BnlatError):
            q.quality_metric(sig, rows=bnlat.BN_ROWS_GAUSSIAN)
