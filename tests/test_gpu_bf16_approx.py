"""BF16 matrix-core form, approximate mode (N > 256 or Gaussian rows): the
Gram products run on BF16-rounded error vectors, every accepted move is
re-evaluated exactly and committed only if confirmed (vetoes counted).

Per colour phase, from the GPU's phase-start offsets the oracle recomputes
counts and Gaussian estimates and checks:
  - proposals and recounts: bit-exact;
  - the matrix-core energy change against the oracle's BF16 form
    (oracle/precision.py): within 1e-5 of the sum of the magnitudes of its
    terms for the Heaviside rows; the Gaussian rows' BF16 operands are formed
    from FP32 estimates (within 1e-6 of the oracle's FP64 ones), so their
    part may move by its own BF16 rounding size;
  - decisions away from ties: the GPU's BF16 decision equals the oracle's, and
    a move is committed exactly when the BF16 value and the exact value (the
    FP32 form's arithmetic) both accept it; accepted moves carry the exact
    energy change; rejected-after-acceptance moves are the vetoes."""
import numpy as np
import pytest

from oracle import energy, estimator, precision, sweep as osw
import synthgen

from cases import gpu_problem, oracle_problem, say, workload

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")

U = 2.0 ** -8

CASES = {
    "n1024_r5": workload(n=1024, g=(1, 381), t_heaviside=66, width=12, height=12, radius=5, precision=1),
    "n512_k4": workload(n=512, g=(3, 101), t_heaviside=70, width=16, height=16, radius=3, colour_k=4,
                        precision=1),
    "n64_gauss": workload(n=64, g=(1, 19), t_heaviside=40, t_gauss=30, width=16, height=12, radius=3,
                          precision=1),
    "n1024_gauss_r5": workload(n=1024, g=(1, 381), t_heaviside=48, t_gauss=20, width=12, height=12, radius=5,
                               precision=1),
    "n2048_k1_ascend": workload(n=2048, g=(1, 763), t_heaviside=40, width=8, height=8, radius=2, colour_k=1,
                                objective=-1, precision=1),
}


def _parts(w, ref, c, gq, ys, xs, c_new, g_new):
    """Exact energy changes, the oracle's BF16-form ones, and their tolerance
    (Heaviside rows 1e-5 of the terms' size; Gaussian rows their BF16 size)."""
    n, r, sig = w["n"], w["radius"], w["sigma"]
    exact = energy.delta_exact(c, ys, xs, c_new, n, r, sig)
    size = np.abs(exact)
    if gq is not None:
        dg = np.array([energy.delta_plain(gq, y, x, g_new[j], r, sig) for j, (y, x) in enumerate(zip(ys, xs))])
        size = size + np.abs(dg)
        exact = exact + dg
    kw = dict(g=gq, g_new=g_new, gint=ref.gauss_integrals) if gq is not None else {}
    bf = precision.delta_bf16(c, ys, xs, c_new, n, ref.areas, r, sig, **kw)
    tol = 1e-5 * precision.delta_bf16_scale(c, ys, xs, c_new, n, ref.areas, r, sig, **kw)
    if gq is not None:
        H, W, _ = gq.shape
        eg = gq - ref.gauss_integrals
        d = g_new - gq[ys, xs]
        gpart = np.zeros(len(ys))
        for ox, oy in energy.window_offsets(r):
            gpart += energy.weight(ox * ox + oy * oy, sig) * np.sum(
                (np.abs(d) * 4 * U + 4e-6) * (np.abs(eg[(ys + oy) % H, (xs + ox) % W]) + 1e-6), axis=1)
        selfg = np.sum(4e-6 * (np.abs(g_new + gq[ys, xs] - 2 * ref.gauss_integrals) + np.abs(d) + 1e-6), axis=1)
        tol = tol + 4.0 * gpart + 2.0 * energy.weight_sum(r, sig) * selfg
    return exact, size, bf, tol


def _check_phase(w, ref, inp, p, kappa, sweep):
    W, H, K = w["width"], w["height"], w["colour_k"]
    u = p.get_offsets().reshape(-1, 2).astype(np.int64)
    c = estimator.hit_counts(w["n"], w["g"], u, inp["heaviside"]).reshape(H, W, -1)
    gq = None
    if w.get("t_gauss", 0):
        gq = estimator.gauss_estimates(w["n"], w["g"], u, inp["gauss"]).reshape(H, W, -1)
    p.phase_propose(kappa)
    p.phase_evaluate(kappa)
    got = p.get_phase()
    dbf = p.get_phase_bf16()
    ys, xs = osw.class_pixels(W, H, K, kappa)
    u_new = osw.proposals(ref, ys, xs, sweep).astype(np.int64)
    np.testing.assert_array_equal(got["u_new"], u_new)
    c_new = estimator.hit_counts(w["n"], w["g"], u_new, inp["heaviside"])
    np.testing.assert_array_equal(got["c_new"], c_new)
    g_new = estimator.gauss_estimates(w["n"], w["g"], u_new, inp["gauss"]) if gq is not None else None
    exact, size, bf, tol = _parts(w, ref, c, gq, ys, xs, c_new, g_new)
    assert np.all(np.abs(dbf - bf) <= tol), np.max(np.abs(dbf - bf) / tol)
    sign = 1.0 if w.get("objective", 1) == 1 else -1.0
    bf_gpu = sign * dbf < 0
    far = np.abs(bf) > tol
    np.testing.assert_array_equal(bf_gpu[far], (sign * bf < 0)[far])
    acc = got["accept"]
    # committed = BF16 accepts and the exact re-evaluation confirms
    exact_tie = np.abs(exact) <= 1e-9 * np.maximum(1.0, np.abs(exact))
    assert np.all(bf_gpu[acc]) and np.all((sign * exact < 0)[acc])
    np.testing.assert_array_equal(acc[~exact_tie], (bf_gpu & (sign * exact < 0))[~exact_tie])
    # exact integers for Heaviside rows; FP32 estimates for Gaussian rows (the FP32 form's bar)
    rel = 1e-12 if gq is None else 1e-5
    assert np.all(np.abs(got["delta"][acc] - exact[acc]) <= rel * size[acc] + 1e-300)
    np.testing.assert_array_equal(got["delta"][~acc & ~bf_gpu], dbf[~acc & ~bf_gpu])
    p.phase_commit(kappa)
    return int(np.sum(bf_gpu & ~acc)), int(acc.sum())


@pytest.mark.parametrize("name", list(CASES))
def test_bf16_approx_phases_against_oracle(name):
    w = CASES[name]
    say("case", name)
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    vetoes = accepts = 0
    with gpu_problem(w, inp) as p:
        for s in range(2):
            for kappa in range(w["colour_k"] ** 2):
                v, a = _check_phase(w, ref, inp, p, kappa, s)
                vetoes += v
                accepts += a
            p.phase_advance()
    say("accepts", accepts, "vetoes", vetoes)
    assert accepts > 0


def test_bf16_approx_energy_against_oracle():
    """bn_energy_bf16 is the energy of the BF16-rounded error field
    (oracle/precision.py) and bn_energy the exact one; their gap is the form's
    error on the energy."""
    w = CASES["n1024_gauss_r5"]
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    u = inp["offsets"].reshape(-1, 2).astype(np.int64)
    H, W = w["height"], w["width"]
    c = estimator.hit_counts(w["n"], w["g"], u, inp["heaviside"]).reshape(H, W, -1)
    gq = estimator.gauss_estimates(w["n"], w["g"], u, inp["gauss"]).reshape(H, W, -1)
    want = precision.energy_bf16(c, w["n"], ref.areas, w["radius"], w["sigma"], g=gq, gint=ref.gauss_integrals)
    st = osw.initial_state(ref, inp["offsets"])
    with gpu_problem(w, inp) as p:
        ebf, e64 = p.energy_bf16(), p.energy()
    assert ebf == pytest.approx(want, rel=1e-5)
    assert e64 == pytest.approx(osw.energy_of(ref, st), rel=1e-9)
    say("BF16 energy", ebf, "FP64 energy", e64, "relative gap", abs(ebf - e64) / e64)
    assert abs(ebf - e64) <= 0.02 * e64


def test_bf16_approx_sweeps_reach_the_fp32_quality():
    """Graph-replayed sweeps of the BF16 form against the FP32 form on the
    same inputs (N = 1024, Heavisides and Gaussians, 11x11 window): final
    energies and blurred errors within 2 %, vetoes reported, and every
    committed state consistent (counts equal a recount of the offsets)."""
    w = workload(n=1024, g=(1, 381), t_heaviside=96, t_gauss=32, width=48, height=48, radius=5, seed=4)
    inp = synthgen.problem_inputs(w)
    out = {}
    for prec in (0, 1):
        with gpu_problem(dict(w, precision=prec), inp) as p:
            e0 = p.energy()
            st = p.sweep(12, stats=True)
            out[prec] = dict(e=p.energy(), q=p.quality_metric([1.0, 4.0]), st=st, u=p.get_offsets(),
                             c=p.get_counts(), ebf=p.energy_bf16() if prec else None)
    say("fp32", out[0]["e"], out[0]["st"], "bf16", out[1]["e"], out[1]["st"], "bf16 energy", out[1]["ebf"])
    assert out[1]["e"] < e0 and out[0]["e"] < e0
    assert abs(out[1]["e"] - out[0]["e"]) <= 0.02 * out[0]["e"]
    np.testing.assert_allclose(out[1]["q"], out[0]["q"], rtol=0.02)
    assert out[1]["st"]["bf16_vetoes"] >= 0 and out[0]["st"]["bf16_vetoes"] == 0
    assert abs(out[1]["ebf"] - out[1]["e"]) <= 0.02 * out[1]["e"]
    u = out[1]["u"].reshape(-1, 2).astype(np.int64)
    sample = synthgen.pixel_sample(w["width"] * w["height"], 40, seed=2)
    np.testing.assert_array_equal(out[1]["c"][sample], estimator.hit_counts(w["n"], w["g"], u[sample],
                                                                            inp["heaviside"]))
