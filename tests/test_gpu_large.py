"""Full size of the largest configuration: a 512x512 tile, N = 1024,
g = (1, 381), 3072 Heavisides + 1024 Gaussians, 11x11 window, BF16 form (the
members of the benchmark's large batch).  Sampled outputs are computed one by
one by the oracle from the inputs: hit counts and error vectors after
bn_compute_errors, and the first colour phase's proposals, recounts, energy
changes and decisions.  N = 1024 with Gaussian rows runs the BF16 form's
approximate mode: the matrix-core energy change is compared with the
oracle's BF16 form, and a move is committed exactly when that value and the
exact re-evaluation both accept it."""
import numpy as np
import pytest

from oracle import energy, estimator, precision, sweep as osw
import synthgen

from cases import check_errors, gpu_problem, oracle_problem, say, workload

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")


def test_large_config_sampled():
    w = dict(workload("tile512_n1024_t4096"), precision=1)
    say("case", "tile512_n1024_t4096 bf16")
    inp = synthgen.problem_inputs(w)
    W, H, T, r, n = w["width"], w["height"], w["t_heaviside"], w["radius"], w["n"]
    u0 = inp["offsets"].reshape(-1, 2).astype(np.int64)
    ref = oracle_problem(w, inp)
    gint = ref.gauss_integrals
    with gpu_problem(w, inp) as p:
        c_gpu = p.get_counts()
        e_gpu = p.get_errors()
        p.phase_propose(0)
        p.phase_evaluate(0)
        ph = p.get_phase()
        dbf = p.get_phase_bf16()
    sample = synthgen.pixel_sample(W * H, 16, seed=5)
    c_ref = estimator.hit_counts(n, w["g"], u0[sample], inp["heaviside"], chunk=4)
    np.testing.assert_array_equal(c_gpu[sample], c_ref)
    check_errors(e_gpu[sample, :T], c_ref, n, ref.areas)
    g_ref = estimator.gauss_estimates(n, w["g"], u0[sample], inp["gauss"], chunk=4)
    e64 = g_ref - gint
    scale = np.maximum(np.maximum(np.abs(e64), gint), np.abs(g_ref))
    assert np.all(np.abs(e_gpu[sample, T:].astype(np.float64) - e64) <= 1e-6 * scale + 1e-12)
    del c_gpu, e_gpu
    # first phase, class 0: class pixel j sits at (2a, 2b), j = a * W/2 + b; the
    # window is rebuilt as an 11x11 tile centred on the pixel (offsets within
    # the radius never wrap there)
    for j in synthgen.pixel_sample((W // 2) * (H // 2), 2, seed=6):
        y, x = 2 * (int(j) // (W // 2)), 2 * (int(j) % (W // 2))
        ids = np.array([((y + oy) % H) * W + (x + ox) % W for oy in range(-r, r + 1) for ox in range(-r, r + 1)])
        s = 2 * r + 1
        c_loc = estimator.hit_counts(n, w["g"], u0[ids], inp["heaviside"], chunk=4).reshape(s, s, T)
        g_loc = estimator.gauss_estimates(n, w["g"], u0[ids], inp["gauss"], chunk=4).reshape(s, s, -1)
        u_new = osw.proposals(ref, np.array([y]), np.array([x]), 0).astype(np.int64)
        np.testing.assert_array_equal(ph["u_new"][j], u_new[0])
        c_new = estimator.hit_counts(n, w["g"], u_new, inp["heaviside"], chunk=4)
        np.testing.assert_array_equal(ph["c_new"][j], c_new[0])
        g_new = estimator.gauss_estimates(n, w["g"], u_new, inp["gauss"], chunk=4)[0]
        d_h = energy.delta_exact(c_loc, [r], [r], c_new, n, r, w["sigma"])[0]
        d_g = energy.delta_plain(g_loc, r, r, g_new, r, w["sigma"])
        want = d_h + d_g
        kw = dict(g=g_loc, g_new=g_new[None], gint=gint)
        bf = precision.delta_bf16(c_loc, [r], [r], c_new, n, ref.areas, r, w["sigma"], **kw)[0]
        size = precision.delta_bf16_scale(c_loc, [r], [r], c_new, n, ref.areas, r, w["sigma"], **kw)[0]
        say("pixel", j, "BF16 delta", dbf[j], "oracle BF16", bf, "exact", want, "final", ph["delta"][j])
        # the Gaussian rows' BF16 operands come from FP32 estimates: allow their part's own
        # rounding size (4 unit roundoffs of its terms)
        gsize = size - precision.delta_bf16_scale(c_loc, [r], [r], c_new, n, ref.areas, r, w["sigma"])[0]
        assert abs(dbf[j] - bf) <= 1e-5 * size + 4 * 2.0 ** -8 * gsize
        bf_acc = dbf[j] < 0
        assert bool(ph["accept"][j]) == bool(bf_acc and want < 0)
        if ph["accept"][j]:
            assert abs(ph["delta"][j] - want) <= 1e-5 * (abs(d_h) + abs(d_g))
        else:
            assert ph["delta"][j] == dbf[j] or (bf_acc and abs(ph["delta"][j] - want) <= 1e-5 * (abs(d_h) + abs(d_g)))
