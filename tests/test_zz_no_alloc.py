"""The allocation-free entry point bn_delta_energy_noalloc against
bn_delta_energy (same kernels, list buffers in the library's fixed per-GPU
scratch array): energy changes and recounted hits equal on two calls in a row,
the second with fewer pixels, and across problems of different shapes that
share the one array."""
import numpy as np
import pytest

import synthgen
from oracle import energy, estimator

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")

from cases import gpu_problem, oracle_problem, say, workload  # noqa: E402


def _lists(w, m, seed):
    P = w["width"] * w["height"]
    return synthgen.pixel_sample(P, m, seed=seed), synthgen.proposals(m, seed=seed + 1)


@pytest.mark.parametrize("shape", [
    dict(n=256, g=(1, 79), width=64, height=64, t_heaviside=1024, radius=4),
    dict(n=64, g=(1, 19), width=48, height=32, t_heaviside=300, t_gauss=70, radius=3),
    dict(n=1024, g=(1, 381), width=24, height=24, t_heaviside=100, radius=5),
])
def test_noalloc_matches_allocating_entry_point(shape):
    w = workload(**shape)
    say("noalloc case", shape)
    inp = synthgen.problem_inputs(w)
    with gpu_problem(w, inp) as p:
        for m, seed in ((min(500, w["width"] * w["height"]), 3), (37, 5)):
            pix, prop = _lists(w, m, seed)
            de_ref, cn_ref = p.delta_energy(pix, prop, counts=True)
            de, cn = p.delta_energy_noalloc(pix, prop, counts=True)
            np.testing.assert_array_equal(cn, cn_ref)
            np.testing.assert_array_equal(de, de_ref)
            # without the row-layout counts
            np.testing.assert_array_equal(p.delta_energy_noalloc(pix, prop), de_ref)


def test_noalloc_against_oracle_and_shared_array():
    """Two problems use the same array one after the other; results still
    equal the oracle's exact energy changes and recounts."""
    wa = workload(n=256, g=(1, 79), width=16, height=16, t_heaviside=200, radius=4)
    wb = workload(n=16, g=(1, 7), width=32, height=32, t_heaviside=64, radius=3, seed=3)
    ia, ib = synthgen.problem_inputs(wa), synthgen.problem_inputs(wb)
    with gpu_problem(wa, ia) as pa, gpu_problem(wb, ib) as pb:
        for w, inp, p, m in ((wa, ia, pa, 120), (wb, ib, pb, 300), (wa, ia, pa, 9)):
            pix, prop = _lists(w, m, seed=m)
            de, cn = p.delta_energy_noalloc(pix, prop, counts=True)
            ref = oracle_problem(w, inp)
            c0 = estimator.hit_counts(w["n"], w["g"], inp["offsets"].reshape(-1, 2).astype(np.int64),
                                      inp["heaviside"]).reshape(w["height"], w["width"], -1)
            c_new = estimator.hit_counts(w["n"], w["g"], prop.astype(np.int64), inp["heaviside"])
            ys, xs = np.divmod(pix.astype(np.int64), w["width"])
            want = energy.delta_exact(c0, ys, xs, c_new, w["n"], w["radius"], w["sigma"])
            np.testing.assert_array_equal(cn, c_new)
            np.testing.assert_allclose(de, want, rtol=1e-12, atol=0)
            assert ref.areas.shape[0] == w["t_heaviside"]


def test_noalloc_rejects_lists_beyond_the_array():
    w = workload(n=16, g=(1, 7), width=128, height=128, t_heaviside=1024, radius=3)
    inp = synthgen.problem_inputs(w)
    with gpu_problem(w, inp) as p:
        pix, prop = _lists(w, 16384, seed=1)
        with pytest.raises(bnlat.BnlatError) as ei:
            p.delta_energy_noalloc(pix, prop, counts=True)
        assert ei.value.status == bnlat.BN_EINVAL
        # a list that fits still works afterwards
        pix, prop = _lists(w, 64, seed=2)
        np.testing.assert_array_equal(p.delta_energy_noalloc(pix, prop), p.delta_energy(pix, prop))
