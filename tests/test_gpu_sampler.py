"""Padded sampler query (Sec. 3.1/3.2) on the GPU against the oracle: exact
sample values for random screen pixels, sample indices and dimension pairs."""
import numpy as np
import pytest

from oracle import sampler, sweep as osw
import synthgen

from cases import gpu_problem, oracle_problem, say, workload

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")


def test_batch_members_as_dimension_pairs():
    members = synthgen.dimension_pair_batch(count=6, seed=3, t=8, radius=1)
    probs, pairs = [], []
    try:
        for mw in members:
            say("pair", mw["width"], mw["height"], mw["n"], mw["g"])
            inp = synthgen.problem_inputs(mw)
            p = bnlat.create_problem(mw, bnlat.heaviside_array(inp["heaviside"]))
            p.init_offsets(inp["offsets"])
            probs.append(p)
            pairs.append(dict(n=mw["n"], g=mw["g"], width=mw["width"], height=mw["height"], u=inp["offsets"]))
        g = np.random.default_rng(7)
        m = 3000
        x, y = g.integers(0, 4096, m), g.integers(0, 4096, m)
        k = g.integers(0, 1 << 20, m)
        got = bnlat.sample(probs, x, y, k)
        want = sampler.sample_q16(pairs, x, y, k) / 65536.0
        np.testing.assert_array_equal(got.astype(np.float64), want)
    finally:
        for p in probs:
            p.close()


def test_sampler_reads_the_optimised_tile():
    """After swap sweeps the sampler returns the optimised tile's samples
    (the oracle's trajectory from the same inputs)."""
    w = workload(move=1, objective=-1, width=16, height=16, n=64, g=(1, 19), t_heaviside=20)
    inp = synthgen.problem_inputs(w)
    ref = osw.Problem(n=w["n"], g=w["g"], width=16, height=16, radius=w["radius"], sigma=w["sigma"],
                      colour_k=2, seed=w["seed"], problem_id=0, table=inp["heaviside"], objective=-1, move=1)
    st = osw.run(ref, osw.initial_state(ref, inp["offsets"]), 3)
    with gpu_problem(w, inp) as p:
        p.sweep(3)
        q = np.arange(16 * 16 * 4)
        x, y, k = q % 16, (q // 16) % 16, q // 256 + 5
        got = bnlat.sample([p], x, y, k)
    pair = dict(n=64, g=(1, 19), width=16, height=16, u=st.u.astype(np.uint16))
    np.testing.assert_array_equal(got.astype(np.float64), sampler.sample_q16([pair], x, y, k) / 65536.0)


def test_sampler_errors():
    w = workload()
    with bnlat.create_problem(w, None) as p:
        with pytest.raises(bnlat.BnlatError) as e:
            bnlat.sample([p], [0], [0], [0])
        assert e.value.status == bnlat.BN_ESTATE
        p.init_offsets(synthgen.offsets(w["width"], w["height"], seed=1))
        assert bnlat.sample([p], [], [], []).shape == (0, 2)
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.sample([], [0], [0], [0])
    assert e.value.status == bnlat.BN_EINVAL
