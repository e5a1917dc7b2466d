"""Batched form: many independent problems of uneven shapes swept by shared,
graph-captured launches.  Each member's trajectory must equal the oracle's
(small members) and the one it follows when swept alone (larger members)."""
import numpy as np
import pytest

from oracle import sweep as osw
import synthgen

from cases import oracle_problem, say, workload

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")


@pytest.fixture(scope="module")
def stream():
    import torch
    assert torch.cuda.is_available()
    return torch.cuda.Stream()


MEMBERS = [
    workload(n=4, g=(1, 3), width=16, height=16, t_heaviside=70, problem_id=0),
    workload(n=16, g=(1, 7), width=32, height=16, t_heaviside=40, problem_id=1),
    workload(n=64, g=(1, 19), width=16, height=16, t_heaviside=130, problem_id=2),
    workload(n=256, g=(1, 79), width=12, height=12, t_heaviside=64, radius=4, problem_id=3),
    workload(n=16, g=(3, 5), width=8, height=8, t_heaviside=20, radius=2, problem_id=4),
    workload(n=64, g=(5, 27), width=24, height=24, t_heaviside=33, problem_id=5),
]


def make(w, inp, stream):
    p = bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"]), stream=stream.cuda_stream)
    p.init_offsets(inp["offsets"])
    p.compute_errors()
    return p


def test_batched_members_follow_oracle(stream, tmp_path):
    k = 3
    inps = [synthgen.problem_inputs(w) for w in MEMBERS]
    probs = [make(w, inp, stream) for w, inp in zip(MEMBERS, inps)]
    cache = str(tmp_path / "tune.txt")
    with bnlat.Batch(probs, tune_cache=cache) as b:
        say("tuning", b.tuning())
        b.sweep(k)
    for w, inp, p in zip(MEMBERS, inps, probs):
        say("member", w["problem_id"], w["n"], w["width"], w["height"])
        ref = oracle_problem(w, inp)
        st = osw.run(ref, osw.initial_state(ref, inp["offsets"]), k)
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        np.testing.assert_array_equal(p.get_counts(), st.c.reshape(-1, w["t_heaviside"]))
        assert p.get_sweep_index() == k
        assert p.energy() == pytest.approx(osw.energy_of(ref, st), rel=1e-12)
        p.close()
    text = open(cache).read()
    assert "tch=" in text and "slices=" in text


def test_tune_cache_round_trip(stream, tmp_path):
    """The tuner's choice is written under the members' shape key and read
    back; a hand-written entry for the key is honoured."""
    inps = [synthgen.problem_inputs(w) for w in MEMBERS[:3]]
    probs = [make(w, inp, stream) for w, inp in zip(MEMBERS[:3], inps)]
    cache = str(tmp_path / "tune.txt")
    with bnlat.Batch(probs, tune_cache=cache) as b:
        first = b.tuning()
    assert first["tch"] in (64, 128, 256, 512)
    assert first["slice_target"] in (128, 256, 512, 1024, 2048)
    key = open(cache).read().split()[0]
    with bnlat.Batch(probs, tune_cache=cache) as b:
        assert b.tuning() == first
    fixed = str(tmp_path / "fixed.txt")
    with open(fixed, "w") as f:
        f.write(f"{key} tch=64 slices=2048\n")
    with bnlat.Batch(probs, tune_cache=fixed) as b:
        # a line written before the block shape was a choice: shape 0
        assert b.tuning() == {"tch": 64, "slice_target": 2048, "stage_shape": 0}
        b.sweep(1)
    with open(fixed, "w") as f:
        f.write(f"{key} tch=128 slices=512 shape=1\n")
    with bnlat.Batch(probs, tune_cache=fixed) as b:
        assert b.tuning() == {"tch": 128, "slice_target": 512, "stage_shape": 1}
        b.sweep(2)
    for p in probs:
        p.close()


def test_tune_cache_rejects_foreign_choices(stream, tmp_path):
    """A cache line for the members' key whose chunk is not one of the tuner's
    candidates (100 integrands per counting wave would make the waves' 16-byte
    count tiles overlap) is ignored: the tuner runs again, its valid choice is
    appended and the batched sweep still follows the members' own sweeps."""
    inps = [synthgen.problem_inputs(w) for w in MEMBERS[:3]]
    probs = [make(w, inp, stream) for w, inp in zip(MEMBERS[:3], inps)]
    probe = str(tmp_path / "probe.txt")
    with bnlat.Batch(probs, tune_cache=probe) as b:
        pass
    key = open(probe).read().split()[0]
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write(f"{key} tch=100 slices=2048\n{key} tch=256 slices=7\n{key} tch=256 slices=512 shape=2\n")
    with bnlat.Batch(probs, tune_cache=bad) as b:
        got = b.tuning()
        assert got["tch"] in (64, 128, 256, 512)
        assert got["slice_target"] in (128, 256, 512, 1024, 2048)
        b.sweep(1)
    lines = open(bad).read().splitlines()
    assert len(lines) == 4 and lines[3].startswith(key)
    for w, inp, p in zip(MEMBERS[:3], inps, probs):
        with make(w, inp, stream) as alone:
            alone.sweep(1)
            np.testing.assert_array_equal(p.get_offsets(), alone.get_offsets())
        p.close()


def test_dimension_pair_batch_equals_members_alone(stream):
    """Uneven batch shaped like the padded-sampler workload (tiles 64-256,
    N in {4, 16, 64, 256}, T = 256, 7x7 window): one batched sweep equals
    each member's own sweep, bit for bit."""
    members = synthgen.dimension_pair_batch(count=8)
    inps = [synthgen.problem_inputs(w) for w in members]
    batched = [make(w, inp, stream) for w, inp in zip(members, inps)]
    with bnlat.Batch(batched) as b:
        b.sweep(2)
    for w, inp, p in zip(members, inps, batched):
        say("member", w["problem_id"], w["n"], w["width"])
        with make(w, inp, stream) as alone:
            alone.sweep(2)
            np.testing.assert_array_equal(p.get_offsets(), alone.get_offsets())
        p.close()


def test_batch_validation(stream):
    w = MEMBERS[0]
    inp = synthgen.problem_inputs(w)
    p = make(w, inp, stream)
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Batch([p, p])
    assert e.value.status == bnlat.BN_EINVAL
    q = bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"]), stream=stream.cuda_stream)
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Batch([p, q])
    assert e.value.status == bnlat.BN_ESTATE
    other = bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"]))
    other.init_offsets(inp["offsets"])
    other.compute_errors()
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Batch([p, other])
    assert e.value.status == bnlat.BN_EINVAL
    for x in (p, q, other):
        x.close()


MIXED = [
    workload(n=64, g=(1, 19), width=16, height=16, t_heaviside=40, problem_id=10),
    workload(n=256, g=(1, 79), width=16, height=16, t_heaviside=48, radius=4, precision=1, problem_id=11),
    workload(n=64, g=(1, 19), width=16, height=16, t_heaviside=20, t_gauss=36, problem_id=12),
    workload(n=256, g=(1, 79), width=16, height=16, t_heaviside=40, t_gauss=24, radius=4, precision=1,
             problem_id=13),
    workload(n=16, g=(1, 7), width=16, height=16, t_heaviside=30, move=1, objective=-1, problem_id=14),
    workload(n=16, g=(1, 7), width=32, height=16, t_heaviside=12, problem_id=15),
]


def make_any(w, inp, stream):
    g = bnlat.gaussian_array(inp["gauss"]) if w.get("t_gauss", 0) else None
    p = bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"]), stream=stream.cuda_stream, gaussians=g)
    p.init_offsets(inp["offsets"])
    p.compute_errors()
    return p


def test_mixed_forms_in_one_batch(stream):
    """Members in the BF16 form, with Gaussian rows or with swap moves are
    recorded into the batch's graph beside the grouped FP32 members; every
    member's trajectory and counts equal its own sweeps alone, and so does
    its energy (to FP64 summation order)."""
    inps = [synthgen.problem_inputs(w) for w in MIXED]
    batched = [make_any(w, inp, stream) for w, inp in zip(MIXED, inps)]
    with bnlat.Batch(batched) as b:
        b.sweep(3)
    for w, inp, p in zip(MIXED, inps, batched):
        say("member", w["problem_id"], w.get("precision", 0), w.get("t_gauss", 0), w.get("move", 0))
        with make_any(w, inp, stream) as alone:
            alone.sweep(3)
            np.testing.assert_array_equal(p.get_offsets(), alone.get_offsets())
            np.testing.assert_array_equal(p.get_counts(), alone.get_counts())
            # the Gaussian rows' FP64 energy part is summed with atomics, so
            # its last bits depend on the order
            assert p.energy() == pytest.approx(alone.energy(), rel=1e-12)
            assert p.get_sweep_index() == 3
        p.close()


def test_benchmark_batch_full_size(stream):
    """The benchmark's 32 dimension-pair members (tiles 64^2 to 256^2, N from 4
    to 256, T = 256, 7x7 window) batched with the launch tuner, one sweep: the
    offsets of every 64^2 member equal the oracle's sweep, and the larger
    members equal their own sweeps outside the batch."""
    members = synthgen.dimension_pair_batch()
    inps = [synthgen.problem_inputs(mw) for mw in members]
    probs = [make(mw, mi, stream) for mw, mi in zip(members, inps)]
    try:
        with bnlat.Batch(probs) as b:
            b.sweep(1)
            say("tuning", b.tuning())
        got = [q.get_offsets() for q in probs]
    finally:
        for q in probs:
            q.close()
    for j, (mw, mi) in enumerate(zip(members, inps)):
        if mw["width"] == 64:
            ref = oracle_problem(mw, mi)
            st = osw.run(ref, osw.initial_state(ref, mi["offsets"]), 1)
            np.testing.assert_array_equal(got[j], st.u, err_msg=f"member {j} vs oracle")
        elif j % 4 == 0:
            with make(mw, mi, stream) as alone:
                alone.sweep(1)
                np.testing.assert_array_equal(got[j], alone.get_offsets(), err_msg=f"member {j} vs solo")


def test_batch_of_solo_members_only(stream):
    """A batch whose members all sweep on their own (BF16 form, Gaussian rows,
    swap moves): no grouped launches at all; one sweep, then a graph-replayed
    pair plus one more, each member equal to its own sweeps alone."""
    ws = [MIXED[1], MIXED[2], MIXED[3], MIXED[4]]
    inps = [synthgen.problem_inputs(w) for w in ws]
    batched = [make_any(w, inp, stream) for w, inp in zip(ws, inps)]
    with bnlat.Batch(batched) as b:
        b.sweep(1)
        b.sweep(3)
    for w, inp, p in zip(ws, inps, batched):
        with make_any(w, inp, stream) as alone:
            alone.sweep(4)
            np.testing.assert_array_equal(p.get_offsets(), alone.get_offsets())
            assert p.get_sweep_index() == 4
        p.close()


@pytest.mark.parametrize("k_col,shape", [(1, 0), (1, 1), (4, 0), (4, 1)])
def test_batched_colour_moduli_and_stage_shapes(stream, tmp_path, k_col, shape):
    """Colour moduli 1 and 4 with either stage block shape (forced through the
    tune cache), over a pair graph and an odd sweep: every member equals the
    oracle's trajectory."""
    ws = [workload(n=16, g=(1, 7), width=16, height=16, t_heaviside=40, colour_k=k_col, problem_id=20),
          workload(n=256, g=(1, 79), width=16, height=8, t_heaviside=70, radius=2, colour_k=k_col,
                   problem_id=21),
          workload(n=4, g=(1, 3), width=32, height=16, t_heaviside=30, radius=3, colour_k=k_col, problem_id=22)]
    inps = [synthgen.problem_inputs(w) for w in ws]
    probs = [make(w, inp, stream) for w, inp in zip(ws, inps)]
    probe = str(tmp_path / "probe.txt")
    with bnlat.Batch(probs, tune_cache=probe):
        pass
    key = open(probe).read().split()[0]
    forced = str(tmp_path / "forced.txt")
    with open(forced, "w") as f:
        f.write(f"{key} tch=128 slices=256 shape={shape}\n")
    with bnlat.Batch(probs, tune_cache=forced) as b:
        assert b.tuning()["stage_shape"] == shape
        b.sweep(3)
    for w, inp, p in zip(ws, inps, probs):
        ref = oracle_problem(w, inp)
        st = osw.run(ref, osw.initial_state(ref, inp["offsets"]), 3)
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        p.close()
