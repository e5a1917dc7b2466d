"""Parity of the gfx950 path (through the C ABI) against the CPU oracle.

Bars: hit counts, lattice points, offsets and trajectories bit-exact; error
vectors within 1e-6 of the larger operand of c/N - A; energy changes and
energies within 1e-12 relative (both sides evaluate the same integer class
sums with the same FP64 weights in the same order); blur criterion within
1e-5 relative (FP32 convolution against FP64)."""
import numpy as np
import pytest

from oracle import energy, estimator, lattice, quality, sweep as osw
import synthgen

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")


from cases import EDGE, check_errors, gpu_problem, oracle_problem, say, workload  # noqa: E402


@pytest.mark.parametrize("name", list(EDGE) + ["tile32_n16_t64", "tile128_n64_t256"])
def test_counts_errors_and_points(name):
    w = EDGE.get(name) or workload(name)
    say("case", name, {k: w[k] for k in ("n", "width", "height", "t_heaviside", "radius", "colour_k")})
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    c_ref = estimator.hit_counts(w["n"], w["g"], inp["offsets"].reshape(-1, 2), inp["heaviside"])
    with gpu_problem(w, inp) as p:
        np.testing.assert_array_equal(p.get_counts(), c_ref)
        check_errors(p.get_errors(), c_ref, w["n"], ref.areas)
        h, a = p.get_integrands()
        np.testing.assert_array_equal(a, ref.areas)
        seq = lattice.sequence_q16(w["n"], w["g"])
        P = w["width"] * w["height"]
        for pix in (0, P // 3, P - 1):
            want = lattice.scramble(seq, inp["offsets"].reshape(-1, 2)[pix].astype(np.int64))
            np.testing.assert_array_equal(p.get_points(pix), want)


def test_philox_offsets_match_oracle():
    w = workload(width=40, height=24, colour_k=2, seed=123456789012, problem_id=5)
    inp = synthgen.problem_inputs(w)
    with bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"])) as p:
        p.init_offsets(None)
        np.testing.assert_array_equal(p.get_offsets(), osw.philox_offsets(oracle_problem(w, inp)))


def test_drawn_integrands_used_when_none_given():
    w = workload(t_heaviside=33, seed=9)
    with bnlat.create_problem(w, None) as p:
        h, _ = p.get_integrands()
    np.testing.assert_array_equal(h, bnlat.draw_heavisides(9, 0, 33))


@pytest.mark.parametrize("name", ["n4_ragged", "n256_r4", "tile4_alias", "k4_conflict_free",
                                  "rect_ascend", "n1024_r5", "tile32_n16_t64", "r6", "n4096",
                                  "k4_r6", "wide64", "k1"])
def test_phase_steps_match_oracle(name):
    """Every step of two sweeps' phases: proposals, recounts, energy changes,
    decisions and the committed state."""
    w = EDGE.get(name) or workload(name)
    say("case", name)
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    with gpu_problem(w, inp) as p:
        for s in range(2):
            for kappa in range(w["colour_k"] ** 2):
                p.phase_propose(kappa)
                p.phase_evaluate(kappa)
                got = p.get_phase()
                ph = osw.phase(ref, st, kappa)
                np.testing.assert_array_equal(got["u_new"], ph["u_new"])
                np.testing.assert_array_equal(got["c_new"], ph["c_new"])
                np.testing.assert_allclose(got["delta"], ph["delta"], rtol=1e-12, atol=0)
                np.testing.assert_array_equal(got["accept"], ph["accept"])
                p.phase_commit(kappa)
            p.phase_advance()
            st.sweep += 1
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        np.testing.assert_array_equal(p.get_counts(), st.c.reshape(-1, w["t_heaviside"]))
        assert p.get_sweep_index() == 2


@pytest.mark.parametrize("name,k", [("tile32_n16_t64", 100), ("tile128_n64_t256", 2),
                                    ("n256_r4", 4), ("k1", 3), ("rect_ascend", 5)])
def test_sweep_trajectory_matches_oracle(name, k):
    """bn_sweep (graph-replayed) gives the oracle's trajectory bit for bit,
    and the same energy and blur criterion."""
    w = EDGE.get(name) or workload(name)
    say("case", name, "sweeps", k)
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.run(ref, osw.initial_state(ref, inp["offsets"]), k)
    with gpu_problem(w, inp) as p:
        stats = p.sweep(k, stats=True)
        assert stats["sweep_index"] == k
        assert stats["accepts"] == sum(st.accepts)
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        np.testing.assert_array_equal(p.get_counts(), st.c.reshape(-1, w["t_heaviside"]))
        check_errors(p.get_errors(), st.c.reshape(-1, w["t_heaviside"]), w["n"], ref.areas)
        e_ref = osw.energy_of(ref, st)
        assert p.energy() == pytest.approx(e_ref, rel=1e-12)
        assert p.energy() == pytest.approx(energy.energy_plain(osw.errors(ref, st), w["radius"], w["sigma"]),
                                           rel=1e-9)
        sig = (0.25, 1.0, 4.0, 20.0)
        np.testing.assert_allclose(p.quality_metric(sig), quality.quality(osw.errors(ref, st), sig),
                                   rtol=1e-5)


def test_delta_energy_list_matches_oracle():
    w = EDGE["n256_r4"]
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    P = w["width"] * w["height"]
    pix = synthgen.pixel_sample(P, 40, seed=1)
    prop = synthgen.proposals(40, seed=2)
    ys, xs = np.divmod(pix.astype(np.int64), w["width"])
    c_new = estimator.hit_counts(w["n"], w["g"], prop.astype(np.int64), inp["heaviside"])
    want = energy.delta_exact(st.c, ys, xs, c_new, w["n"], w["radius"], w["sigma"])
    e = osw.errors(ref, st)
    with gpu_problem(w, inp) as p:
        de, cn = p.delta_energy(pix, prop, counts=True)
    np.testing.assert_array_equal(cn, c_new)
    np.testing.assert_allclose(de, want, rtol=1e-12, atol=0)
    for j in range(len(pix)):
        plain = energy.delta_plain(e, ys[j], xs[j], c_new[j] / w["n"] - ref.areas, w["radius"], w["sigma"])
        scale = abs(plain) + 1e-3
        assert abs(de[j] - plain) <= 1e-5 * scale


def test_full_size_tile256_sampled():
    """256x256 tile, N=256, T=1024, 9x9 window in the benchmark's launch
    configuration: sampled pixels' hit counts after bn_compute_errors, and the
    first phase's proposals, recounts, energy changes and decisions for
    sampled class pixels, each computed by the oracle from the inputs."""
    w = workload("tile256_n256_t1024")
    inp = synthgen.problem_inputs(w)
    W, H, T, r = w["width"], w["height"], w["t_heaviside"], w["radius"]
    u0 = inp["offsets"].reshape(-1, 2).astype(np.int64)
    ref = oracle_problem(w, inp)
    with gpu_problem(w, inp) as p:
        c_gpu = p.get_counts()
        e_gpu = p.get_errors()
        p.phase_propose(0)
        p.phase_evaluate(0)
        ph = p.get_phase()
    sample = synthgen.pixel_sample(W * H, 48, seed=3)
    c_ref = estimator.hit_counts(w["n"], w["g"], u0[sample], inp["heaviside"])
    np.testing.assert_array_equal(c_gpu[sample], c_ref)
    check_errors(e_gpu[sample], c_ref, w["n"], ref.areas)
    # first phase, class 0: class pixel j sits at (2a, 2b), j = a * W/2 + b
    js = synthgen.pixel_sample((W // 2) * (H // 2), 6, seed=4)
    for j in js:
        y, x = 2 * (int(j) // (W // 2)), 2 * (int(j) % (W // 2))
        win = [((y + oy) % H, (x + ox) % W) for oy in range(-r, r + 1) for ox in range(-r, r + 1)]
        ids = np.array([yy * W + xx for yy, xx in win])
        local = np.zeros((H, W, T), dtype=np.int16)
        local[tuple(np.array(win).T)] = estimator.hit_counts(w["n"], w["g"], u0[ids], inp["heaviside"])
        u_new = osw.proposals(ref, np.array([y]), np.array([x]), 0).astype(np.int64)
        c_new = estimator.hit_counts(w["n"], w["g"], u_new, inp["heaviside"])
        np.testing.assert_array_equal(ph["u_new"][j], u_new[0])
        np.testing.assert_array_equal(ph["c_new"][j], c_new[0])
        d = energy.delta_exact(local, [y], [x], c_new, w["n"], r, w["sigma"])
        assert ph["delta"][j] == pytest.approx(d[0], rel=1e-12)
        assert bool(ph["accept"][j]) == bool(d[0] < 0)


def test_full_size_tile256_sweeps_sampled():
    """The benchmark's own schedule at full size (256x256, N=256, T=1024, two
    graph-replayed overlapped sweeps with the capped sweep-wide recount):
    every sampled pixel's offset is its initial one or the oracle's proposal
    for one of the two sweeps, its counts are the oracle's estimator at that
    offset, the energy fell, and the energy and the blur criterion equal the
    oracle's from all exported counts (Eq. (1) in exact integers per distance
    class, summed over 128-integrand slices; Q at sigma_b = 4)."""
    w = workload("tile256_n256_t1024")
    inp = synthgen.problem_inputs(w)
    W = w["width"]
    ref = oracle_problem(w, inp)
    u0 = inp["offsets"].reshape(-1, 2).astype(np.int64)
    with gpu_problem(w, inp) as p:
        e0 = p.energy()
        p.sweep(2)
        u = p.get_offsets().reshape(-1, 2).astype(np.int64)
        c = p.get_counts()
        e2 = p.energy()
        q2 = p.quality_metric([4.0])
    assert e2 < e0
    moved = np.any(u != u0, axis=1)
    assert 0.01 < moved.mean() < 0.99
    sample = synthgen.pixel_sample(W * w["height"], 64, seed=5)
    ys, xs = sample // W, sample % W
    props = [osw.proposals(ref, ys, xs, s).astype(np.int64) for s in (0, 1)]
    for i, q in enumerate(sample):
        assert (np.array_equal(u[q], u0[q]) or np.array_equal(u[q], props[0][i])
                or np.array_equal(u[q], props[1][i])), q
    np.testing.assert_array_equal(c[sample], estimator.hit_counts(w["n"], w["g"], u[sample], inp["heaviside"]))
    c3 = c.reshape(w["height"], W, -1)
    xd = sum(energy.energy_class_sums(c3[:, :, t:t + 128], w["radius"]) for t in range(0, c3.shape[2], 128))
    e_ref = float(energy.weighted_class_sum(xd, w["radius"], w["sigma"])) / (w["n"] * w["n"])
    assert e2 == pytest.approx(e_ref, rel=1e-12)
    # the blur criterion at sigma_b = 4 from the same counts
    np.testing.assert_allclose(q2, quality.quality(estimator.errors_from_counts(c3, w["n"], ref.areas), [4.0]),
                               rtol=1e-5)


def test_rerun_and_resume_are_bit_identical():
    w = EDGE["n256_r4"]
    inp = synthgen.problem_inputs(w)
    with gpu_problem(w, inp) as a:
        a.sweep(3)
        ua = a.get_offsets()
    with gpu_problem(w, inp) as b:
        b.sweep(3)
        np.testing.assert_array_equal(b.get_offsets(), ua)
    with gpu_problem(w, inp) as c:
        c.sweep(1)
        mid = c.get_offsets()
    with bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"])) as d:
        d.init_offsets(mid)
        d.compute_errors()
        d.set_sweep_index(1)
        d.sweep(2)
        np.testing.assert_array_equal(d.get_offsets(), ua)


def test_call_order_is_enforced():
    w = EDGE["n4_ragged"]
    inp = synthgen.problem_inputs(w)
    with bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"])) as p:
        with pytest.raises(bnlat.BnlatError) as e:
            p.compute_errors()
        assert e.value.status == bnlat.BN_ESTATE
        p.init_offsets(inp["offsets"])
        with pytest.raises(bnlat.BnlatError) as e:
            p.sweep(1)
        assert e.value.status == bnlat.BN_ESTATE
        p.compute_errors()
        with pytest.raises(bnlat.BnlatError) as e:
            p.get_points(w["width"] * w["height"])
        assert e.value.status == bnlat.BN_EINVAL
        with pytest.raises(bnlat.BnlatError) as e:
            p.phase_propose(4)
        assert e.value.status == bnlat.BN_EINVAL


def test_profiled_and_mixed_schedules_agree():
    """bn_sweep with kernel profiling (eager overlapped launches) gives the
    graph-replayed trajectory; mixing phase steps and bn_sweep keeps the
    proposal prefetch consistent with the sweep index."""
    w = EDGE["n256_r4"]
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.run(ref, osw.initial_state(ref, inp["offsets"]), 5)
    with gpu_problem(w, inp) as p:
        p.set_profiling(True)
        p.sweep(3)
        prof = p.get_profile()
        assert prof["recount_launches"] >= 3 and prof["phases"] == 12
        assert prof["recount_ms"] > 0 and prof["evaluate_ms"] > 0
        p.set_profiling(False)
        for kappa in range(4):
            p.phase_propose(kappa)
            p.phase_evaluate(kappa)
            p.phase_commit(kappa)
        p.phase_advance()
        p.sweep(1)
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        assert p.get_sweep_index() == 5


@pytest.mark.parametrize("precision", [0, 1])
def test_profiled_pairs_chain_recounts(precision):
    """Three eager overlapped pairs in one call (kernel profiling on): every
    recount reads the recount index, and the first recount of the second and
    third pairs waits only for the previous pair's last phases.  The offsets
    and counts equal the oracle's after the six sweeps, and a graph-replayed
    call (the index set again from the sweep counter) continues the oracle's
    trajectory."""
    w = dict(EDGE["n256_r4"], precision=precision)
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    osw.run(ref, st, 6)
    u6, c6 = st.u.copy(), st.c.reshape(-1, w["t_heaviside"]).copy()
    osw.run(ref, st, 4)
    with gpu_problem(w, inp) as p:
        p.set_profiling(True)
        p.sweep(6)
        prof = p.get_profile()
        assert prof["recount_launches"] >= 6 and prof["phases"] == 24
        p.set_profiling(False)
        np.testing.assert_array_equal(p.get_offsets(), u6)
        np.testing.assert_array_equal(p.get_counts(), c6)
        p.sweep(4)
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        np.testing.assert_array_equal(p.get_counts(), st.c.reshape(-1, w["t_heaviside"]))
        assert p.get_sweep_index() == 10


@pytest.mark.parametrize("precision", [0, 1])
def test_recount_cap_does_not_change_results(precision):
    """The sweep-wide recount with a workgroup cap (workgroups striding over
    the work) gives the oracle's trajectory for any cap, before and after the
    captured graph is rebuilt."""
    w = dict(EDGE["n256_r4"], precision=precision)
    inp = synthgen.problem_inputs(w)
    ref = oracle_problem(w, inp)
    st = osw.run(ref, osw.initial_state(ref, inp["offsets"]), 6)
    with gpu_problem(w, inp) as p:
        p.set_recount_blocks(3)
        p.sweep(2)
        p.set_recount_blocks(0)
        p.sweep(2)
        p.set_recount_blocks(7)
        p.sweep(2)
        np.testing.assert_array_equal(p.get_offsets(), st.u)
        np.testing.assert_array_equal(p.get_counts().reshape(st.c.shape), st.c)


def _local_sweep_decisions(w, ref, heav, u_start, sweep, cy, cx, half):
    """Decisions of one sweep on the square patch of side 2*half centred at
    (cy, cx) (wrapped on the torus), simulated by the oracle from the offsets
    u_start at the sweep's start: phase by phase, a class pixel is evaluated
    (exact integer energy change against the phase-start state) only when its
    whole window has a known state; the pixels it could not evaluate become
    unknown for later phases.  Returns {pixel index: accepted}."""
    W, H, T, r, K = w["width"], w["height"], w["t_heaviside"], w["radius"], w["colour_k"]
    ys = (cy + np.arange(-half, half)) % H
    xs = (cx + np.arange(-half, half)) % W
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    gy, gx = gy.ravel(), gx.ravel()
    ids = gy * W + gx
    c = np.zeros((H, W, T), dtype=np.int16)
    c[gy, gx] = estimator.hit_counts(w["n"], w["g"], u_start[ids], heav)
    known = np.zeros((H, W), dtype=bool)
    known[gy, gx] = True
    decided = {}
    for kappa in range(K * K):
        sel = (gy % K) * K + (gx % K) == kappa
        py, px = gy[sel], gx[sel]
        ok = np.ones(py.shape[0], dtype=bool)
        for oy in range(-r, r + 1):
            for ox in range(-r, r + 1):
                ok &= known[(py + oy) % H, (px + ox) % W]
        ey, ex = py[ok], px[ok]
        known[py[~ok], px[~ok]] = False
        if ey.size == 0:
            continue
        u_new = osw.proposals(ref, ey, ex, sweep).astype(np.int64)
        c_new = estimator.hit_counts(w["n"], w["g"], u_new, heav)
        d = energy.delta_exact(c, ey, ex, c_new, w["n"], r, w["sigma"])
        acc = d < 0.0
        c[ey[acc], ex[acc]] = c_new[acc]
        for yy, xx, a in zip(ey, ex, acc):
            decided[int(yy) * W + int(xx)] = bool(a)
    return decided


def test_full_size_tile256_graph_sweep_decisions():
    """Decisions of the benchmark's own schedule at full size (256x256, N=256,
    T=1024, 9x9 window): two sweeps by one replay of the captured pair graph
    (overlapped sweep-wide recount with its workgroup cap, raised-priority
    colour phases), the state exported, then two more graph-replayed sweeps.
    The oracle simulates the third sweep (index 2) exactly on a 48x48 patch
    across the tile's corner (torus wrap) from the exported offsets, and every
    class pixel of every phase whose window state it knows must have the
    GPU's decision; a pixel's GPU decision in that sweep is read from its
    final offset whenever that offset is its start offset (rejected) or the
    sweep's proposal (accepted)."""
    w = workload("tile256_n256_t1024")
    inp = synthgen.problem_inputs(w)
    W, H = w["width"], w["height"]
    ref = oracle_problem(w, inp)
    with gpu_problem(w, inp) as p:
        p.sweep(2)
        assert p.get_sweep_index() == 2
        u2 = p.get_offsets().reshape(-1, 2).astype(np.int64)
        c2 = p.get_counts()
        p.sweep(2)
        u4 = p.get_offsets().reshape(-1, 2).astype(np.int64)
    say("exported state after two graph-replayed sweeps; simulating sweep 2 on a 48x48 patch")
    decided = _local_sweep_decisions(w, ref, inp["heaviside"], u2, 2, 0, 0, 24)
    pix = np.array(sorted(decided), dtype=np.int64)
    np.testing.assert_array_equal(c2[pix], estimator.hit_counts(w["n"], w["g"], u2[pix], inp["heaviside"]))
    ys, xs = pix // W, pix % W
    p2 = osw.proposals(ref, ys, xs, 2).astype(np.int64)
    p3 = osw.proposals(ref, ys, xs, 3).astype(np.int64)
    checked = {k: 0 for k in range(4)}
    accepts = 0
    for i, q in enumerate(pix):
        if np.array_equal(u4[q], u2[q]):
            gpu = False
        elif np.array_equal(u4[q], p2[i]):
            gpu = True
        else:
            assert np.array_equal(u4[q], p3[i]), q   # accepted in sweep 3: sweep 2 undetermined
            continue
        assert gpu == decided[int(q)], (int(q), gpu)
        checked[int((ys[i] % 2) * 2 + xs[i] % 2)] += 1
        accepts += gpu
    say("decisions checked per class", checked, "accepted", accepts)
    assert min(checked.values()) >= 20 and 0 < accepts < sum(checked.values())
