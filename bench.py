"""Benchmark: pixel-updates/s of the lattice-offset optimiser sweep.

One step = one sweep of the whole hot path (proposals and their recount for
every pixel, then for every colour class: energy change and commit) over a
256x256 tile with N = 256 samples per pixel, T = 1024 Heaviside integrands
and a 9x9 window.  Inputs are synthetic (seeded) and resident in HBM before
the timed region.

Prints one JSON line.  The timed region runs bn_sweep's overlapped schedule
with HIP events recorded on each launch's own stream (the recount on the
library's auxiliary stream, evaluation and commit on the problem stream);
the graph-replayed rate of the same schedule is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthgen  # noqa: E402

METRIC = "pixel-updates/sec at 256² tile, T=1024, N=256; HBM GB/s vs peak; BF16 vs FP32"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit vector lane-operations per second
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# dense BF16 matrix-core peak (vendor), TFLOP/s
MFMA_BF16_PEAK_TFLOPS = 2500.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tile256_n256_t1024_fp32.md")


COUNT_KERNEL_SOURCES = ("bnlat_dev.h", "device_common.h", "count.hip")


def kernel_digest() -> str:
    """sha256 over the sources the counting kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in COUNT_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2105_12620_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the counting kernel from the committed counter
    summary, or None when the kernels changed since it was taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    if f"counting kernel sources sha256: {kernel_digest()}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("count_kernel_traffic_bytes:"):
            return float(line.split(":")[1])
    return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_POOL = {}


def _pool_init(n, g, table):
    _POOL.update(n=n, g=g, table=table)


def _pool_counts(u):
    from oracle import estimator
    return estimator.hit_counts(_POOL["n"], _POOL["g"], u, _POOL["table"])


def cpu_baseline(w: dict, inp: dict, sweeps: int = 128, row_pixels: int = 128) -> dict:
    """The oracle timed on a band of class-0 pixels (one class row) of the same
    workload: proposals, recount, energy change and commit, repeated over
    ``sweeps`` sweeps, once on one core and once with the recounts of each
    sweep's pixels spread over a pool of worker processes (the class pixels of
    a phase are independent: snapshot semantics).  The window state of the
    band is computed first (not timed).  Runs before the GPU is initialised,
    so the pool's processes are plain forks of a CPU-only process."""
    import multiprocessing as mp
    from oracle import energy, estimator, sweep as osw

    W, H, T, r = w["width"], w["height"], w["t_heaviside"], w["radius"]
    ref = osw.Problem(n=w["n"], g=w["g"], width=W, height=H, radius=r, sigma=w["sigma"],
                      colour_k=w["colour_k"], seed=w["seed"], problem_id=0, table=inp["heaviside"])
    u0 = inp["offsets"].reshape(-1, 2).astype(np.int64)
    c0 = np.zeros((H, W, T), dtype=np.int16)
    rows = [(y + H) % H for y in range(-r, r + 1)]
    for y in rows:
        c0[y] = estimator.hit_counts(w["n"], w["g"], u0[y * W:(y + 1) * W], inp["heaviside"])
    xs = np.arange(0, W, w["colour_k"])[:row_pixels]
    ys = np.zeros_like(xs)

    def run(recount):
        c = c0.copy()
        t0 = time.perf_counter()
        for s in range(sweeps):
            u_new = osw.proposals(ref, ys, xs, s).astype(np.int64)
            c_new = recount(u_new)
            d = energy.weighted_class_sum(energy.delta_class_sums(c, ys, xs, c_new, r), r, w["sigma"])
            acc = d < 0.0
            c[ys[acc], xs[acc]] = c_new[acc]
        return time.perf_counter() - t0, c

    dt1, c1 = run(lambda u: estimator.hit_counts(w["n"], w["g"], u, inp["heaviside"]))
    cores = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(cores, initializer=_pool_init,
                                     initargs=(w["n"], w["g"], inp["heaviside"])) as pool:
        pool.map(_pool_counts, np.array_split(u0[:cores], cores))   # workers up
        dtn, cn = run(lambda u: np.concatenate(pool.map(_pool_counts, np.array_split(u, cores))))
    assert np.array_equal(c1, cn)
    sample = (f"{sweeps} sweeps x {len(xs)} class-0 pixels of one row (recount N*T predicates "
              f"+ exact energy change + commit), numpy FP64/int64 oracle")
    return {"value": sweeps * len(xs) / dt1, "unit": "pixel-updates/s", "cores": 1, "kind": "oracle",
            "sample": sample + ", single thread", "seconds": dt1, "cpu_model": cpu_model(),
            "nproc": os.cpu_count(),
            "all_cores": {"value": sweeps * len(xs) / dtn, "unit": "pixel-updates/s", "cores": cores,
                          "kind": "oracle", "seconds": dtn,
                          "sample": sample + f", recounts spread over {cores} worker processes, "
                                             "energy changes and commits in the parent"}}


SIGMAS_B = [0.25, 0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 20.0]


def quality_experiment(sweeps: int) -> dict:
    """The criterion of Sec. 3.3 (Fig. 1c) and the versatility claim of
    Sec. 3.5 on the GPU path: a 128x128 tile at 16 samples per pixel
    (generator (1, 5), the one of Fig. 1a), optimised on 256 Heavisides with
    each mutation and each direction, then scored by the blurred error of
    held-out integrands (1024 other Heavisides; 1024 Gaussians) against the
    random tile it started from."""
    from paper_2105_12620_amd import bnlat

    w = dict(n=16, g=(1, 5), width=128, height=128, t_heaviside=256, t_gauss=0, sigma=2.1, radius=3,
             colour_k=2, seed=11, problem_id=0)
    train = bnlat.draw_heavisides(11, 0, 256)
    held_h = bnlat.draw_heavisides(12, 0, 1024)
    held_g = bnlat.draw_gaussians(13, 0, 1024)
    u0 = synthgen.offsets(128, 128, seed=14)

    def score(u):
        with bnlat.create_problem(dict(w, t_heaviside=1024), held_h) as q:
            q.init_offsets(u)
            q.compute_errors()
            qh = q.quality_metric(SIGMAS_B)
        with bnlat.create_problem(dict(w, t_heaviside=1, t_gauss=1024), held_h[:1], gaussians=held_g) as q:
            q.init_offsets(u)
            q.compute_errors()
            qg = q.quality_metric(SIGMAS_B, rows=bnlat.BN_ROWS_GAUSSIAN)
        return qh, qg

    base_h, base_g = score(u0)
    out = {"sigmas_b": SIGMAS_B, "sweeps": sweeps,
           "random": {"heaviside": base_h.tolist(), "gaussian": base_g.tolist()}}
    for move, mname in ((bnlat.BN_REDRAW, "redraw"), (bnlat.BN_SWAP, "swap")):
        for objective, oname in ((1, "descend"), (-1, "ascend")):
            with bnlat.create_problem(w, train, move=move, objective=objective) as p:
                p.init_offsets(u0)
                p.compute_errors()
                e0 = p.energy()
                t0 = time.perf_counter()
                st = p.sweep(sweeps, stats=True)
                e1 = p.energy()
                dt = time.perf_counter() - t0
                u = p.get_offsets()
            qh, qg = score(u)
            out[f"{mname}_{oname}"] = {
                "energy_before": e0, "energy_after": e1, "accepts": st["accepts"], "seconds": dt,
                "heaviside": qh.tolist(), "gaussian": qg.tolist(),
                "heaviside_ratio": (qh / base_h).tolist(), "gaussian_ratio": (qg / base_g).tolist()}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="tile256_n256_t1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp32,bf16,swap,batched,large,precision_large",
                    help="comma list of forms to run: fp32 (headline), bf16, swap, batched, large, "
                         "precision_large")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--experiment", choices=["quality"], default=None,
                    help="instead of the benchmark, run the blur-criterion experiment and print its JSON line")
    ap.add_argument("--sweeps", type=int, default=1000, help="sweeps per optimisation in --experiment")
    args = ap.parse_args()
    forms = set(args.forms.split(","))
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the optimiser's batched "
                                   "and multi-tile sharding is not built for several GPUs", "n_gpus": args.gpus}))
        return 2

    w = dict(synthgen.WORKLOADS[args.workload])
    inp = synthgen.problem_inputs(w)
    # the CPU baseline runs first: its worker pool forks a process that has
    # not initialised the GPU
    cpu = None
    if not args.no_cpu_baseline and args.experiment is None:
        cpu = cpu_baseline(w, inp)
        print(f"cpu baseline: {cpu['value']:.1f} pixel-updates/s on 1 core, "
              f"{cpu['all_cores']['value']:.1f} on {cpu['all_cores']['cores']}", file=sys.stderr, flush=True)

    import torch
    from paper_2105_12620_amd import bnlat

    torch.cuda.set_device(0)
    if args.experiment == "quality":
        print(json.dumps(quality_experiment(args.sweeps)), flush=True)
        return 0
    # this GPU's attainable peaks: a 4 GiB device copy, v_dot2 chains, BF16 MFMA chains
    peaks = {"hbm_gbs": bnlat.measure_peak(bnlat.BN_PEAK_HBM_COPY, 4 << 30, 5) / 1e9,
             "valu_tops": bnlat.measure_peak(bnlat.BN_PEAK_VALU_DOT2, 0, 5) / 1e12,
             "mfma_bf16_tflops": bnlat.measure_peak(bnlat.BN_PEAK_MFMA_BF16, 0, 5) / 1e12}
    print(f"measured peaks: {peaks}", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    K2 = w["colour_k"] ** 2
    P, T, N = w["width"] * w["height"], w["t_heaviside"], w["n"]

    def timed_form(precision: int, move: int = 0) -> dict:
        """K sweeps of the overlapped schedule with HIP events around every
        launch (the timed region), then K graph-replayed sweeps."""
        prob = bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"]), stream=stream.cuda_stream,
                                    precision=precision, move=move)
        prob.init_offsets(inp["offsets"])
        prob.compute_errors()
        prob.sweep(args.warmup)
        prob.set_profiling(True)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        prob.sweep(args.steps)
        stop.record(stream)
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        prof = prob.get_profile()
        prob.set_profiling(False)
        prob.sweep(2)
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        prob.sweep(args.steps)
        g1.record(stream)
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1)
        alone_ms = None
        if move == bnlat.BN_REDRAW:
            # the colour-phase evaluation measured alone (no recount beside it):
            # propose class 0 once, then time twenty evaluations of it (one slow
            # evaluation among five once moved the average by half)
            prob.phase_propose(0)
            prob.phase_evaluate(0)
            torch.cuda.synchronize()
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            for _ in range(20):
                prob.phase_evaluate(0)
            a1.record(stream)
            torch.cuda.synchronize()
            alone_ms = a0.elapsed_time(a1) / 20
        energy = prob.energy()
        quality = prob.quality_metric([1.0, 4.0, 16.0]).tolist()
        prob.close()
        kernels = {"recount_per_sweep": prof["recount_ms"] / max(1, prof["recount_launches"]),
                   "evaluate_per_phase": prof["evaluate_ms"] / max(1, prof["phases"]),
                   "commit_per_phase": prof["commit_ms"] / max(1, prof["phases"]),
                   "recount_launches": prof["recount_launches"], "phases": prof["phases"]}
        return {"total_ms": total_ms, "kernels_ms": kernels, "graph_ms": graph_ms, "energy": energy,
                "quality_sigma_1_4_16": quality, "evaluate_alone_ms": alone_ms}

    if args.copy_calibration:
        # a plain copy kernel of known size: 1 GiB read, 1 GiB written
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    fp32 = timed_form(bnlat.BN_FP32)
    bf16 = timed_form(bnlat.BN_BF16) if "bf16" in forms else None
    swap = timed_form(bnlat.BN_FP32, bnlat.BN_SWAP) if "swap" in forms else None
    avg, total_ms = fp32["kernels_ms"], fp32["total_ms"]
    M = P // K2

    def batched() -> dict:
        members = synthgen.dimension_pair_batch()
        probs = []
        for mw in members:
            mi = synthgen.problem_inputs(mw)
            q = bnlat.create_problem(mw, bnlat.heaviside_array(mi["heaviside"]), stream=stream.cuda_stream)
            q.init_offsets(mi["offsets"])
            q.compute_errors()
            probs.append(q)
        b = bnlat.Batch(probs)
        b.sweep(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = max(1, args.steps // 2)
        e0.record(stream)
        b.sweep(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        pix = sum(mw["width"] * mw["height"] for mw in members)
        ops = sum(2.0 * mw["width"] * mw["height"] * mw["n"] * mw["t_heaviside"] for mw in members)
        out = {"value": pix * steps / (ms * 1e-3), "unit": "pixel-updates/s", "members": len(members),
               "count_lane_ops_per_sweep": ops,
               "pixels": pix, "sweeps": steps, "ms_per_sweep": ms / steps, "tuning": b.tuning(),
               "shapes": [f"{mw['width']}^2/N{mw['n']}" for mw in members]}
        b.close()
        for q in probs:
            q.close()
        return out

    batch = batched() if "batched" in forms else None

    def large() -> dict:
        """Four 512x512 problems (N = 1024, 3072 Heavisides + 1024 Gaussians,
        11x11 window) in the BF16 form, batched into one graph."""
        base = dict(synthgen.WORKLOADS["tile512_n1024_t4096"])
        probs = []
        for j in range(4):
            mw = dict(base, problem_id=j)
            mi = synthgen.problem_inputs(mw)
            q = bnlat.create_problem(mw, bnlat.heaviside_array(mi["heaviside"]), stream=stream.cuda_stream,
                                     gaussians=bnlat.gaussian_array(mi["gauss"]), precision=bnlat.BN_BF16)
            q.init_offsets(mi["offsets"])
            q.compute_errors()
            probs.append(q)
        b = bnlat.Batch(probs)
        b.sweep(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = 2
        e0.record(stream)
        b.sweep(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        pix = 4 * base["width"] * base["height"]
        out = {"value": pix * steps / (ms * 1e-3), "unit": "pixel-updates/s", "members": 4,
               "shape": "512^2, N=1024, 3072 Heavisides + 1024 Gaussians, 11x11, BF16",
               "sweeps": steps, "ms_per_sweep": ms / steps}
        b.close()
        for q in probs:
            q.close()
        return out

    big = large() if "large" in forms else None

    def precision_large() -> dict:
        """One 512x512 problem of the largest configuration (N = 1024, 3072
        Heavisides + 1024 Gaussians, 11x11 window) in the FP32 form and in the
        BF16 form's approximate mode from the same start: colour-phase
        evaluation time (event-timed, overlapped schedule), sweep time, the
        BF16 form's vetoes, the energies after the same number of sweeps, and
        the BF16 field's energy against the FP64 energy of the same state."""
        base = dict(synthgen.WORKLOADS["tile512_n1024_t4096"])
        mi = synthgen.problem_inputs(base)
        res = {}
        for name, prec in (("fp32", bnlat.BN_FP32), ("bf16", bnlat.BN_BF16)):
            q = bnlat.create_problem(base, bnlat.heaviside_array(mi["heaviside"]), stream=stream.cuda_stream,
                                     gaussians=bnlat.gaussian_array(mi["gauss"]), precision=prec)
            q.init_offsets(mi["offsets"])
            q.compute_errors()
            e0 = q.energy()
            q.set_profiling(True)
            st = q.sweep(3, stats=True)
            prof = q.get_profile()
            q.set_profiling(False)
            torch.cuda.synchronize()
            e0v, e1v = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0v.record(stream)
            q.sweep(2)
            e1v.record(stream)
            torch.cuda.synchronize()
            res[name] = {"evaluate_ms_per_phase": prof["evaluate_ms"] / max(1, prof["phases"]),
                         "ms_per_sweep": e0v.elapsed_time(e1v) / 2, "energy_start": e0,
                         "energy_after_3_sweeps": None, "accepts_3_sweeps": st["accepts"],
                         "bf16_vetoes_3_sweeps": st["bf16_vetoes"]}
            res[name]["energy_after_5_sweeps"] = q.energy()
            del res[name]["energy_after_3_sweeps"]
            if prec == bnlat.BN_BF16:
                ebf = q.energy_bf16()
                res[name]["bf16_field_energy"] = ebf
                res[name]["bf16_field_energy_rel_gap_vs_fp64"] = abs(ebf - res[name]["energy_after_5_sweeps"]) / \
                    res[name]["energy_after_5_sweeps"]
            res[name]["quality_sigma_1_4_16"] = q.quality_metric([1.0, 4.0, 16.0]).tolist()
            q.close()
        res["energy_rel_diff_bf16_vs_fp32"] = abs(res["bf16"]["energy_after_5_sweeps"] -
                                                  res["fp32"]["energy_after_5_sweeps"]) / \
            res["fp32"]["energy_after_5_sweeps"]
        res["quality_rel_diff_bf16_vs_fp32"] = max(abs(a - b) / b for a, b in zip(res["bf16"]["quality_sigma_1_4_16"],
                                                                                res["fp32"]["quality_sigma_1_4_16"]))
        res["shape"] = "512^2, N=1024, 3072 Heavisides + 1024 Gaussians, 11x11"
        return res

    prec_large = precision_large() if "precision_large" in forms else None

    # Algorithmic work per launch of the counting kernel (one sweep-wide
    # recount): N*T predicates per proposal at two vector lane-operations each
    # (int16 dot product + sign test).  The kernel's own instruction count is
    # 1.75 per predicate (one v_dot2, half a v_perm_b32, a quarter of a
    # v_add3_u32), reported beside it.
    count_ops = 2.0 * P * N * T
    count_tops = count_ops / (avg["recount_per_sweep"] * 1e-3) / 1e12
    win = (2 * w["radius"] + 1) ** 2 - 1
    # evaluation of a phase: the tile's counts once (2 B each) plus the moved
    # pixels' proposal rows, and the decisions
    delta_bytes = 2.0 * T * (P + M) + 9.0 * M
    # a swap pass reads the tile's counts once and every member's partner row
    swap_bytes = 2.0 * T * (P + M)
    # the stencils' arithmetic: one product per (moved pixel, window offset,
    # integrand), two per v_dot2 lane-instruction
    stencil_lane_ops = M * win * T / 2.0

    def roof(bound, achieved, unit, kernel, work):
        vendor = {"hbm": HBM_PEAK_GBS, "alu": VALU_PEAK_TOPS, "mfma": MFMA_BF16_PEAK_TFLOPS}[bound]
        meas = {"hbm": peaks["hbm_gbs"], "alu": peaks["valu_tops"], "mfma": peaks["mfma_bf16_tflops"]}[bound]
        return {"bound": bound, "kernel": kernel, "achieved": achieved, "peak": vendor, "unit": unit,
                "frac": achieved / vendor, "peak_measured": meas, "frac_measured": achieved / meas,
                "work_per_launch": work}

    value = P * args.steps / (total_ms * 1e-3)
    out = {
        "metric": METRIC, "value": value, "unit": "pixel-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i16",
        "data": "synthetic",
        "config": {"workload": args.workload, "tile": f"{w['width']}x{w['height']}", "n": N, "t": T,
                   "window": f"{2 * w['radius'] + 1}x{2 * w['radius'] + 1}", "colour_classes": K2,
                   "precision": "fp32", "mutation": "redraw"},
        "roofline": dict(roof("alu", count_tops, "TOP/s", "k_count<64, 4, 3> (sweep-wide proposal recount)",
                              f"{P} pixels x {N} samples x {T} integrands x 2 lane-ops"),
                         traffic=measured_traffic(),
                         frac_at_instruction_count=0.875 * count_tops / VALU_PEAK_TOPS),
        "measured_peaks": peaks,
        "kernels_ms": avg,
        "evaluate_hbm_gbs": delta_bytes / (avg["evaluate_per_phase"] * 1e-3) / 1e9,
        "evaluate_hbm_frac": delta_bytes / (avg["evaluate_per_phase"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "evaluate_alone": {"ms_per_phase": fp32["evaluate_alone_ms"],
                           "hbm_gbs": delta_bytes / (fp32["evaluate_alone_ms"] * 1e-3) / 1e9,
                           "frac": delta_bytes / (fp32["evaluate_alone_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "roofline": roof("hbm", delta_bytes / (fp32["evaluate_alone_ms"] * 1e-3) / 1e9,
                                            "GB/s", "k_delta_stage + k_delta_finish (one colour phase, alone)",
                                            f"tile counts once + {M} proposal rows, 2 B per integrand"),
                           "roofline_alu": roof("alu", stencil_lane_ops / (fp32["evaluate_alone_ms"] * 1e-3) / 1e12,
                                                "TOP/s", "k_delta_stage + k_delta_finish (one colour phase, alone)",
                                                f"{M} pixels x {win} offsets x {T} integrands / 2 per v_dot2")},
        "graph_value": P * args.steps / (fp32["graph_ms"] * 1e-3),
        "bf16": None if bf16 is None else {
            "value": P * args.steps / (bf16["total_ms"] * 1e-3),
            "graph_value": P * args.steps / (bf16["graph_ms"] * 1e-3),
            "kernels_ms": bf16["kernels_ms"],
            "evaluate_hbm_gbs": delta_bytes / (bf16["kernels_ms"]["evaluate_per_phase"] * 1e-3) / 1e9,
            "evaluate_alone_ms_per_phase": bf16["evaluate_alone_ms"],
            "roofline": roof("hbm", delta_bytes / (bf16["evaluate_alone_ms"] * 1e-3) / 1e9, "GB/s",
                             "BF16 matrix-core energy change of one colour phase, run alone",
                             f"tile counts once + {M} proposal rows, 2 B per integrand"),
            "mfma_useful_tflops": 2.0 * win * T * M / (bf16["evaluate_alone_ms"] * 1e-3) / 1e12,
            "energy_rel_diff_vs_fp32": abs(bf16["energy"] - fp32["energy"]) / abs(fp32["energy"]),
            "quality_rel_diff_vs_fp32": max(abs(a - b) / b for a, b in zip(bf16["quality_sigma_1_4_16"],
                                                                            fp32["quality_sigma_1_4_16"]))},
        "swap": None if swap is None else {
            "mutation": "swap (couples from the XOR-scrambled pixel permutation, no recount)",
            "value": P * args.steps / (swap["total_ms"] * 1e-3),
            "graph_value": P * args.steps / (swap["graph_ms"] * 1e-3),
            "kernels_ms": {"evaluate_per_pass": swap["kernels_ms"]["evaluate_per_phase"],
                           "commit_per_pass": swap["kernels_ms"]["commit_per_phase"],
                           "passes": swap["kernels_ms"]["phases"]},
            "evaluate_hbm_gbs": swap_bytes / (swap["kernels_ms"]["evaluate_per_phase"] * 1e-3) / 1e9,
            "roofline": roof("hbm", swap_bytes / (swap["kernels_ms"]["evaluate_per_phase"] * 1e-3) / 1e9, "GB/s",
                             "k_swap_stage (class sums of one swap pass)",
                             f"tile counts once + {M} partner rows ({T} integrands x 2 B)"),
            "roofline_alu": roof("alu", stencil_lane_ops / (swap["kernels_ms"]["evaluate_per_phase"] * 1e-3) / 1e12,
                                 "TOP/s", "k_swap_stage (class sums of one swap pass)",
                                 f"{M} members x {win} offsets x {T} integrands / 2 per v_dot2")},
        "batched": None if batch is None else dict(batch, roofline=roof(
            "alu", batch["count_lane_ops_per_sweep"] / (batch["ms_per_sweep"] * 1e-3) / 1e12, "TOP/s",
            "whole batched sweep (recounts of every member's proposals over the sweep time)",
            "sum over members of P N T x 2 lane-ops")),
        "batched_large": big,
        "precision_large": prec_large,
        "window_offsets": win,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
