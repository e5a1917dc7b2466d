"""Workloads and helpers shared by the GPU parity tests."""
import numpy as np

from oracle import sweep as osw
import synthgen


def say(*a):
    print(*a, flush=True)


def workload(name=None, **kw):
    w = dict(synthgen.WORKLOADS[name]) if name else dict(
        n=16, g=(1, 7), width=16, height=16, t_heaviside=12, t_gauss=0, sigma=2.1, radius=3,
        colour_k=2, sweeps=3, seed=7, problem_id=0)
    w.update(kw)
    return w


EDGE = {
    "n1": workload(n=1, g=(1, 1), t_heaviside=5),
    "n2": workload(n=2, g=(1, 1), t_heaviside=33),
    "n4_ragged": workload(n=4, g=(1, 3), t_heaviside=70),
    "n8": workload(n=8, g=(1, 3), t_heaviside=70, radius=2),
    "n32": workload(n=32, g=(1, 13), t_heaviside=40),
    "n128": workload(n=128, g=(1, 45), t_heaviside=130, width=8, height=8, radius=2),
    "n256_r4": workload(n=256, g=(1, 79), t_heaviside=200, width=12, height=12, radius=4),
    "n512": workload(n=512, g=(3, 101), t_heaviside=64, width=8, height=8, radius=3),
    "n1024_r5": workload(n=1024, g=(1, 381), t_heaviside=66, width=12, height=12, radius=5),
    "n2048": workload(n=2048, g=(1, 763), t_heaviside=65, width=8, height=8, radius=2),
    "tile4_alias": workload(width=4, height=4, radius=3, t_heaviside=9),
    "k1": workload(colour_k=1, width=8, height=8, radius=2),
    "k4_conflict_free": workload(colour_k=4, width=16, height=16, radius=3),
    "rect_ascend": workload(width=12, height=8, radius=3, objective=-1),
    "r6": workload(width=16, height=16, radius=6, n=64, g=(1, 19), t_heaviside=20),
    "n4096": workload(n=4096, g=(1, 1365), t_heaviside=40, width=8, height=8, radius=2),
    "k4_r6": workload(colour_k=4, width=16, height=16, radius=6, t_heaviside=150),
    "wide64": workload(width=64, height=32, radius=4, n=64, g=(1, 19), t_heaviside=140),
}


def oracle_problem(w, inp):
    return osw.Problem(n=w["n"], g=w["g"], width=w["width"], height=w["height"], radius=w["radius"],
                       sigma=w["sigma"], colour_k=w["colour_k"], seed=w["seed"],
                       problem_id=w.get("problem_id", 0), table=inp["heaviside"],
                       objective=w.get("objective", 1),
                       gauss=inp["gauss"] if w.get("t_gauss", 0) else None)


def gpu_problem(w, inp):
    b = _bnlat()
    g = b.gaussian_array(inp["gauss"]) if w.get("t_gauss", 0) else None
    p = b.create_problem(w, b.heaviside_array(inp["heaviside"]), gaussians=g)
    p.init_offsets(inp["offsets"])
    p.compute_errors()
    return p


def check_errors(err32, counts, n, areas):
    e64 = counts / n - areas
    scale = np.maximum(np.maximum(np.abs(e64), areas), counts / n)
    assert np.all(np.abs(err32.astype(np.float64) - e64) <= 1e-6 * scale + 1e-30)




def _bnlat():
    from paper_2105_12620_amd import bnlat
    return bnlat
