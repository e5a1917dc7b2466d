"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws the *inputs* of the lattice-offset optimisation and holds
none of the method's arithmetic: no sample generation, no hit counting, no
integrals, no energies.  Both the CPU oracle and the HIP library consume what
it returns; neither imports the other.

Workload shapes follow the paper's setting: per-pixel scrambled rank-1
lattices (Sec. 3.2), random Heaviside test integrands (Sec. 2, the test
integrand map beside Eq. (1)), a Gaussian-windowed screen-space energy
(Eq. (1), kernel width 2.1 pixels) and, for the low-frequency study of
Sec. 3.5, isotropic Gaussian integrands.

Input formats
-------------
* Offsets ``U``: ``uint16 [H, W, 2]``; the value ``u`` stands for ``u / 2**16``
  (Q0.16 fixed point), component 0 is x, component 1 is y.
* Heaviside table: dict of equal-length arrays ``nx, ny`` (int16, the edge
  normal scaled to length ~2**14 and rounded to the nearest integer, ties to
  even) and ``cx, cy`` (uint16, a Q0.16 point on the edge).  The integrand is
  ``f(x) = 1`` where ``n . (x - c) > 0`` and ``0`` elsewhere (edge excluded).
* Gaussian table: dict of float64 arrays ``mx, my`` (centre) and ``s`` (std).
"""
from __future__ import annotations

import numpy as np

Q16 = 1 << 16
NORMAL_SCALE = 1 << 14


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """Independent numpy generator per (seed, stream)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def heaviside_table(t: int, seed: int, stream: int = 1) -> dict:
    """``t`` random Heavisides: orientation uniform in [0, 2pi), edge through a
    point uniform in the unit square (stored in Q0.16)."""
    g = rng(seed, stream)
    theta = g.uniform(0.0, 2.0 * np.pi, size=t)
    nx = np.rint(NORMAL_SCALE * np.cos(theta)).astype(np.int16)
    ny = np.rint(NORMAL_SCALE * np.sin(theta)).astype(np.int16)
    cx = g.integers(0, Q16, size=t, dtype=np.uint16)
    cy = g.integers(0, Q16, size=t, dtype=np.uint16)
    return {"nx": nx, "ny": ny, "cx": cx, "cy": cy}


def gaussian_table(t: int, seed: int, stream: int = 2) -> dict:
    """``t`` isotropic Gaussians: centre uniform in the unit square, standard
    deviation uniform in [0.05, 0.3]."""
    g = rng(seed, stream)
    return {
        "mx": g.uniform(0.0, 1.0, size=t),
        "my": g.uniform(0.0, 1.0, size=t),
        "s": g.uniform(0.05, 0.3, size=t),
    }


def offsets(width: int, height: int, seed: int, stream: int = 3) -> np.ndarray:
    """Uniform Q0.16 offsets, ``uint16 [H, W, 2]``."""
    return rng(seed, stream).integers(0, Q16, size=(height, width, 2), dtype=np.uint16)


def proposals(m: int, seed: int, stream: int = 4) -> np.ndarray:
    """``m`` uniform Q0.16 candidate offsets, ``uint16 [m, 2]``."""
    return rng(seed, stream).integers(0, Q16, size=(m, 2), dtype=np.uint16)


def pixel_sample(npix: int, m: int, seed: int, stream: int = 5) -> np.ndarray:
    """``m`` distinct pixel indices drawn from ``range(npix)`` (sorted)."""
    m = min(m, npix)
    return np.sort(rng(seed, stream).choice(npix, size=m, replace=False)).astype(np.uint32)


# ---------------------------------------------------------------------------
# Workloads.  Each entry is a plain description of one optimisation problem.
# ---------------------------------------------------------------------------

def _problem(n, g, w, h, th, tg, r, sweeps, seed, k=2, sigma=2.1, problem_id=0):
    return {"n": n, "g": tuple(int(v) for v in g), "width": w, "height": h,
            "t_heaviside": th, "t_gauss": tg, "sigma": sigma, "radius": r,
            "colour_k": k, "sweeps": sweeps, "seed": seed, "problem_id": problem_id}


WORKLOADS = {
    # small case: 32x32 tile, 16 spp, 64 Heavisides, 7x7 window, 100 sweeps
    "tile32_n16_t64": _problem(16, (1, 7), 32, 32, 64, 0, 3, 100, 0),
    # 128x128 tile, 64 spp, 256 Heavisides, 7x7 window, 1000 sweeps
    "tile128_n64_t256": _problem(64, (1, 19), 128, 128, 256, 0, 3, 1000, 1),
    # 256x256 tile, 256 spp, 1024 Heavisides, 9x9 window, 2000 sweeps
    "tile256_n256_t1024": _problem(256, (1, 79), 256, 256, 1024, 0, 4, 2000, 2),
    # 512x512 tile, 1024 spp, 3072 Heavisides + 1024 Gaussians, 11x11 window
    "tile512_n1024_t4096": _problem(1024, (1, 381), 512, 512, 3072, 1024, 5, 5000, 4),
}


def dimension_pair_batch(count: int = 32, seed: int = 3, t: int = 256, radius: int = 3,
                         sweeps: int = 1000) -> list:
    """Independent problems, one per 2D dimension pair of a ``2*count``-D rank-1
    lattice (Sec. 3.1 pads higher dimensions with pairs of 2D tiles).

    One odd generator of ``2*count`` components is drawn in [1, 2**16); member j
    uses components (2j, 2j+1) reduced mod its own N (odd stays odd, hence
    coprime to any power of two).  Tile side is drawn from {64, 128, 256} and
    the sample count from {4, 16, 64, 256}.
    """
    g = rng(seed, 6)
    gen = 2 * g.integers(0, Q16 // 2, size=2 * count) + 1
    sides = g.choice([64, 128, 256], size=count)
    spp = g.choice([4, 16, 64, 256], size=count)
    out = []
    for j in range(count):
        n = int(spp[j])
        gx, gy = int(gen[2 * j]) % n, int(gen[2 * j + 1]) % n
        out.append(_problem(n, (gx, gy), int(sides[j]), int(sides[j]), t, 0, radius, sweeps,
                            seed, problem_id=j))
    return out


def problem_inputs(cfg: dict) -> dict:
    """Integrand tables and initial offsets of one workload entry."""
    s = cfg["seed"] * 1000 + cfg.get("problem_id", 0)
    return {
        "heaviside": heaviside_table(cfg["t_heaviside"], s),
        "gauss": gaussian_table(cfg["t_gauss"], s),
        "offsets": offsets(cfg["width"], cfg["height"], s),
    }
