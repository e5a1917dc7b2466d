"""Parallel propose / evaluate / accept sweeps over colour classes of pixels.

Sec. 3.4 parallelises the optimiser by mutating many pixels at once, keeping
the mutated sets disjoint, evaluating the unmodified cost for each candidate
and accepting improving moves as the sequential optimiser would; roughly a
quarter of the pixels move concurrently.  Readings used here:
  * mutation: the pixel's offset is redrawn from a counter-based Philox
    stream at counter (p, sweep, problem, S_PROP), and its hit counts are
    recomputed;
  * disjoint sets: colour classes kappa = (y mod K) K + (x mod K), visited in
    increasing kappa; K = 2 gives four classes (a quarter of the pixels each);
  * snapshot semantics: every pixel of a class is evaluated against the
    state at the start of its phase, then all accepted moves are committed;
  * accept iff the energy change is strictly negative (no temperature).
    Sec. 2 says the loss of Eq. (1) is reduced, yet lowering that sum makes
    neighbouring error vectors alike, which moves error energy to low
    frequencies, against the blue-noise goal of Sec. 3.3 and Fig. 1c.  The
    default follows the text (descend); ``objective = -1`` accepts moves that
    raise the sum instead (ascend), the only sign under which swapping pixels
    lowers the blurred error.

The paper's own mutation (Sec. 3.4, and the pixel permutation of Sec. 2)
exchanges the offsets of two pixels; ``move = 1`` selects it.  Readings:
  * the precomputed permutation pi lists the pixels sorted by 64-bit Philox
    keys drawn at counters (p, 0, problem, S_PERM) (ties by pixel index);
  * pass kappa of sweep s scrambles the listed indices with the XOR mask
    x = word 0 of Philox((kappa, s, problem, S_SWAP)) mod P (P a power of two,
    so the scrambled list is again a permutation);
  * pass kappa takes list positions [kappa M, (kappa + 1) M), M = P / K^2
    (K = 2: a quarter of the pixels), and couples positions 2i and 2i + 1;
  * each couple is evaluated on the pass-start state (the two exchanged
    vectors plus the pair correction, energy module) and accepted by the same
    strict sign rule; accepted couples exchange offsets, counts and
    estimates, so no recount happens.

Decisions use the exact integer form of the energy change for Heaviside rows
(energy module); Gaussian rows (Sec. 3.5's low-frequency integrands) add their
FP64 plain-form change, and the decision is taken on the sum.

Test infrastructure: this file is part of the CPU oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import energy, estimator, integrands, philox


@dataclass
class Problem:
    n: int
    g: tuple
    width: int
    height: int
    radius: int
    sigma: float
    colour_k: int
    seed: int
    problem_id: int
    table: dict                       # Heaviside table (synthgen format)
    objective: int = 1                # +1: accept dE < 0 (descend); -1: accept dE > 0
    gauss: dict | None = None         # Gaussian table (synthgen format), optional
    move: int = 0                     # 0: redraw offsets; 1: swap couples of pixels

    def __post_init__(self):
        validate(self)
        self.perm = swap_permutation(self) if self.move == 1 else None
        self.areas = integrands.heaviside_areas(self.table)
        tg = 0 if self.gauss is None else len(self.gauss["mx"])
        self.gauss_integrals = (integrands.gaussian_integrals(self.gauss) if tg
                                else np.zeros(0, dtype=np.float64))


def validate(p) -> None:
    """Configuration checks (the library applies the same rules)."""
    m = int(p.n).bit_length() - 1
    if p.n < 1 or (1 << m) != p.n or m > 15:
        raise ValueError("N must be a power of two in [1, 2**15]")
    if any(int(v) % 2 == 0 for v in p.g) and p.n > 1:
        raise ValueError("generator components must be odd (coprime to N)")
    if p.colour_k < 1 or p.width % p.colour_k or p.height % p.colour_k:
        raise ValueError("K must divide the tile width and height")
    if p.radius < 1 or p.radius >= min(p.width, p.height):
        raise ValueError("window radius must satisfy 1 <= r < min(W, H)")
    if getattr(p, "objective", 1) not in (1, -1):
        raise ValueError("objective must be +1 (descend) or -1 (ascend)")
    if len(p.table["nx"]) < 1:
        raise ValueError("at least one integrand is required")
    if getattr(p, "move", 0) not in (0, 1):
        raise ValueError("move must be 0 (redraw) or 1 (swap)")
    if getattr(p, "move", 0) == 1:
        npix = p.width * p.height
        if npix & (npix - 1) or npix < 2 * p.colour_k ** 2:
            raise ValueError("swap mutation: W*H must be a power of two and at least 2 K^2")
        if p.gauss is not None and len(p.gauss["mx"]):
            raise ValueError("swap mutation: Heaviside integrands only")


@dataclass
class State:
    u: np.ndarray            # int64 [H, W, 2]  (Q0.16 offsets)
    c: np.ndarray            # int64 [H, W, T]  (hit counts)
    g: np.ndarray | None = None   # float64 [H, W, T_G] Gaussian estimates
    sweep: int = 0
    accepts: list = field(default_factory=list)   # per phase


def initial_state(prob: Problem, u0: np.ndarray) -> State:
    u = np.asarray(u0, dtype=np.int64).reshape(prob.height, prob.width, 2).copy()
    c = estimator.hit_counts(prob.n, prob.g, u.reshape(-1, 2), prob.table)
    g = None
    if prob.gauss is not None and len(prob.gauss["mx"]):
        g = estimator.gauss_estimates(prob.n, prob.g, u.reshape(-1, 2), prob.gauss).reshape(
            prob.height, prob.width, -1)
    return State(u=u, c=c.reshape(prob.height, prob.width, -1), g=g)


def philox_offsets(prob: Problem) -> np.ndarray:
    """Initial offsets from the counter stream S_INIT at counters (p, 0, problem, S_INIT)."""
    w = philox.draw(np.arange(prob.width * prob.height), 0, prob.problem_id, philox.S_INIT, prob.seed)
    return philox.q16_pair(w).reshape(prob.height, prob.width, 2)


def class_pixels(width: int, height: int, k: int, kappa: int):
    """(ys, xs) of colour class kappa in raster order."""
    ys, xs = np.divmod(np.arange(width * height, dtype=np.int64), width)
    sel = (ys % k) * k + (xs % k) == kappa
    return ys[sel], xs[sel]


def proposals(prob: Problem, ys, xs, sweep: int) -> np.ndarray:
    """Candidate offsets of pixels (ys, xs) at a sweep: uint16 [M, 2]."""
    p = np.asarray(ys, dtype=np.int64) * prob.width + np.asarray(xs, dtype=np.int64)
    return philox.q16_pair(philox.draw(p, sweep, prob.problem_id, philox.S_PROP, prob.seed))


def phase(prob: Problem, st: State, kappa: int) -> dict:
    """One colour phase at sweep st.sweep; commits accepted moves into st."""
    ys, xs = class_pixels(prob.width, prob.height, prob.colour_k, kappa)
    u_new = proposals(prob, ys, xs, st.sweep).astype(np.int64)
    c_new = estimator.hit_counts(prob.n, prob.g, u_new, prob.table)
    xd = energy.delta_class_sums(st.c, ys, xs, c_new, prob.radius)
    acc = energy.weighted_class_sum(xd, prob.radius, prob.sigma)
    delta = acc * (2.0 / (prob.n * prob.n))
    g_new = None
    if st.g is not None:
        g_new = estimator.gauss_estimates(prob.n, prob.g, u_new, prob.gauss)
        delta = delta + np.array([energy.delta_plain(st.g, y, x, g_new[j], prob.radius, prob.sigma)
                                  for j, (y, x) in enumerate(zip(ys, xs))])
    accept = (delta < 0.0) if prob.objective == 1 else (delta > 0.0)
    st.u[ys[accept], xs[accept]] = u_new[accept]
    st.c[ys[accept], xs[accept]] = c_new[accept]
    if st.g is not None:
        st.g[ys[accept], xs[accept]] = g_new[accept]
    return {"ys": ys, "xs": xs, "u_new": u_new, "c_new": c_new, "g_new": g_new, "xd": xd,
            "delta": delta, "accept": accept}


def swap_permutation(prob: Problem) -> np.ndarray:
    """pi: pixel indices sorted by the keys (w0 << 32) | w1 of
    Philox((p, 0, problem, S_PERM)), ties by pixel index."""
    npix = prob.width * prob.height
    w = philox.draw(np.arange(npix), 0, prob.problem_id, philox.S_PERM, prob.seed)
    key = (w[:, 0].astype(np.uint64) << np.uint64(32)) | w[:, 1].astype(np.uint64)
    return np.argsort(key, kind="stable").astype(np.int64)


def swap_mask(prob: Problem, sweep: int, kappa: int) -> int:
    """XOR mask of pass kappa of a sweep: word 0 of Philox((kappa, sweep,
    problem, S_SWAP)) modulo the (power-of-two) pixel count."""
    w = philox.draw(np.array([kappa]), sweep, prob.problem_id, philox.S_SWAP, prob.seed)
    return int(w[0, 0]) & (prob.width * prob.height - 1)


def swap_couples(prob: Problem, sweep: int, kappa: int):
    """Pixel indices (a, b) of the couples of pass kappa, in list order."""
    m = prob.width * prob.height // prob.colour_k ** 2
    pix = prob.perm[kappa * m:(kappa + 1) * m] ^ swap_mask(prob, sweep, kappa)
    return pix[0::2], pix[1::2]


def swap_pass(prob: Problem, st: State, kappa: int) -> dict:
    """One swap pass at sweep st.sweep; commits accepted exchanges into st."""
    a, b = swap_couples(prob, st.sweep, kappa)
    ay, ax = np.divmod(a, prob.width)
    by, bx = np.divmod(b, prob.width)
    xd = energy.swap_class_sums(st.c, ay, ax, by, bx, prob.radius)
    delta = energy.weighted_class_sum(xd, prob.radius, prob.sigma) * (2.0 / (prob.n * prob.n))
    accept = (delta < 0.0) if prob.objective == 1 else (delta > 0.0)
    sa, sb = (ay[accept], ax[accept]), (by[accept], bx[accept])
    st.u[sa], st.u[sb] = st.u[sb].copy(), st.u[sa].copy()
    st.c[sa], st.c[sb] = st.c[sb].copy(), st.c[sa].copy()
    return {"a": a, "b": b, "xd": xd, "delta": delta, "accept": accept}


def sweep(prob: Problem, st: State) -> None:
    """All K^2 phases (or swap passes) of one sweep, then advance the sweep index."""
    step = swap_pass if prob.move == 1 else phase
    for kappa in range(prob.colour_k ** 2):
        st.accepts.append(int(step(prob, st, kappa)["accept"].sum()))
    st.sweep += 1


def run(prob: Problem, st: State, k: int) -> State:
    for _ in range(k):
        sweep(prob, st)
    return st


def errors(prob: Problem, st: State) -> np.ndarray:
    """Error vectors [H, W, T + T_G]: Heaviside rows then Gaussian rows."""
    e = estimator.errors_from_counts(st.c, prob.n, prob.areas)
    if st.g is not None:
        e = np.concatenate([e, st.g - prob.gauss_integrals], axis=-1)
    return e


def energy_of(prob: Problem, st: State) -> float:
    e = energy.energy_exact(st.c, prob.n, prob.radius, prob.sigma)
    if st.g is not None:
        e += energy.energy_plain(st.g, prob.radius, prob.sigma)
    return e
