"""Pins of the oracle's BF16 precision form (oracle/precision.py).

- round_bf16 against PyTorch's own FP32 -> bfloat16 conversion (a library
  routine), on random values of many magnitudes and on constructed ties;
- when every operand is exactly representable in BF16 (N <= 256 counts with
  zero integrals) the BF16-form energy change equals the exact one;
- otherwise it stays within the rounding bound derived from BF16's unit
  roundoff 2^-8 (both Gram operands rounded once, products exact) around the
  plain FP64 change computed independently; a flipped Gram sign, a wrong
  weight or factor leaves that bound, and unrounded operands fail the check
  that the rounding shows;
- the BF16-form energy equals the exact energy for representable operands
  and is within its rounding bound otherwise."""
import numpy as np
import pytest

from oracle import energy, estimator, precision
import synthgen

torch = pytest.importorskip("torch")

U = 2.0 ** -8


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * s for s in (1e-30, 1e-6, 1e-2, 1.0, 1e3, 1e20)])
    # exact ties: low 16 bits 0x8000 with even and odd kept parts
    hi = rng.integers(0x3000, 0x4800, size=4000, dtype=np.uint32) << 16
    ties = (hi | 0x8000).view(np.float32)
    x = np.concatenate([x.astype(np.float32), ties, -ties, np.float32([0.0, -0.0, 1.0, 2.0 ** -133])])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(precision.round_bf16(x), want)


def _state(n, g, W, H, T, TG, seed, areas_zero=False):
    tab = synthgen.heaviside_table(T, seed=seed)
    u = synthgen.offsets(W, H, seed=seed + 1).reshape(-1, 2).astype(np.int64)
    c = estimator.hit_counts(n, g, u, tab).reshape(H, W, T)
    from oracle import integrands
    A = np.zeros(T) if areas_zero else integrands.heaviside_areas(tab)
    gt = gq = gint = None
    if TG:
        gt = synthgen.gaussian_table(TG, seed=seed + 2)
        gq = estimator.gauss_estimates(n, g, u, gt).reshape(H, W, TG)
        gint = integrands.gaussian_integrals(gt)
    return tab, c, A, gt, gq, gint


def test_representable_operands_give_the_exact_change():
    n, g, W, H, T, r, sig = 16, (1, 7), 12, 10, 40, 3, 2.1
    tab, c, A, *_ = _state(n, g, W, H, T, 0, seed=3, areas_zero=True)
    ys, xs = np.array([0, 3, 9, 5]), np.array([0, 7, 11, 2])
    u_new = synthgen.proposals(4, seed=5).astype(np.int64)
    c_new = estimator.hit_counts(n, g, u_new, tab)
    want = energy.delta_exact(c, ys, xs, c_new, n, r, sig)
    got = precision.delta_bf16(c, ys, xs, c_new, n, A, r, sig)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)
    e = c / n
    assert precision.energy_bf16(c, n, A, r, sig) == pytest.approx(energy.energy_plain(e, r, sig), rel=1e-12)


@pytest.mark.parametrize("n,g,TG", [(1024, (1, 381), 0), (1024, (1, 381), 24), (64, (1, 19), 16)])
def test_change_within_bf16_rounding_bound(n, g, TG):
    W, H, T, r, sig = 14, 12, 60, 4, 2.1
    tab, c, A, gt, gq, gint = _state(n, g, W, H, T, TG, seed=7)
    ys, xs = np.divmod(synthgen.pixel_sample(W * H, 30, seed=8).astype(np.int64), W)
    u_new = synthgen.proposals(30, seed=9).astype(np.int64)
    c_new = estimator.hit_counts(n, g, u_new, tab)
    g_new = estimator.gauss_estimates(n, g, u_new, gt) if TG else None
    got = precision.delta_bf16(c, ys, xs, c_new, n, A, r, sig, g=gq, g_new=g_new, gint=gint)
    # exact change of the same move, plain FP64 form over all rows
    e = c / n - A
    en = c_new / n - A
    if TG:
        e = np.concatenate([e, gq - gint], axis=2)
        en = np.concatenate([en, g_new - gint], axis=1)
    exact = np.array([energy.delta_plain(e, y, x, en[j], r, sig) for j, (y, x) in enumerate(zip(ys, xs))])
    # |dE_bf - dE| <= 4 sum_o w_o sum_t |delta_t e_q,t| ((1+u)^2 (1+2^-23)^2 - 1)
    gram_abs = np.zeros(len(ys))
    for ox, oy in energy.window_offsets(r):
        eq = e[(ys + oy) % H, (xs + ox) % W]
        gram_abs += energy.weight(ox * ox + oy * oy, sig) * np.sum(np.abs((en - e[ys, xs]) * eq), axis=1)
    bound = 4.0 * gram_abs * ((1 + U) ** 2 * (1 + 2.0 ** -23) ** 2 - 1)
    err = np.abs(got - exact)
    assert np.all(err <= bound), (err / bound).max()
    # the operands really are rounded (the form is approximate here)
    assert err.max() > 0
    # the scale used by GPU tolerances covers every term
    scale = precision.delta_bf16_scale(c, ys, xs, c_new, n, A, r, sig, g=gq, g_new=g_new, gint=gint)
    assert np.all(scale >= np.abs(got)) and np.all(scale >= 4.0 * gram_abs * (1 - 2 * U))


def test_energy_within_bf16_rounding_bound():
    n, g, W, H, T, r, sig = 1024, (1, 381), 12, 12, 50, 3, 2.1
    tab, c, A, *_ = _state(n, g, W, H, T, 0, seed=11)
    e = c / n - A
    exact = energy.energy_plain(e, r, sig)
    got = precision.energy_bf16(c, n, A, r, sig)
    # each |e^_p - e^_q|^2 term moves by at most 2 |d| (u |e_p| + u |e_q|) + (u |e_p| + u |e_q|)^2 (u with
    # the FP32 step)
    uu = (1 + U) * (1 + 2.0 ** -23) - 1
    bound = 0.0
    for ox, oy in energy.window_offsets(r):
        q = np.roll(e, shift=(-oy, -ox), axis=(0, 1))
        s = uu * (np.abs(e) + np.abs(q))
        bound += energy.weight(ox * ox + oy * oy, sig) * float(np.sum(2 * np.abs(e - q) * s + s * s))
    assert 0 < abs(got - exact) <= bound
