"""C-ABI checks that need no GPU: the library loads, exports every declared
entry point, validates configurations before any device work, and its host
tables (window classes, Heaviside integrals, Philox-drawn integrands) agree
with the oracle."""
import os
import re

import numpy as np
import pytest

from oracle import energy, integrands
import synthgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(bnlat.LIB_PATH):
        pytest.skip("libbnlat.so is not built")
    return bnlat.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bnlat.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bn_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 29
    for n in names:
        assert hasattr(L, n), n


def cfg(**kw):
    base = dict(synthgen.WORKLOADS["tile32_n16_t64"])
    base.update(kw)
    return bnlat.make_config(**base)


@pytest.mark.parametrize("kw", [dict(n=12), dict(n=0), dict(g=(2, 7)), dict(colour_k=3),
                                dict(radius=0), dict(radius=32), dict(radius=9), dict(sigma=0.0),
                                dict(t_heaviside=0), dict(objective=0), dict(width=30, colour_k=4)])
def test_validation_rejects(L, kw):
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.validate_config(cfg(**kw))
    assert e.value.status == bnlat.BN_EINVAL


def test_validation_accepts_workloads(L):
    for wl in synthgen.WORKLOADS.values():
        bnlat.validate_config(bnlat.make_config(**wl))
    for wl in synthgen.dimension_pair_batch():
        bnlat.validate_config(bnlat.make_config(**wl))


def test_create_rejects_bad_config_before_device(L):
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Problem(cfg(n=12))
    assert e.value.status == bnlat.BN_EINVAL
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Problem(cfg(t_heaviside=0, t_gauss=4))
    assert e.value.status == bnlat.BN_EUNSUPPORTED


def test_create_rejects_bad_normal_before_device(L):
    h = bnlat.heaviside_array(synthgen.heaviside_table(64, seed=0))
    h["nx"][3], h["ny"][3] = 0, 0
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Problem(cfg(), h)
    assert e.value.status == bnlat.BN_EINVAL


def test_window_classes_match_oracle_bitwise(L):
    for r, sigma in ((3, 2.1), (4, 2.1), (5, 2.1), (2, 0.7), (6, 3.3)):
        d, w = bnlat.window_classes(cfg(radius=r, sigma=sigma, width=64, height=64))
        assert list(d) == energy.distance_classes(r)
        np.testing.assert_array_equal(w, energy.class_weights(r, sigma))


def test_heaviside_areas_match_oracle(L):
    t = synthgen.heaviside_table(500, seed=11)
    for nx, ny, cx, cy in zip(t["nx"], t["ny"], t["cx"], t["cy"]):
        assert bnlat.heaviside_area(nx, ny, cx, cy) == pytest.approx(
            integrands.heaviside_area(nx, ny, cx, cy), abs=2e-16)
    for args in ((16384, 0, 1000, 5), (0, -16384, 9, 40000), (1000, 1000, 50000, 50000)):
        assert bnlat.heaviside_area(*args) == pytest.approx(integrands.heaviside_area(*args), abs=2e-16)


def test_drawn_heavisides_match_oracle_draw(L):
    got = bnlat.draw_heavisides(seed=5, problem_id=3, t=2000)
    want = integrands.heaviside_table_philox(2000, seed=5, problem=3)
    for k in ("nx", "ny", "cx", "cy"):
        np.testing.assert_array_equal(got[k], want[k])


def test_gaussians_match_oracle(L):
    got = bnlat.draw_gaussians(seed=7, problem_id=2, t=500)
    want = integrands.gaussian_table_philox(500, seed=7, problem=2)
    for k in ("mx", "my", "s"):
        np.testing.assert_array_equal(got[k], want[k])
    for mx, my, s in zip(got["mx"][:100], got["my"][:100], got["s"][:100]):
        assert bnlat.gaussian_integral(mx, my, s) == pytest.approx(integrands.gaussian_integral(mx, my, s),
                                                                   rel=1e-14, abs=1e-16)
    with pytest.raises(bnlat.BnlatError):
        bnlat.gaussian_integral(0.5, 0.5, 0.0)


def test_device_calls_fail_loudly_without_gpu(L):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Problem(cfg())
    assert e.value.status == bnlat.BN_EHIP


def test_swap_permutation_matches_oracle(L):
    from oracle import sweep as osw
    for w, h, seed, pid in [(16, 8, 5, 0), (64, 64, 3, 7), (256, 256, 2, 0)]:
        c = cfg(width=w, height=h, seed=seed, problem_id=pid, move=bnlat.BN_SWAP)
        ref = osw.Problem(n=16, g=(1, 7), width=w, height=h, radius=3, sigma=2.1, colour_k=2, seed=seed,
                          problem_id=pid, table=synthgen.heaviside_table(4, seed=0), move=1)
        np.testing.assert_array_equal(bnlat.swap_permutation(c), ref.perm)


@pytest.mark.parametrize("kw", [dict(width=48, height=32), dict(precision=1), dict(t_gauss=8),
                                dict(width=2, height=2, colour_k=2, radius=1)])
def test_swap_unsupported_forms_rejected_before_device(L, kw):
    with pytest.raises(bnlat.BnlatError) as e:
        bnlat.Problem(cfg(move=bnlat.BN_SWAP, **kw))
    assert e.value.status == bnlat.BN_EUNSUPPORTED
