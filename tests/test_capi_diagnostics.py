"""Host-side diagnostics of the C ABI, no GPU needed:
- BNLAT_LOG=1 reports failures on stderr;
- a build whose host code is instrumented with AddressSanitizer and
  UndefinedBehaviorSanitizer runs every host-only entry point (validation,
  window tables, integrand draws and integrals, the swap permutation, status
  strings, the no-device failure path) without a report."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent('''
    import sys
    sys.path.insert(0, {root!r})
    import numpy as np
    from paper_2105_12620_amd import bnlat
    import synthgen
    w = dict(synthgen.WORKLOADS["tile32_n16_t64"])
    bnlat.validate_config(bnlat.make_config(**w))
    for bad in (dict(n=12), dict(g=(2, 7)), dict(colour_k=3), dict(radius=0), dict(radius=40), dict(sigma=0.0),
                dict(t_heaviside=0), dict(objective=0), dict(width=30, colour_k=4), dict(width=1, height=1)):
        try:
            bnlat.validate_config(bnlat.make_config(**dict(w, **bad)))
            raise SystemExit("accepted " + repr(bad))
        except bnlat.BnlatError as e:
            assert e.status == bnlat.BN_EINVAL
    for r in range(1, 7):
        d, wt = bnlat.window_classes(bnlat.make_config(**dict(w, radius=r, width=16, height=16)))
        assert len(d) == len(wt) > 0
    h = bnlat.draw_heavisides(5, 2, 300)
    for row in h[:50]:
        a = bnlat.heaviside_area(row["nx"], row["ny"], row["cx"], row["cy"])
        assert 0.0 <= a <= 1.0
    g = bnlat.draw_gaussians(5, 2, 100)
    assert all(bnlat.gaussian_integral(x["mx"], x["my"], x["s"]) > 0 for x in g)
    for bad in ((0, 0, 5, 5), (20000, 0, 5, 5)):
        try:
            bnlat.heaviside_area(*bad)
            raise SystemExit("accepted normal " + repr(bad))
        except bnlat.BnlatError:
            pass
    perm = bnlat.swap_permutation(bnlat.make_config(**dict(w, width=64, height=32, move=1)))
    assert np.array_equal(np.sort(perm), np.arange(64 * 32))
    L = bnlat.lib()
    for s in range(-7, 1):
        assert L.bn_status_string(s)
    try:
        bnlat.Problem(bnlat.make_config(**w))
    except bnlat.BnlatError as e:
        assert e.status in (bnlat.BN_EHIP, bnlat.BN_OK)
    print("host entry points ok")
''')


def _no_gpu():
    try:
        import torch
        return not torch.cuda.is_available()
    except ImportError:
        return True


def test_log_reports_failures():
    env = dict(os.environ, BNLAT_LOG="1")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2105_12620_amd import bnlat\n"
            "try:\n"
            "    bnlat.validate_config(bnlat.make_config(n=12, g=(1, 7), width=8, height=8, t_heaviside=4))\n"
            "except bnlat.BnlatError:\n"
            "    pass\n") % ROOT
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert "[bnlat] error -1: N=12 must be a power of two" in res.stderr
    env["BNLAT_LOG"] = "0"
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert "[bnlat]" not in res.stderr


@pytest.mark.skipif(not _no_gpu(), reason="host-only check; run where no GPU is present")
def test_host_code_clean_under_address_and_undefined_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2105_12620_amd import build
    rt = build.asan_runtime()
    if not os.path.exists(rt):
        pytest.skip("sanitizer runtime not found")
    lib = build.build(sanitize_host=True, out=str(tmp_path / "libbnlat_san.so"))
    env = dict(os.environ, BNLAT_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], env=env, capture_output=True,
                         text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "host entry points ok" in res.stdout
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
