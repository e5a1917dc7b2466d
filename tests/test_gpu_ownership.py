"""Buffer ownership and allocation failures of the C ABI on the GPU:
- bn_create_problem_ext with caller-owned device buffers (PyTorch tensors):
  the problem's offsets, hit counts and error vectors are written in place in
  the documented layouts, the trajectory equals the library-owned problem's,
  and the tensors stay valid after destroy;
- BNLAT_FAULT=alloc:K makes the K-th device allocation of a problem being
  created fail: every K gives BN_ENOMEM, and the earlier allocations are
  released (free device memory is back where it was)."""
import os

import numpy as np
import pytest

from oracle import sweep as osw
import synthgen

from cases import EDGE, gpu_problem, oracle_problem, say, workload

pytestmark = pytest.mark.gpu
bnlat = pytest.importorskip("paper_2105_12620_amd.bnlat")
torch = pytest.importorskip("torch")


def test_caller_owned_buffers_hold_the_state():
    w = EDGE["n256_r4"]
    inp = synthgen.problem_inputs(w)
    P, T = w["width"] * w["height"], w["t_heaviside"]
    Tp = (T + 127) // 128 * 128
    u = torch.zeros(P, dtype=torch.int32, device="cuda")
    c = torch.full((Tp // 8, P, 8), -1, dtype=torch.int16, device="cuda")
    e = torch.zeros((P, Tp), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ref = oracle_problem(w, inp)
    st = osw.initial_state(ref, inp["offsets"])
    with bnlat.create_problem(w, bnlat.heaviside_array(inp["heaviside"]),
                              buffers=(u.data_ptr(), c.data_ptr(), e.data_ptr())) as p:
        p.init_offsets(inp["offsets"])
        p.compute_errors()
        torch.cuda.synchronize()
        uu = u.cpu().numpy().view(np.uint32)
        np.testing.assert_array_equal(uu & 0xFFFF, inp["offsets"].reshape(-1, 2)[:, 0])
        np.testing.assert_array_equal(uu >> 16, inp["offsets"].reshape(-1, 2)[:, 1])
        cc = c.cpu().numpy().view(np.uint16)                 # [Tp/8][P][8]
        rows = cc.transpose(1, 0, 2).reshape(P, Tp)
        np.testing.assert_array_equal(rows[:, :T], st.c.reshape(P, T))
        assert not rows[:, T:].any()
        ee = e.cpu().numpy()
        np.testing.assert_allclose(ee[:, :T], st.c.reshape(P, T) / w["n"] - ref.areas, atol=1e-6)
        p.sweep(3)
        got = p.get_offsets()
        torch.cuda.synchronize()
        uu = u.cpu().numpy().view(np.uint32)
    with gpu_problem(w, inp) as q:
        q.sweep(3)
        np.testing.assert_array_equal(q.get_offsets(), got)
    np.testing.assert_array_equal(uu & 0xFFFF, got.reshape(-1, 2)[:, 0])
    # the caller's tensors are still theirs after destroy
    c.fill_(3)
    torch.cuda.synchronize()
    assert int(c[0, 0, 0]) == 3


def test_caller_owned_buffers_must_be_aligned():
    w = EDGE["n4_ragged"]
    t = torch.zeros(4096, dtype=torch.int32, device="cuda")
    with pytest.raises(bnlat.BnlatError) as ei:
        bnlat.create_problem(w, None, buffers=(t.data_ptr() + 4, None, None))
    assert ei.value.status == bnlat.BN_EINVAL


def test_injected_allocation_failures_release_everything():
    w = workload(n=64, g=(1, 19), t_heaviside=40, t_gauss=30, width=16, height=12, radius=3)
    inp = synthgen.problem_inputs(w)
    h = bnlat.heaviside_array(inp["heaviside"])
    g = bnlat.gaussian_array(inp["gauss"]) if w.get("t_gauss", 0) else None
    with bnlat.create_problem(w, h, gaussians=g) as p:   # warm the runtime
        p.init_offsets(None)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failures = 0
    try:
        for k in range(1, 40):
            os.environ["BNLAT_FAULT"] = f"alloc:{k}"
            try:
                q = bnlat.create_problem(w, h, gaussians=g)
            except bnlat.BnlatError as e:
                assert e.status == bnlat.BN_ENOMEM
                failures += 1
                continue
            q.close()     # K past the problem's allocation count: nothing failed
            break
    finally:
        os.environ.pop("BNLAT_FAULT", None)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("injected failures", failures, "free before", free0, "after", free1)
    assert failures >= 15
    assert abs(free1 - free0) <= 4 << 20
