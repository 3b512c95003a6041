"""The allocation-free forward (nursd_forward_hist_static) against the
forward with a caller workspace (nursd_forward_hist), both through the C ABI.

Two calls in a row share the library's fixed device scratch, the second on
a smaller input (the differentiation workload, then the tiny one), and a
third call repeats the first: each must give what nursd_forward_hist gives
on the same plan (bit-exact, since the launch sequence is the same; the
tiny case is also checked against the FP64 oracle at rel-L2 <= 1e-4).  A
plan whose workspace exceeds the fixed scratch is refused before any
launch."""
from ctypes import c_void_p

import numpy as np
import pytest
import torch

from oracle import nursd_ref as o
from workloads import scenes

pytestmark = pytest.mark.gpu

SCRATCH = 512 << 20


def _plan(w, device):
    from paper_2501_05244_amd.api import plan_from_workload
    return plan_from_workload(w, device)


def _static(plan, hist):
    from paper_2501_05244_amd import _lib
    lib = _lib.load()
    V = torch.full(plan.out_shape(), complex(7.0, -7.0), dtype=torch.complex64, device=hist.device)
    I = torch.full(plan.out_shape(), 7.0, dtype=torch.float32, device=hist.device)
    s = c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.nursd_forward_hist_static(plan.handle, c_void_p(hist.data_ptr()), c_void_p(V.data_ptr()),
                                       c_void_p(I.data_ptr()), s)
    _lib.check(rc, "nursd_forward_hist_static")
    torch.cuda.synchronize()
    return V, I


def _with_workspace(plan, hist):
    V, I = plan.forward_hist(hist)
    torch.cuda.synchronize()
    return V, I


def _same(a, b, what):
    d = (a - b).abs().max().item()
    print(f"  {what}: max |static - workspace| = {d:.3e}", flush=True)
    assert torch.equal(a, b), what


def test_static_scratch_two_calls_then_repeat(device):
    big = scenes.config_diff()
    small = scenes.config_tiny()
    pb, ps = _plan(big, device), _plan(small, device)
    for p, name in ((pb, "differentiation"), (ps, "tiny")):
        print(f"  {name}: workspace {p.info['workspace_bytes']} bytes", flush=True)
        assert p.info["workspace_bytes"] <= SCRATCH
    assert ps.info["workspace_bytes"] < pb.info["workspace_bytes"]
    hb = torch.from_numpy(big.hist).to(device)
    hs = torch.from_numpy(small.hist).to(device)

    Vb_ref, Ib_ref = _with_workspace(pb, hb)
    Vs_ref, Is_ref = _with_workspace(ps, hs)

    Vb, Ib = _static(pb, hb)                 # first call
    _same(Vb, Vb_ref, "differentiation V")
    _same(Ib, Ib_ref, "differentiation I")
    Vs, Is = _static(ps, hs)                 # second call, smaller input
    _same(Vs, Vs_ref, "tiny V")
    _same(Is, Is_ref, "tiny I")
    Vb2, Ib2 = _static(pb, hb)               # the scratch now holds the tiny call's data
    _same(Vb2, Vb_ref, "differentiation V, repeated")
    _same(Ib2, Ib_ref, "differentiation I, repeated")

    P, f = o.phasors_from_workload(small)
    ref = o.nursd_grid(P, small.relay_xy.astype(np.float64), f, o.frame_for_workload(small), small.grid, small.xp)
    err = float(np.linalg.norm(Vs.cpu().numpy() - ref) / np.linalg.norm(ref))
    print(f"  tiny V vs the FP64 oracle: rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-4


def test_static_scratch_refuses_a_large_plan(device):
    from paper_2501_05244_amd import _lib
    w = scenes.config_spad(render=False)
    p = _plan(w, device)
    assert p.info["workspace_bytes"] > SCRATCH
    lib = _lib.load()
    hist = torch.zeros(1, dtype=torch.float32, device=device)     # never read: the call fails first
    I = torch.zeros(1, dtype=torch.float32, device=device)
    rc = lib.nursd_forward_hist_static(p.handle, c_void_p(hist.data_ptr()), None, c_void_p(I.data_ptr()),
                                       c_void_p(torch.cuda.current_stream().cuda_stream))
    msg = lib.nursd_last_error().decode()
    print(f"  rc {rc}: {msg}", flush=True)
    assert rc == -4 and "fixed scratch" in msg
    torch.cuda.synchronize()
