"""GPU parity of the plan options against the FP64 oracle, through the C ABI:
the upsampled frame (upsample_q), the unit-amplitude kernel (kernel_inv_r =
0), per-sample weights (forward and adjoint), the frame check of
nursd_plan_set_points, the position binding of the autograd function, and
the batch with scenes propagated by ordinary launches inside its graph.
Tolerance: relative L2 <= 1e-4 (the method's FP32 target)."""
import numpy as np
import pytest
import torch

from oracle import nursd_ref as o
from workloads import scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4


def rel(a, b):
    r = float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))
    print(f"  rel-L2 {r:.3e}", flush=True)
    return r


def case(seed=5, nx=20, ny=13, nz=3, L=300, F=3):
    rng = np.random.default_rng(seed)
    dx = 0.02
    g = scenes.Grid(x0=-0.19, y0=-0.13, dx=dx, dy=dx, nx=nx, ny=ny, z=np.linspace(0.21, 0.6, nz))
    xy = np.stack([rng.uniform(-0.18, 0.18, L), rng.uniform(-0.12, 0.12, L)], 1).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=512, dt=8e-12, t0=0.0, n_freq=F, bins=np.array([13, 19, 26])[:F])
    w = scenes.Workload("options", xy, np.array([0.01, -0.02, 0.0]), wl, g)
    P = (rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64)
    return w, P


def freqs(w):
    return o.wavelet_bins(w.wavelet.lambda_c, w.wavelet.n_time, w.wavelet.dt, w.wavelet.n_freq, w.wavelet.bins)[1]


def plan_for(w, device, **kw):
    from paper_2501_05244_amd.api import plan_from_workload
    return plan_from_workload(w, device, **kw)


@pytest.mark.parametrize("q,chunks", [(2, (0, 0)), (3, (2, 2))])
def test_upsampled_frame_forward(device, q, chunks):
    print("case: upsample_q", q, chunks, flush=True)
    w, P = case(seed=10 + q)
    plan = plan_for(w, device, upsample_q=q, freq_chunk=chunks[0], plane_chunk=chunks[1])
    fr = o.frame_for_workload(w, q)
    assert plan.info["M"] == fr.M and plan.info["upsample_q"] == q
    assert abs(plan.info["cx"] - fr.cx) < 1e-12 and abs(plan.info["dx"] - fr.dx) < 1e-15
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    ref = o.nursd_grid(P.astype(np.complex128), w.relay_xy.astype(np.float64), freqs(w), fr, w.grid, w.xp)
    assert rel(V.cpu().numpy(), ref) < TOL
    assert rel(I.cpu().numpy(), np.abs(ref)) < TOL


def test_upsampled_frame_adjoint(device):
    print("case: upsample_q adjoint", flush=True)
    w, P = case(seed=21)
    plan = plan_for(w, device, upsample_q=2)
    fr = o.frame_for_workload(w, 2)
    rng = np.random.default_rng(22)
    gV = (rng.normal(size=plan.out_shape()) + 1j * rng.normal(size=plan.out_shape())).astype(np.complex64)
    gP, gxy = plan.adjoint(torch.from_numpy(gV).to(device), torch.from_numpy(P).to(device))
    rP, rxy = o.nursd_grid_adjoint(gV.astype(np.complex128), w.relay_xy.astype(np.float64), freqs(w), fr, w.grid,
                                   w.xp, P.astype(np.complex128))
    assert rel(gP.cpu().numpy(), rP) < TOL
    assert rel(gxy.cpu().numpy(), rxy) < TOL


def test_unit_amplitude_kernel_grid(device):
    print("case: kernel without 1/r (grid)", flush=True)
    w, P = case(seed=31)
    plan = plan_for(w, device, kernel_inv_r=False)
    V, _ = plan.forward_phasor(torch.from_numpy(P).to(device), intensity=False)
    ref = o.nursd_grid(P.astype(np.complex128), w.relay_xy.astype(np.float64), freqs(w), o.frame_for_workload(w),
                       w.grid, w.xp, inv_r=False)
    assert rel(V.cpu().numpy(), ref) < TOL


def test_unit_amplitude_kernel_points(device):
    print("case: kernel without 1/r (voxel lists)", flush=True)
    rng = np.random.default_rng(33)
    L, counts, F = 900, (300, 0, 517), 2
    xy = rng.uniform(-0.9, 0.9, size=(L, 2)).astype(np.float32)
    zs = np.array([0.5, 0.8, 1.2])
    voxel_xy = np.concatenate([rng.uniform(-0.85, 0.85, size=(c, 2)) for c in counts]).astype(np.float32)
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=4096, dt=4e-12, t0=0.0, n_freq=F, bins=np.array([64, 101]))
    g = scenes.Grid(x0=0, y0=0, dx=0.0078125, dy=0.0078125, nx=0, ny=0, z=zs)
    w = scenes.Workload("points_inv_r", xy, np.array([0.01, 0.02, 0.0]), wl, g, mode="points", plane_ptr=ptr,
                        voxel_xy=voxel_xy)
    P = np.ascontiguousarray((rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64))
    plan = plan_for(w, device, M=512, kernel_inv_r=False)
    fr = o.choose_frame("points", xy, dx=g.dx, dy=g.dy, voxel_xy=voxel_xy, sizes=(512,))
    V, _ = plan.forward_phasor(torch.from_numpy(P).to(device), intensity=False)
    ref = o.nursd_points(P.astype(np.complex128), xy.astype(np.float64), freqs(w), fr, zs, ptr,
                         voxel_xy.astype(np.float64), w.xp, inv_r=False)
    assert rel(V.cpu().numpy(), ref) < TOL


def test_weights_forward_and_adjoint(device):
    print("case: per-sample weights", flush=True)
    w, P = case(seed=41)
    rng = np.random.default_rng(42)
    wts = rng.uniform(0.2, 1.5, size=w.relay_xy.shape[0]).astype(np.float32)
    plan = plan_for(w, device, weights=torch.from_numpy(wts).to(device))
    fr = o.frame_for_workload(w)
    f = freqs(w)
    xy = w.relay_xy.astype(np.float64)
    V, _ = plan.forward_phasor(torch.from_numpy(P).to(device), intensity=False)
    ref = o.nursd_grid(P.astype(np.complex128), xy, f, fr, w.grid, w.xp, weights=wts)
    assert rel(V.cpu().numpy(), ref) < TOL
    gV = (rng.normal(size=plan.out_shape()) + 1j * rng.normal(size=plan.out_shape())).astype(np.complex64)
    gP, gxy = plan.adjoint(torch.from_numpy(gV).to(device), torch.from_numpy(P).to(device))
    rP, rxy = o.nursd_grid_adjoint(gV.astype(np.complex128), xy, f, fr, w.grid, w.xp, P.astype(np.complex128),
                                   weights=wts)
    assert rel(gP.cpu().numpy(), rP) < TOL
    assert rel(gxy.cpu().numpy(), rxy) < TOL


def test_set_points_enforces_the_frame_rule(device):
    """A relay moved inside the period but more than half a period from a
    voxel would wrap around the circular convolution: set_points refuses it
    and the plan keeps its previous positions."""
    w, P = case(seed=51)
    plan = plan_for(w, device, M=64)
    Pd = torch.from_numpy(P).to(device)
    V0, _ = plan.forward_phasor(Pd, intensity=False)
    fr = o.frame_for_workload(w)
    assert fr.M == 64
    moved = w.relay_xy.copy()
    moved[3, 0] = fr.cx - 30 * fr.dx          # inside [c - 32 dx, c + 32 dx), 39 dx from the last voxel
    with pytest.raises(RuntimeError, match="GEOMETRY"):
        plan.set_points(torch.from_numpy(moved).to(device))
    outside = w.relay_xy.copy()
    outside[5, 1] = fr.cy + 40 * fr.dy        # outside the period
    with pytest.raises(RuntimeError, match="GEOMETRY"):
        plan.set_points(torch.from_numpy(outside).to(device))
    V1, _ = plan.forward_phasor(Pd, intensity=False)
    assert torch.equal(torch.view_as_real(V0), torch.view_as_real(V1))


def test_autograd_binds_each_forwards_positions(device):
    """Two forwards at different positions, then the first one's backward:
    the gradients are those of the first positions.  Temporaries created one
    after another (finite-difference style) each get their own positions."""
    print("case: autograd position binding", flush=True)
    from paper_2501_05244_amd.autograd import nursd
    w, P = case(seed=61, L=200)
    plan = plan_for(w, device)
    fr = o.frame_for_workload(w)
    f = freqs(w)
    rng = np.random.default_rng(62)
    xy1 = torch.from_numpy(w.relay_xy).to(device)
    xy2 = xy1 + torch.from_numpy(rng.normal(0, 0.003, size=w.relay_xy.shape).astype(np.float32)).to(device)
    Pg = torch.from_numpy(P).to(device).requires_grad_(True)
    x1 = xy1.clone().requires_grad_(True)
    tgt = torch.zeros(plan.out_shape(), dtype=torch.complex64, device=device)
    V1 = nursd(Pg, x1, plan)
    with torch.no_grad():
        V2 = nursd(Pg.detach(), xy2, plan)
    loss = (V1 - tgt).abs().pow(2).sum()
    loss.backward()
    x1n = w.relay_xy.astype(np.float64)
    Vr = o.nursd_grid(P.astype(np.complex128), x1n, f, fr, w.grid, w.xp)
    rP, rxy = o.nursd_grid_adjoint(2 * Vr, x1n, f, fr, w.grid, w.xp, P.astype(np.complex128))
    assert rel(V1.detach().cpu().numpy(), Vr) < TOL
    assert rel(Pg.grad.cpu().numpy(), rP) < TOL
    assert rel(x1.grad.cpu().numpy(), rxy) < TOL
    V2r = o.nursd_grid(P.astype(np.complex128), xy2.cpu().numpy().astype(np.float64), f, fr, w.grid, w.xp)
    assert rel(V2.cpu().numpy(), V2r) < TOL
    # temporaries: +h and -h offsets of one coordinate, one after the other
    h = 1e-3
    for sign in (1.0, -1.0):
        xt = xy1.clone()
        xt[7, 0] += sign * h
        with torch.no_grad():
            Vt = nursd(Pg.detach(), xt, plan)
        ref = o.nursd_grid(P.astype(np.complex128), xt.cpu().numpy().astype(np.float64), f, fr, w.grid, w.xp)
        assert rel(Vt.cpu().numpy(), ref) < TOL
        del xt, Vt
    # fresh leaves detached from one tensor (an optimisation loop) share its
    # memory and version: the plan bins them once
    calls = []
    orig = plan.set_points
    plan.set_points = lambda t, stream=None: (calls.append(1), orig(t, stream))
    base = xy1.clone()
    for _ in range(3):
        with torch.no_grad():
            nursd(Pg.detach(), base.detach().requires_grad_(True), plan)
    assert len(calls) == 1
    base[0, 0] += 1e-3                      # in place: the next call re-bins
    with torch.no_grad():
        Vb = nursd(Pg.detach(), base.detach(), plan)
    assert len(calls) == 2
    ref = o.nursd_grid(P.astype(np.complex128), base.cpu().numpy().astype(np.float64), f, fr, w.grid, w.xp)
    assert rel(Vb.cpu().numpy(), ref) < TOL


def batch_scenes():
    """Three small scenes (transform sizes 64 and 128) and one with M = 512,
    which the default configuration propagates with ordinary launches."""
    out = []
    dx = 0.0078125
    for s, (n, L, F, Z, lam) in enumerate([(32, 300, 3, 2, 0.05), (48, 1200, 5, 3, 0.06), (256, 2000, 3, 2, 0.06),
                                           (20, 400, 4, 3, 0.08)]):
        half = n * dx / 2
        relay = scenes.relay_uniform(L, half * 0.98, seed=300 + s)
        wl = scenes.Wavelet(lambda_c=lam, n_time=2048, dt=4e-12, t0=0.0, n_freq=F)
        g = scenes.Grid(x0=-half + dx / 2, y0=-half + dx / 2, dx=dx, dy=dx, nx=n, ny=n,
                        z=scenes.cell_centres(0.3, 0.3 + n * dx, Z))
        w = scenes.Workload(f"b{s}", relay, np.zeros(3), wl, g)
        bins = o.wavelet_bins(lam, 2048, 4e-12, F)[0]
        w.hist = scenes.tone_histograms(L, 2048, bins[[0, F - 1]], seed=400 + s)
        out.append(w)
    return out


def test_batch_with_chunked_scene_and_caller_workspace(device):
    print("case: batch with a chunk-by-chunk scene", flush=True)
    from paper_2501_05244_amd.api import Batch, plan_from_workload
    ws = batch_scenes()
    plans = [plan_from_workload(w, device) for w in ws]
    assert [p.M for p in plans] == [64, 128, 512, 64]
    hists = [torch.from_numpy(w.hist).to(device) for w in ws]
    plain = [p.forward_hist(h, vol=False)[1] for p, h in zip(plans, hists)]
    b = Batch(plans, autotune=False)
    info = b.info()
    assert info["serial"] == "M>=512" and info["workspace_bytes"] == b.workspace_bytes > 0
    outs = b.forward(hists)
    torch.cuda.synchronize()
    for x, y in zip(outs, plain):
        assert rel(x.cpu().numpy(), y.cpu().numpy()) < 1e-5
    # new outputs and a new workspace: the tables are rebuilt and the graph
    # re-captured; results unchanged
    b._ws = torch.empty(b.workspace_bytes + 512, dtype=torch.uint8, device=device)
    base = b._ws.data_ptr()
    b._ws_ptr = base + (-base) % 256
    outs2 = b.forward(hists, [torch.full_like(x, 7.0) for x in outs])
    torch.cuda.synchronize()
    for x, y in zip(outs2, plain):
        assert rel(x.cpu().numpy(), y.cpu().numpy()) < 1e-5
    # the oracle on the scene propagated chunk by chunk
    w = ws[2]
    P, f = o.phasors_from_workload(w)
    ref = o.nursd_grid(P, w.relay_xy.astype(np.float64), f, o.frame_for_workload(w), w.grid, w.xp, intensity=True)
    assert rel(outs2[2].cpu().numpy(), ref) < TOL


def test_batch_rejects_a_small_workspace(device):
    from ctypes import c_size_t, c_void_p
    from paper_2501_05244_amd import _lib
    from paper_2501_05244_amd.api import Batch, _stream, plan_from_workload
    ws = batch_scenes()[:2]
    plans = [plan_from_workload(w, device) for w in ws]
    hists = [torch.from_numpy(w.hist).to(device) for w in ws]
    b = Batch(plans, autotune=False)
    outs = [torch.empty(p.out_shape(), dtype=torch.float32, device=device) for p in plans]
    hp = (c_void_p * 2)(*[h.data_ptr() for h in hists])
    op = (c_void_p * 2)(*[x.data_ptr() for x in outs])
    lib = _lib.load()
    rc = lib.nursd_batch_forward(b.handle, hp, op, c_void_p(b._ws_ptr), c_size_t(b.workspace_bytes - 256),
                                 _stream(None))
    assert _lib.ERRORS.get(rc) == "NURSD_ERR_WORKSPACE"
    rc = lib.nursd_batch_autotune(b.handle, hp, op, c_void_p(b._ws_ptr), c_size_t(b.workspace_bytes),
                                  _stream(None))
    assert _lib.ERRORS.get(rc) == "NURSD_ERR_ARG"       # created without autotuning
