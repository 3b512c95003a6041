"""GPU parity at the sizes the benchmark times, through the C ABI, against
the FP64 oracle (relative L2 <= 1e-4).

The oracle cannot evaluate whole full-size volumes in seconds, so each test
runs the full-size launch (every frequency and plane of the workload, in
the launch configuration the benchmark uses) with phasors that vanish
outside a few bins, and the oracle evaluates those bins on a subset of
planes or voxels; by linearity the remaining bins add exactly zero.  The
bins are chosen so that every in-chunk position of the propagation's
frequency chunks occurs (the row pass advances each voxel's illumination
phase recursively across a chunk), and the planes so that every in-chunk
plane position occurs.
  * SPAD workload (256 x 256 x 128, 96 frequencies): 8 bins x 16 whole planes.
  * non-planar relays (3D NURSD, M = 512, depth grid 16): 2 bins x 2 planes.
  * frustum voxel lists (64 planes): 4 bins x 64 planes x 256 voxels.
  * scaled RSD frustum: 4 bins x 16 planes.
  * the 64-scene batch: every scene on 2 bins x 4 planes (tone histograms
    whose spectrum vanishes outside those bins), batched and plain.
"""
import numpy as np
import pytest
import torch

from oracle import nursd_ref as o
from workloads import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
TOL = 1e-4


def rel(a, b):
    r = float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))
    print(f"  rel-L2 {r:.3e}", flush=True)
    return r


def plan_for(w, device, **kw):
    from paper_2501_05244_amd.api import plan_from_workload
    return plan_from_workload(w, device, **kw)


def band_phasors(w, hist, sel):
    """Phasors of the workload's band that are zero outside bins `sel`, the
    selected ones from the oracle's direct temporal DFT of `hist`."""
    wl = w.wavelet
    bins, f = o.wavelet_bins(wl.lambda_c, wl.n_time, wl.dt, wl.n_freq)
    wts = o.phasor_weights(f, wl.lambda_c, wl.sigma_rel, wl.t0)
    Pin = np.zeros((wl.n_freq, w.relay_xy.shape[0]), np.complex64)
    Pin[sel] = o.temporal_phasor(hist, bins[sel], wts[sel])
    return Pin, f


def test_spad_full_launch_8_bins_16_planes(device, spad_hist):
    print("case: spad full launch, 8 bins x 16 planes", flush=True)
    w = scenes.config_spad(render=False)
    plan = plan_for(w, device)
    assert plan.info["freq_chunk"] == 8 and plan.info["plane_chunk"] == 16
    # the phasor stage at full size, all 96 bins, on 256 sampled relays
    P = plan.phasor(torch.from_numpy(spad_hist).to(device)).cpu().numpy()
    wl = w.wavelet
    bins, f = o.wavelet_bins(wl.lambda_c, wl.n_time, wl.dt, wl.n_freq)
    wts = o.phasor_weights(f, wl.lambda_c, wl.sigma_rel, wl.t0)
    rows = np.random.default_rng(0).choice(w.relay_xy.shape[0], 256, replace=False)
    assert rel(P[:, rows], o.temporal_phasor(spad_hist[rows], bins, wts)) < 5e-6
    # bins at in-chunk positions 0..7 of eight different chunks of 8
    sel = [0, 9, 18, 27, 44, 53, 70, 95]
    assert sorted(b % 8 for b in sel) == list(range(8))
    Pin, f = band_phasors(w, spad_hist, sel)
    V, I = plan.forward_phasor(torch.from_numpy(Pin).to(device))
    V, I = V.cpu().numpy(), I.cpu().numpy()
    # planes at in-chunk positions 0..15 of the chunks of 16
    zi = sorted([0, 17, 34, 51, 68, 85, 102, 119, 8, 25, 42, 59, 76, 93, 110, 127])
    assert sorted(z % 16 for z in zi) == list(range(16))
    g = w.grid
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z[zi])
    Vref = o.nursd_grid(Pin[sel].astype(np.complex128), w.relay_xy.astype(np.float64), f[sel],
                        o.frame_for_workload(w), sub, w.xp)
    assert rel(V[zi], Vref) < TOL
    assert rel(I[zi], np.abs(Vref)) < TOL


def test_spad_forward_bitwise_reproducible(device, spad_hist):
    """The full SPAD forward from histograms, as the benchmark times it, gives
    the same volume bit for bit when repeated and when a second plan is built
    from the same inputs (fixed spreading order, no atomics)."""
    print("case: spad forward bitwise reproducible", flush=True)
    w = scenes.config_spad(render=False)
    H = torch.from_numpy(spad_hist).to(device)
    plan = plan_for(w, device)
    V1, I1 = plan.forward_hist(H)
    V2, I2 = plan.forward_hist(H)
    plan_b = plan_for(w, device)
    V3, I3 = plan_b.forward_hist(H)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(V1)).all()
    assert torch.equal(V1, V2) and torch.equal(I1, I2)
    assert torch.equal(V1, V3) and torch.equal(I1, I3)


def test_nursd3d_m512(device):
    """3D NURSD with the non-planar workload's frame (M = 512, depth grid of
    16 at 2 cm around z_mid = 6 cm): 2,048 of its relays on the curved wall,
    all 96 frequencies and 128 planes launched, 2 bins x 2 planes checked."""
    print("case: nursd3d M=512", flush=True)
    w = scenes.config_nonplanar()
    rng = np.random.default_rng(5)
    keep = np.sort(rng.choice(w.relay_xy.shape[0], 2048, replace=False))
    w.relay_xy = np.ascontiguousarray(w.relay_xy[keep])
    w.extra = dict(w.extra, relay_z=np.ascontiguousarray(w.extra["relay_z"][keep]), mz3=16)
    plan = plan_for(w, device)
    assert plan.info["M"] == 512 and plan.info["depth3d"] == 16
    F, L = w.wavelet.n_freq, w.relay_xy.shape[0]
    sel = [21, 66]
    Pin = np.zeros((F, L), np.complex64)
    Pin[sel] = (rng.normal(size=(2, L)) + 1j * rng.normal(size=(2, L))).astype(np.complex64)
    V, _ = plan.forward_phasor(torch.from_numpy(Pin).to(device), intensity=False)
    V = V.cpu().numpy()
    _, f = o.wavelet_bins(w.wavelet.lambda_c, w.wavelet.n_time, w.wavelet.dt, F)
    zi = [5, 90]
    g = w.grid
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z[zi])
    xyz = np.concatenate([w.relay_xy.astype(np.float64), w.extra["relay_z"].astype(np.float64)[:, None]], 1)
    ref = o.nursd3d_grid(Pin[sel].astype(np.complex128), xyz, f[sel], o.frame_for_workload(w), sub, w.xp,
                         w.extra["z_mid"], w.extra["dz3"], 16)
    assert rel(V[zi], ref) < TOL


def test_frustum_points_4_bins_64_planes(device, spad_hist):
    """The 1,048,576-voxel frustum (64 planes over [1, 4] m): 4 bins, every
    plane, 256 sampled voxels per plane."""
    print("case: frustum points, 4 bins x 64 planes x 256 voxels", flush=True)
    w = scenes.config_frustum_points(render=False)
    plan = plan_for(w, device)
    fr = o.frame_for_workload(w)
    assert plan.info["M"] == fr.M == 512
    sel = [3, 30, 61, 94]
    Pin, f = band_phasors(w, spad_hist, sel)
    V, _ = plan.forward_phasor(torch.from_numpy(Pin).to(device), intensity=False)
    V = V.cpu().numpy()
    rng = np.random.default_rng(1)
    idx = np.concatenate([np.sort(rng.choice(np.arange(w.plane_ptr[i], w.plane_ptr[i + 1]), 256, replace=False))
                          for i in range(len(w.grid.z))])
    ptr = np.arange(len(w.grid.z) + 1) * 256
    ref = o.nursd_points(Pin[sel].astype(np.complex128), w.relay_xy.astype(np.float64), f[sel], fr, w.grid.z, ptr,
                         w.voxel_xy[idx].astype(np.float64), w.xp)
    assert rel(V[idx], ref) < TOL


def test_srsd_4_bins_16_planes(device, spad_hist):
    """The scaled-RSD workload (256 x 256 samples on 128 planes over [1, 4] m):
    4 bins x 16 whole planes."""
    print("case: srsd full launch, 4 bins x 16 planes", flush=True)
    w = scenes.config_srsd(render=False)
    plan = plan_for(w, device)
    sel = [5, 38, 67, 92]
    Pin, f = band_phasors(w, spad_hist, sel)
    V, _ = plan.forward_phasor(torch.from_numpy(Pin).to(device), intensity=False)
    V = V.cpu().numpy()
    zc = plan.info["plane_chunk"]
    zi = sorted({(k * 8 + k % zc) % 128 for k in range(16)})
    assert len(zi) == 16
    g = w.grid
    sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z[zi])
    ref = o.srsd(Pin[sel].astype(np.complex128), w.relay_xy.astype(np.float64), f[sel], o.frame_for_workload(w), sub,
                 w.xp, o.srsd_alpha(sub.z, w.zref))
    assert rel(V[zi], ref) < TOL


@pytest.fixture(scope="module")
def batch64(device):
    """The 64-scene serving workload with tone histograms in 2 evenly spaced
    bins of each scene's band; plain loop and autotuned batch outputs."""
    from paper_2501_05244_amd.api import Batch, plan_from_workload
    print("case: batch 64 scenes (plain and batched)", flush=True)
    ws = scenes.config_batch(render=False)
    sels = []
    for s, w in enumerate(ws):
        F = w.wavelet.n_freq
        sel = [F // 4, (3 * F) // 4]
        bins = o.wavelet_bins(w.wavelet.lambda_c, w.wavelet.n_time, w.wavelet.dt, F)[0]
        w.hist = scenes.tone_histograms(w.relay_xy.shape[0], w.wavelet.n_time, bins[sel], seed=500 + s)
        sels.append(sel)
    plans = [plan_from_workload(w, device) for w in ws]
    hists = [torch.from_numpy(w.hist).to(device) for w in ws]
    plain = [p.forward_hist(h, vol=False)[1].cpu().numpy() for p, h in zip(plans, hists)]
    for p in plans:
        p._ws = None                      # release the plain loop's workspaces
    b = Batch(plans, autotune=True)
    outs = [x.cpu().numpy() for x in b.forward(hists)]
    print("  batch:", {k: v for k, v in b.info().items() if k != "tried"}, flush=True)
    return ws, sels, plain, outs


def test_batch_64_batched_equals_plain(batch64):
    _, _, plain, outs = batch64
    worst = max(rel(x, y) for x, y in zip(outs, plain))
    assert worst < 1e-5


@pytest.mark.parametrize("group", range(4))
def test_batch_64_every_scene_vs_oracle(batch64, group):
    ws, sels, _, outs = batch64
    for s in range(group * 16, group * 16 + 16):
        w, sel = ws[s], sels[s]
        wl = w.wavelet
        bins, f = o.wavelet_bins(wl.lambda_c, wl.n_time, wl.dt, wl.n_freq)
        wts = o.phasor_weights(f, wl.lambda_c, wl.sigma_rel, wl.t0)
        P = o.temporal_phasor(w.hist, bins[sel], wts[sel])
        g = w.grid
        zi = np.linspace(0, len(g.z) - 1, 4).round().astype(int)
        sub = scenes.Grid(g.x0, g.y0, g.dx, g.dy, g.nx, g.ny, g.z[zi])
        ref = o.nursd_grid(P, w.relay_xy.astype(np.float64), f[sel], o.frame_for_workload(w), sub, w.xp,
                           intensity=True)
        print(f"  scene {s}: M {o.frame_for_workload(w).M} L {w.relay_xy.shape[0]} F {wl.n_freq}", flush=True)
        assert rel(outs[s][zi], ref) < TOL
