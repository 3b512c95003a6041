"""GPU parity of the scaled RSD evaluated at per-plane voxel lists (the
fusion of eq. NURSD2_SRSD) against the FP64 oracle's direct scaled DFT and
direct NUDFT-2 in each plane's scaled frame.  Tolerance: relative L2 <= 1e-4."""
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


def case(n, seed, counts=(300, 0, 517), zs=(0.6, 0.9, 1.4), L=1500, F=2, zref=0.55):
    rng = np.random.default_rng(seed)
    dx = 0.0078125
    half = n * dx / 2
    g = scenes.Grid(x0=-half + dx / 2, y0=-half + dx / 2, dx=dx, dy=dx, nx=n, ny=n, z=np.array(zs))
    xy = rng.uniform(-0.95 * half, 0.95 * half, size=(L, 2)).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=4096, dt=4e-12, t0=0.0, n_freq=F, bins=np.array([70, 95])[:F])
    vox = []
    for zz, c in zip(zs, counts):
        a = zref / zz
        vox.append(rng.uniform(-1.1 * half / a, 1.1 * half / a, size=(c, 2)))   # a little past the window
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    w = scenes.Workload("srsd_points_small", xy, np.array([0.02, -0.01, 0.0]), wl, g, mode="srsd_points",
                        zref=zref, plane_ptr=ptr, voxel_xy=np.concatenate(vox).astype(np.float32))
    P = np.ascontiguousarray((rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64))
    return w, P


def oracle(w, P, f, z=None, ptr=None, vox=None):
    fr = o.frame_for_workload(w)
    z = w.grid.z if z is None else z
    return o.srsd_points(P.astype(np.complex128), w.relay_xy.astype(np.float64), f, fr, w.grid.nx, z,
                         o.srsd_alpha(z, w.zref), w.plane_ptr if ptr is None else ptr,
                         (w.voxel_xy if vox is None else vox).astype(np.float64), w.xp)


@pytest.mark.parametrize("n,chunks", [(256, (0, 0)), (200, (1, 2))])
def test_srsd_points_small(device, n, chunks):
    print("case: srsd points small", n, chunks, flush=True)
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = case(n, seed=n + 5)
    plan = plan_from_workload(w, device, freq_chunk=chunks[0], plane_chunk=chunks[1])
    assert plan.info["M"] == 512 and plan.info["n_voxels"] == w.plane_ptr[-1]
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    _, f = o.wavelet_bins(0.06, 4096, 4e-12, 2, w.wavelet.bins)
    ref = oracle(w, P, f)
    assert rel(V.cpu().numpy(), ref) < TOL
    assert rel(I.cpu().numpy(), np.abs(ref)) < TOL


def test_srsd_points_on_scaled_grid_match_srsd(device):
    """Voxel lists on each plane's scaled grid reproduce the uniform scaled
    RSD output there (both on the GPU)."""
    print("case: srsd points vs srsd grid", flush=True)
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = case(256, seed=3)
    ws = scenes.Workload("srsd", w.relay_xy, w.xp, w.wavelet, w.grid, mode="srsd", zref=w.zref)
    Pt = torch.from_numpy(P).to(device)
    Vg, _ = plan_from_workload(ws, device).forward_phasor(Pt, intensity=False)
    Vg = Vg.cpu().numpy()
    rng = np.random.default_rng(4)
    g = w.grid
    m = np.arange(g.nx) - g.nx // 2
    cx, cy = g.x0 + (g.nx // 2) * g.dx, g.y0 + (g.ny // 2) * g.dy
    vox, ref, ptr = [], [], [0]
    for iz, zz in enumerate(g.z):
        a = w.zref / zz
        pick = rng.choice(g.nx * g.ny, 400, replace=False)
        iy, ix = np.divmod(pick, g.nx)
        vox.append(np.stack([cx + m[ix] * g.dx / a, cy + m[iy] * g.dy / a], 1))
        ref.append(Vg[iz, iy, ix])
        ptr.append(ptr[-1] + len(pick))
    w.voxel_xy = np.concatenate(vox).astype(np.float32)
    w.plane_ptr = np.array(ptr, np.int32)
    V, _ = plan_from_workload(w, device).forward_phasor(Pt, intensity=False)
    assert rel(V.cpu().numpy(), np.concatenate(ref)) < TOL


@pytest.mark.slow
def test_srsd_points_frustum_full_launch_sampled(device):
    """The frustum workload (65,536 relays, 96 frequencies, 1,048,576 voxels on
    64 scaled planes over [1,4] m) at full size with phasors nonzero in two
    bins; the oracle evaluates 1,000 sampled voxels on each of three planes."""
    print("case: srsd points frustum full launch", flush=True)
    from paper_2501_05244_amd.api import plan_from_workload
    w = scenes.config_srsd_points()
    plan = plan_from_workload(w, device)
    assert plan.info["M"] == o.frame_for_workload(w).M == 512
    wl = w.wavelet
    bins, f = o.wavelet_bins(wl.lambda_c, wl.n_time, wl.dt, wl.n_freq)
    wts = o.phasor_weights(f, wl.lambda_c, wl.sigma_rel, wl.t0)
    sel = [30, 75]
    Pin = np.zeros((wl.n_freq, w.relay_xy.shape[0]), np.complex64)
    Pin[sel] = o.temporal_phasor(w.hist, bins[sel], wts[sel])
    V, _ = plan.forward_phasor(torch.from_numpy(Pin).to(device), intensity=False)
    V = V.cpu().numpy()
    rng = np.random.default_rng(0)
    for iz in (0, 31, 63):
        a, e = w.plane_ptr[iz], w.plane_ptr[iz + 1]
        idx = np.sort(rng.choice(np.arange(a, e), 1000, replace=False))
        ref = oracle(w, Pin[sel], f[sel], z=w.grid.z[[iz]], ptr=np.array([0, len(idx)]), vox=w.voxel_xy[idx])
        assert rel(V[idx], ref) < TOL
