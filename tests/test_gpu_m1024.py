"""GPU parity at transform size M = 1,024 (fine grid 2,048) for the uniform
grid, the scaled RSD, voxel lists and scaled voxel lists, against the FP64
oracle with the same frame.  Small relay and voxel counts keep the oracle's
direct sums to seconds; the kernels run their M = 1,024 instantiations."""
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


def wavelet(F=2):
    return scenes.Wavelet(lambda_c=0.06, n_time=4096, dt=4e-12, t0=0.0, n_freq=F, bins=np.array([70, 95])[:F])


def random_phasors(rng, F, L):
    return np.ascontiguousarray((rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64))


def plan_for(w, device, **kw):
    from paper_2501_05244_amd.api import plan_from_workload
    return plan_from_workload(w, device, **kw)


def freqs(w):
    _, f = o.wavelet_bins(0.06, 4096, 4e-12, w.wavelet.n_freq, w.wavelet.bins)
    return f


def test_grid_m1024(device):
    print("case: grid M=1024", flush=True)
    rng = np.random.default_rng(41)
    n, dx, L = 96, 0.0078125, 400
    half = n * dx / 2
    g = scenes.Grid(x0=-half + dx / 2, y0=-half + dx / 2, dx=dx, dy=dx, nx=n, ny=n, z=np.array([0.4, 0.9]))
    xy = rng.uniform(-0.9 * half, 0.9 * half, size=(L, 2)).astype(np.float32)
    w = scenes.Workload("grid1024", xy, np.array([0.03, 0.0, 0.0]), wavelet(), g)
    P = random_phasors(rng, 2, L)
    plan = plan_for(w, device, M=1024)
    assert plan.info["M"] == 1024
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    fr = o.choose_frame("grid", w.relay_xy, x0=g.x0, y0=g.y0, dx=dx, dy=dx, nx=n, ny=n, sizes=(1024,))
    ref = o.nursd_grid(P.astype(np.complex128), xy.astype(np.float64), freqs(w), fr, g, w.xp)
    assert rel(V.cpu().numpy(), ref) < TOL
    assert rel(I.cpu().numpy(), np.abs(ref)) < TOL


def test_srsd_m1024(device):
    print("case: srsd M=1024", flush=True)
    rng = np.random.default_rng(42)
    n, dx, L = 256, 0.0078125, 600
    half = n * dx / 2
    g = scenes.Grid(x0=-half + dx / 2, y0=-half + dx / 2, dx=dx, dy=dx, nx=n, ny=n, z=np.array([0.6, 1.3]))
    xy = rng.uniform(-0.95 * half, 0.95 * half, size=(L, 2)).astype(np.float32)
    w = scenes.Workload("srsd1024", xy, np.array([0.02, -0.01, 0.0]), wavelet(), g, mode="srsd", zref=0.55)
    P = random_phasors(rng, 2, L)
    plan = plan_for(w, device, M=1024)
    assert plan.info["M"] == 1024
    V, _ = plan.forward_phasor(torch.from_numpy(P).to(device), intensity=False)
    fr = o.choose_frame("srsd", w.relay_xy, x0=g.x0, y0=g.y0, dx=dx, dy=dx, nx=n, ny=n, sizes=(1024,))
    ref = o.srsd(P.astype(np.complex128), xy.astype(np.float64), freqs(w), fr, g, w.xp,
                 o.srsd_alpha(g.z, w.zref))
    assert rel(V.cpu().numpy(), ref) < TOL


def test_points_m1024(device):
    print("case: points M=1024", flush=True)
    rng = np.random.default_rng(43)
    L, counts = 500, (600, 0, 900)
    xy = rng.uniform(-0.9, 0.9, size=(L, 2)).astype(np.float32)
    zs = np.array([0.5, 0.8, 1.2])
    vox = np.concatenate([rng.uniform(-0.85, 0.85, size=(c, 2)) for c in counts]).astype(np.float32)
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    g = scenes.Grid(x0=0, y0=0, dx=0.0078125, dy=0.0078125, nx=0, ny=0, z=zs)
    w = scenes.Workload("points1024", xy, np.array([0.01, 0.02, 0.0]), wavelet(), g, mode="points", plane_ptr=ptr,
                        voxel_xy=vox)
    P = random_phasors(rng, 2, L)
    plan = plan_for(w, device, M=1024)
    assert plan.info["M"] == 1024
    V, _ = plan.forward_phasor(torch.from_numpy(P).to(device), intensity=False)
    fr = o.choose_frame("points", xy, dx=g.dx, dy=g.dy, voxel_xy=vox, sizes=(1024,))
    ref = o.nursd_points(P.astype(np.complex128), xy.astype(np.float64), freqs(w), fr, zs, ptr,
                         vox.astype(np.float64), w.xp)
    assert rel(V.cpu().numpy(), ref) < TOL


def test_srsd_points_m1024(device):
    print("case: srsd points M=1024", flush=True)
    rng = np.random.default_rng(44)
    n, dx, L, zref = 256, 0.0078125, 600, 0.55
    half = n * dx / 2
    zs = np.array([0.6, 1.4])
    g = scenes.Grid(x0=-half + dx / 2, y0=-half + dx / 2, dx=dx, dy=dx, nx=n, ny=n, z=zs)
    xy = rng.uniform(-0.95 * half, 0.95 * half, size=(L, 2)).astype(np.float32)
    vox = [rng.uniform(-1.05 * half * zz / zref, 1.05 * half * zz / zref, size=(c, 2)) for zz, c in zip(zs, (500, 700))]
    ptr = np.array([0, 500, 1200], np.int32)
    vox = np.concatenate(vox).astype(np.float32)
    w = scenes.Workload("srsd_points1024", xy, np.array([0.02, -0.01, 0.0]), wavelet(), g, mode="srsd_points",
                        zref=zref, plane_ptr=ptr, voxel_xy=vox)
    P = random_phasors(rng, 2, L)
    plan = plan_for(w, device, M=1024)
    assert plan.info["M"] == 1024
    V, _ = plan.forward_phasor(torch.from_numpy(P).to(device), intensity=False)
    fr = o.choose_frame("srsd", xy, x0=g.x0, y0=g.y0, dx=dx, dy=dx, nx=n, ny=n, sizes=(1024,))
    ref = o.srsd_points(P.astype(np.complex128), xy.astype(np.float64), freqs(w), fr, n, zs,
                        o.srsd_alpha(zs, zref), ptr, vox.astype(np.float64), w.xp)
    assert rel(V.cpu().numpy(), ref) < TOL
