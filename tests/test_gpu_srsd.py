"""GPU parity of the scaled RSD (chirp-z) path against the FP64 oracle's
direct scaled DFT.  Tolerance: relative L2 <= 1e-4 on the complex volume."""
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


def srsd_case(n, seed, L=1500, zs=(0.6, 0.9, 1.4), F=2):
    rng = np.random.default_rng(seed)
    dx = 0.0078125
    half = n * dx / 2
    g = scenes.Grid(x0=-half + dx / 2, y0=-half + dx / 2, dx=dx, dy=dx, nx=n, ny=n, z=np.array(zs))
    xy = rng.uniform(-0.95 * half, 0.95 * half, size=(L, 2)).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=4096, dt=4e-12, t0=0.0, n_freq=F,
                        bins=np.array([70, 95])[:F])
    w = scenes.Workload("srsd_small", xy, np.array([0.02, -0.01, 0.0]), wl, g, mode="srsd", zref=0.55)
    P = np.ascontiguousarray((rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64))
    return w, P


def oracle_srsd(w, P, f):
    fr = o.frame_for_workload(w)
    alphas = o.srsd_alpha(w.grid.z, w.zref)
    return o.srsd(P.astype(np.complex128), w.relay_xy.astype(np.float64), f, fr, w.grid, w.xp, alphas)


@pytest.mark.parametrize("n,chunks", [(256, (0, 0)), (200, (1, 2))])
def test_srsd_small(device, n, chunks):
    print("case: srsd small", n, chunks, flush=True)
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = srsd_case(n, seed=n)
    plan = plan_from_workload(w, device, freq_chunk=chunks[0], plane_chunk=chunks[1])
    assert plan.info["M"] == o.frame_for_workload(w).M == 512
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    _, f = o.wavelet_bins(0.06, 4096, 4e-12, 2, w.wavelet.bins)
    ref = oracle_srsd(w, P, f)
    assert rel(V.cpu().numpy(), ref) < TOL
    assert rel(I.cpu().numpy(), np.abs(ref)) < TOL


@pytest.mark.parametrize("n,L,zs", [(256, 1, (0.9,)), (255, 2, (0.6, 1.4))])
def test_srsd_few_relays(device, n, L, zs):
    """One or two relays, one or two planes, an odd window: the Bluestein
    lines are nearly empty and the window is not a multiple of the tiles."""
    print("case: srsd few relays", n, L, zs, flush=True)
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = srsd_case(n, seed=5, L=L, zs=zs)
    plan = plan_from_workload(w, device)
    assert plan.info["M"] == o.frame_for_workload(w).M == 512
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    _, f = o.wavelet_bins(0.06, 4096, 4e-12, 2, w.wavelet.bins)
    ref = oracle_srsd(w, P, f)
    assert rel(V.cpu().numpy(), ref) < TOL
    assert rel(I.cpu().numpy(), np.abs(ref)) < TOL


def test_srsd_rejects_bad_geometry(device):
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = srsd_case(256, seed=1)
    w.zref = 2.0          # alpha = zref / z > 1 on every plane
    with pytest.raises(RuntimeError, match="GEOMETRY"):
        plan_from_workload(w, device)
