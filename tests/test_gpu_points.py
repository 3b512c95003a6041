"""GPU parity of NURSD-3 (type-2 output at per-plane voxel lists) against the
FP64 oracle's direct NUDFT-1 / NUDFT-2.  Tolerance: relative L2 <= 1e-4."""
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


def points_case(seed=3, L=1500, counts=(700, 0, 1333, 90), F=2):
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-0.9, 0.9, size=(L, 2)).astype(np.float32)
    zs = np.array([0.5, 0.8, 1.1, 1.6])[: len(counts)]
    vox = [rng.uniform(-0.85, 0.85, size=(c, 2)) for c in counts]
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    voxel_xy = np.concatenate(vox).astype(np.float32)
    wl = scenes.Wavelet(lambda_c=0.06, n_time=4096, dt=4e-12, t0=0.0, n_freq=F, bins=np.array([64, 101])[:F])
    g = scenes.Grid(x0=0, y0=0, dx=0.0078125, dy=0.0078125, nx=0, ny=0, z=zs)
    w = scenes.Workload("points_small", xy, np.array([0.01, 0.02, 0.0]), wl, g, mode="points", plane_ptr=ptr,
                        voxel_xy=voxel_xy)
    P = np.ascontiguousarray((rng.normal(size=(F, L)) + 1j * rng.normal(size=(F, L))).astype(np.complex64))
    return w, P


@pytest.mark.parametrize("chunks", [(0, 0), (1, 1)])
def test_points_small(device, chunks):
    print("case: points small", chunks, flush=True)
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = points_case()
    plan = plan_from_workload(w, device, M=512, freq_chunk=chunks[0], plane_chunk=chunks[1])
    fr = o.choose_frame("points", w.relay_xy, dx=w.grid.dx, dy=w.grid.dy, voxel_xy=w.voxel_xy, sizes=(512,))
    assert abs(plan.info["cx"] - fr.cx) < 1e-9 and abs(plan.info["cy"] - fr.cy) < 1e-9
    V, I = plan.forward_phasor(torch.from_numpy(P).to(device))
    _, f = o.wavelet_bins(0.06, 4096, 4e-12, 2, w.wavelet.bins)
    ref = o.nursd_points(P.astype(np.complex128), w.relay_xy.astype(np.float64), f, fr, w.grid.z, w.plane_ptr,
                         w.voxel_xy.astype(np.float64), w.xp)
    assert rel(V.cpu().numpy(), ref) < TOL
    assert rel(I.cpu().numpy(), np.abs(ref)) < TOL


def test_points_rejects_small_transform(device):
    from paper_2501_05244_amd.api import plan_from_workload
    w, P = points_case()
    w.relay_xy = np.ascontiguousarray(w.relay_xy * 0.4)
    w.voxel_xy = np.ascontiguousarray(w.voxel_xy * 0.4)
    assert o.frame_for_workload(w).M == 256
    with pytest.raises(RuntimeError, match="UNSUPPORTED_SIZE"):
        plan_from_workload(w, device)
